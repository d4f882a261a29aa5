"""Training and evaluation of the learned normalised min-sum decoder.

Every per-frame step runs in the library's kernels: Philox frame generation,
direct encoding, BPSK/AWGN, the learned forward and its adjoint, decoding,
fallback re-decoding and error counting. PyTorch provides device memory,
the stream and the Adam optimiser; numpy draws the per-frame Eb/N0 values.

    python -m paper_2306_12063_amd.learned --code wifi:5/6:81 --frames 262144
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

import synth
from . import (ldpc_code_info, ldpc_decode_f32, ldpc_decode_i8, ldpc_decode_layouts, ldpc_encode, ldpc_fallback_f32,
               ldpc_fallback_i8, ldpc_frame_stats, ldpc_quantize_i8, ldpc_random_bits, ldpc_set_decode_layout,
               ldpc_awgn_llr)
from .nms import nms_loss, quantize_weights


def awgn_params(ebn0_db, rate):
    """Per-frame noise deviation and LLR scale (FP32) for Eb/N0 values in dB."""
    s2 = synth.sigma2_from_ebn0(np.asarray(ebn0_db, dtype=np.float64), rate)
    return np.sqrt(s2).astype(np.float32), (2.0 / s2).astype(np.float32)


def make_frames(hbm, Z, F, ebn0_db, seed, device="cuda", sigma_scale=None):
    """(info, codewords, channel LLRs) of F seeded frames; ebn0_db is a
    number or an array of per-frame values (dB), or sigma_scale gives the
    per-frame (sigma, scale) as device tensors."""
    info = ldpc_code_info(hbm, Z)
    N, K = info["N"], info["K"]
    rate = K / N
    bits = ldpc_random_bits(seed, F, K, device=device)
    cw = ldpc_encode(hbm, Z, bits)
    if sigma_scale is not None:
        llr = ldpc_awgn_llr(seed ^ 0x5DEECE66D, cw, sigma_scale[0], sigma_scale[1])
    elif np.isscalar(ebn0_db):
        s2 = synth.sigma2_from_ebn0(float(ebn0_db), rate)
        llr = ldpc_awgn_llr(seed ^ 0x5DEECE66D, cw, math.sqrt(s2), 2.0 / s2)
    else:
        sg, sc = awgn_params(ebn0_db, rate)
        llr = ldpc_awgn_llr(seed ^ 0x5DEECE66D, cw, torch.from_numpy(sg).to(device), torch.from_numpy(sc).to(device))
    return bits, cw, llr


def iteration_weights(kind, T, device="cuda"):
    """Weights of the per-iteration losses in the training objective:
    'uniform' (the mean over iterations), 'ramp' (proportional to t + 1),
    'early' (proportional to T - t: early convergence weighs most) or
    'last' (the last iteration only); each sums to one."""
    if kind == "uniform":
        g = torch.ones(T)
    elif kind == "ramp":
        g = torch.arange(1, T + 1, dtype=torch.float32)
    elif kind == "early":
        g = torch.arange(T, 0, -1, dtype=torch.float32)
    elif kind == "last":
        g = torch.zeros(T)
        g[-1] = 1.0
    else:
        raise ValueError(kind)
    return (g * (T / g.sum())).to(device)


def train(hbm, Z, T=10, frames=1 << 20, batch=4096, lr=1e-2, ebn0_range=(1.0, 4.0), seed=1, w0=0.75,
          device="cuda", log_every=0, lr_final=None, tie="none", iter_loss="uniform"):
    """Trains w [T][Mb][Nb] with Adam on fresh frames (Eb/N0 uniform per frame)
    through the kernels' forward and adjoint. lr_final: if given, the step
    size follows a cosine from lr down to lr_final. tie='layer' shares one
    weight per (iteration, block row). iter_loss weights the per-iteration
    losses (iteration_weights). Returns (w, loss history)."""
    Mb, Nb = np.asarray(hbm).shape
    shape = (T, Mb, 1) if tie == "layer" else (T, Mb, Nb)
    p = torch.full(shape, w0, dtype=torch.float32, device=device, requires_grad=True)
    gam = iteration_weights(iter_loss, T, device)
    opt = torch.optim.Adam([p], lr=lr)
    rng = np.random.default_rng(seed)
    history = []
    steps = max(1, frames // batch)
    # every step's per-frame Eb/N0 drawn at once (the same sequence as one
    # draw per step) and copied to the device in one transfer: a per-step
    # copy from pageable memory would make the host wait for the GPU
    info = ldpc_code_info(hbm, Z)
    sg, sc = awgn_params(rng.uniform(ebn0_range[0], ebn0_range[1], (steps, batch)), info["K"] / info["N"])
    sg, sc = torch.from_numpy(sg).to(device), torch.from_numpy(sc).to(device)
    for step in range(steps):
        if lr_final is not None:
            for gr in opt.param_groups:
                gr["lr"] = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * step / steps))
        _, cw, llr = make_frames(hbm, Z, batch, None, seed * 1000003 + step, device, sigma_scale=(sg[step], sc[step]))
        opt.zero_grad(set_to_none=True)
        w = p.expand(T, Mb, Nb)
        per_iter = nms_loss(w, llr, cw, hbm, Z)
        (per_iter * gam).sum().backward()
        opt.step()
        # kept on the device: reading it back every step would make the host
        # wait for the GPU before it can queue the next step
        history.append(per_iter.detach().sum())
        if log_every and (step % log_every == 0 or step == steps - 1):
            print(f"  step {step:4d}/{steps}  loss {float(history[-1]):.5f}", flush=True)
    history = [float(x) for x in torch.stack(history).cpu()]
    return p.detach().expand(T, Mb, Nb).contiguous(), history


class _Dec:
    """One decoder form of the comparison: run(llr, q, bits, iters, ok)
    decodes into the given buffers, fallback(...) re-decodes failed frames;
    path names its kernel's decode layouts ("f32", "f32w", "i8w")."""

    def __init__(self, name, run, fallback, path):
        self.name, self.run, self.fallback, self.path = name, run, fallback, path


def decoders(hbm, Z, w, T=10):
    """Plain NMS (alpha = 0.75), learned FP32 and learned int8 (1/16 steps);
    each falls back to plain min-sum with 20 iterations for failed frames."""
    wq = quantize_weights(w)

    def plain(llr, q, bits, iters, ok):
        ldpc_decode_f32(hbm, Z, llr, max_iter=T, alpha=0.75, early_term=True, bits=bits, iters=iters, ok=ok,
                        want_post=False)

    def learned(llr, q, bits, iters, ok):
        ldpc_decode_f32(hbm, Z, llr, max_iter=T, w=w, early_term=True, bits=bits, iters=iters, ok=ok,
                        want_post=False)

    def learned8(llr, q, bits, iters, ok):
        ldpc_decode_i8(hbm, Z, q, max_iter=T, wq_table=wq, early_term=True, bits=bits, iters=iters, ok=ok,
                       want_post=False)

    def fb32(llr, q, bits, iters, ok, work):
        ldpc_fallback_f32(hbm, Z, llr, bits, iters, ok, max_iter=20, alpha=0.75, work=work)

    def fb8(llr, q, bits, iters, ok, work):
        ldpc_fallback_i8(hbm, Z, q, bits, iters, ok, max_iter=20, wq=12, work=work)

    return [_Dec("plain_nms_f32", plain, fb32, "f32"), _Dec("learned_f32", learned, fb32, "f32w"),
            _Dec("learned_i8", learned8, fb8, "i8w")]


def tune_on_frames(hbm, Z, decs, ebn0, F=1 << 17, seed=12345, reps=2):
    """Keeps, for each decoder form, the decode layout (among those the
    library's tuner would time) that decodes F frames at `ebn0` fastest with
    early termination, i.e. on the sweep's own workload rather than at fixed
    iterations; returns {form: layout}."""
    _, _, llr = make_frames(hbm, Z, F, ebn0, seed)
    q = ldpc_quantize_i8(llr)
    N, K = llr.shape[1], ldpc_code_info(hbm, Z)["K"]
    bits = torch.empty((F, N), dtype=torch.uint8, device=llr.device)
    iters = torch.empty(F, dtype=torch.int32, device=llr.device)
    ok = torch.empty(F, dtype=torch.uint8, device=llr.device)
    chosen = {}
    for d in decs:
        best = None
        for lay in ldpc_decode_layouts(hbm, Z, d.path):
            ldpc_set_decode_layout(hbm, Z, d.path, lay)
            d.run(llr, q, bits, iters, ok)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                d.run(llr, q, bits, iters, ok)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            if best is None or ms < best[0]:
                best = (ms, lay)
        ldpc_set_decode_layout(hbm, Z, d.path, best[1])
        chosen[d.name] = dict(best[1], ms=round(best[0], 4))
    return chosen


class SweepPipeline:
    """One Monte-Carlo sweep chunk on fixed device buffers: seeded random
    bits -> direct encoding -> BPSK/AWGN channel values -> int8 quantisation
    (the frame stage), then per decoder form: decode (the decode stage),
    first-pass counters, fallback re-decoding, final counters (the post
    stage). The seeds (device int64 [2]: bits, noise) and the per-frame
    noise deviation and LLR scale (device f32 [F]) are read by the kernels,
    so the stages can be captured once in HIP graphs and replayed for every
    chunk and Eb/N0 point after those buffers are refilled."""

    def __init__(self, hbm, Z, decs, F, device="cuda"):
        info = ldpc_code_info(hbm, Z)
        self.hbm, self.Z, self.decs, self.F = hbm, Z, decs, F
        self.N, self.K = info["N"], info["K"]
        dev = device
        self.seeds = torch.zeros(2, dtype=torch.int64, device=dev)
        self.sigma = torch.zeros(F, dtype=torch.float32, device=dev)
        self.scale = torch.zeros(F, dtype=torch.float32, device=dev)
        self.info = torch.empty((F, self.K), dtype=torch.uint8, device=dev)
        self.cw = torch.empty((F, self.N), dtype=torch.uint8, device=dev)
        self.llr = torch.empty((F, self.N), dtype=torch.float32, device=dev)
        self.q = torch.empty((F, self.N), dtype=torch.int8, device=dev)
        self.out = {d.name: dict(bits=torch.empty((F, self.N), dtype=torch.uint8, device=dev),
                                 iters=torch.empty(F, dtype=torch.int32, device=dev),
                                 ok=torch.empty(F, dtype=torch.uint8, device=dev),
                                 work=torch.empty(F + 1, dtype=torch.int64, device=dev),
                                 first=torch.zeros(4, dtype=torch.int64, device=dev),
                                 final=torch.zeros(4, dtype=torch.int64, device=dev)) for d in decs}
        self.graphs = None

    def frame_stage(self):
        ldpc_random_bits(self.seeds[0:1], self.F, self.K, out=self.info)
        ldpc_encode(self.hbm, self.Z, self.info, cw=self.cw)
        ldpc_awgn_llr(self.seeds[1:2], self.cw, self.sigma, self.scale, out=self.llr)
        ldpc_quantize_i8(self.llr, out=self.q)

    def decode_stage(self, d):
        o = self.out[d.name]
        d.run(self.llr, self.q, o["bits"], o["iters"], o["ok"])

    def post_stage(self, d):
        o = self.out[d.name]
        ldpc_frame_stats(o["bits"], self.info, o["iters"], o["ok"], counters=o["first"])
        d.fallback(self.llr, self.q, o["bits"], o["iters"], o["ok"], o["work"])
        ldpc_frame_stats(o["bits"], self.info, o["iters"], o["ok"], counters=o["final"])

    def set_point(self, ebn0_db, seed):
        """Refills the seed and noise buffers (fill kernels, no host wait)."""
        s2 = synth.sigma2_from_ebn0(float(ebn0_db), self.K / self.N)
        self.sigma.fill_(math.sqrt(s2))
        self.scale.fill_(2.0 / s2)
        self.seeds[0].fill_(seed)
        self.seeds[1].fill_(seed ^ 0x5DEECE66D)

    def clear_counters(self):
        for o in self.out.values():
            o["first"].zero_()
            o["final"].zero_()

    def capture(self):
        """Captures the frame stage and each decoder's decode and post stages
        in HIP graphs (after one eager pass that loads every kernel)."""
        self.frame_stage()
        for d in self.decs:
            self.decode_stage(d)
            self.post_stage(d)
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        graphs = {}
        with torch.cuda.stream(side):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                self.frame_stage()
            graphs["frames"] = g
            for d in self.decs:
                gd, gp = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
                with torch.cuda.graph(gd, stream=side):
                    self.decode_stage(d)
                with torch.cuda.graph(gp, stream=side):
                    self.post_stage(d)
                graphs[d.name] = (gd, gp)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graphs = graphs

    def run_chunk(self, ms):
        """One chunk at the current point; adds each decoder's decode time
        (ms, events around the decode stage) to ms[name]."""
        if self.graphs is not None:
            self.graphs["frames"].replay()
        else:
            self.frame_stage()
        for d in self.decs:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            if self.graphs is not None:
                self.graphs[d.name][0].replay()
            else:
                self.decode_stage(d)
            e1.record()
            if self.graphs is not None:
                self.graphs[d.name][1].replay()
            else:
                self.post_stage(d)
            ms.append((d.name, e0, e1))


def chunk_seed(seed, point, chunk):
    return seed * 7919 + point * 104729 + chunk


def sweep(hbm, Z, decs, ebn0_list, frames, chunk=1 << 17, seed=7, device="cuda", T=10, graph=True):
    """FER/BER/iterations per decoder and Eb/N0 point, first pass and after
    fallback, and decode throughput (info bits per second of decode time).
    Every chunk holds min(chunk, frames) frames (frames must be a multiple);
    with graph=True each chunk replays the pipeline's captured HIP graphs,
    otherwise it calls the same stages eagerly (identical results)."""
    F = min(chunk, frames)
    if frames % F:
        raise ValueError(f"frames ({frames}) must be a multiple of the chunk ({F})")
    pipe = SweepPipeline(hbm, Z, decs, F, device)
    if graph:
        pipe.set_point(ebn0_list[0], chunk_seed(seed, 0, 0))
        pipe.capture()
    K = pipe.K
    out = {d.name: [] for d in decs}
    for pi, eb in enumerate(ebn0_list):
        pipe.clear_counters()
        ev = []
        for ci in range(frames // F):
            pipe.set_point(eb, chunk_seed(seed, pi, ci))
            pipe.run_chunk(ev)
        torch.cuda.synchronize()
        ms = {d.name: 0.0 for d in decs}
        for name, e0, e1 in ev:
            ms[name] += e0.elapsed_time(e1)
        for d in decs:
            a, b = (pipe.out[d.name][k].cpu().numpy() for k in ("first", "final"))
            out[d.name].append(dict(
                ebn0=float(eb), frames=int(frames), fer=a[1] / frames, ber=a[0] / (frames * K),
                mean_iters=a[2] / frames, failed_syndrome=int(a[3]),
                # a frame that failed ran T first-pass iterations, then the fallback's
                fer_fallback=b[1] / frames, mean_iters_total=(b[2] + T * a[3]) / frames,
                gbit_s=frames * K / (ms[d.name] / 1e3) / 1e9,
                counters_first=[int(x) for x in a], counters_final=[int(x) for x in b]))
    return out


def ebn0_at_fer(points, key="fer", target=1e-3):
    """Eb/N0 where the FER crosses `target`, interpolated linearly in
    log10(FER) between the bracketing sweep points (None if not crossed)."""
    for a, b in zip(points, points[1:]):
        fa, fb = a[key], b[key]
        if fa >= target > fb:
            if fb <= 0:
                return b["ebn0"]
            la, lb, lt = math.log10(fa), math.log10(fb), math.log10(target)
            return a["ebn0"] + (b["ebn0"] - a["ebn0"]) * (la - lt) / (la - lb)
    return None


def iters_at(points, ebn0):
    """Mean first-pass iterations at the sweep point nearest ebn0."""
    p = min(points, key=lambda x: abs(x["ebn0"] - ebn0))
    return p["mean_iters"]


def compare(hbm, Z, train_frames=1 << 20, eval_frames=1 << 18, ebn0_list=None, seed=1, log_every=0,
            train_range=(1.0, 4.0), lr=1e-2, lr_final=None, tie="none", iter_loss="uniform", tune=True):
    """Trains a weight set for one code and compares the three decoder forms
    (with tune, each on the decode layout fastest on the sweep's workload)."""
    if ebn0_list is None:
        ebn0_list = [1.0 + 0.25 * k for k in range(21)]
    t0 = time.perf_counter()
    w, hist = train(hbm, Z, frames=train_frames, seed=seed, log_every=log_every, ebn0_range=train_range, lr=lr,
                    lr_final=lr_final, tie=tie, iter_loss=iter_loss)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    decs = decoders(hbm, Z, w)
    layouts = tune_on_frames(hbm, Z, decs, ebn0_list[len(ebn0_list) // 2]) if tune else None
    res = sweep(hbm, Z, decs, ebn0_list, eval_frames, seed=seed + 1)
    summary = {}
    e_plain = ebn0_at_fer(res["plain_nms_f32"])
    for name, pts in res.items():
        e = ebn0_at_fer(pts)
        summary[name] = dict(ebn0_at_fer_1e3=e, gain_db=(None if e is None or e_plain is None else e_plain - e),
                             mean_iters_at_plain_point=(iters_at(pts, e_plain) if e_plain is not None else None),
                             gbit_s=float(np.mean([p["gbit_s"] for p in pts])))
    if e_plain is not None:
        base = summary["plain_nms_f32"]["mean_iters_at_plain_point"]
        for name in summary:
            it = summary[name]["mean_iters_at_plain_point"]
            summary[name]["iter_reduction"] = (None if it is None or base == 0 else 1.0 - it / base)
    return dict(train_seconds=t_train, loss_first=hist[0], loss_last=float(np.mean(hist[-16:])),
                train_range=list(train_range), lr=lr, lr_final=lr_final, tie=tie, iter_loss=iter_loss,
                summary=summary, sweep=res, layouts=layouts,
                weights=w.cpu().numpy().round(5).tolist(), w=w)


def _code(spec):
    kind, rate, Z = spec.split(":")
    Z = int(Z)
    return (synth.wifi_code(rate, Z) if kind == "wifi" else synth.wimax_code(rate, Z)), Z


def main():
    ap = argparse.ArgumentParser(description="learned vs plain normalised min-sum on one GPU")
    ap.add_argument("--code", default="wifi:5/6:81", help="wifi:<rate>:<Z> or wimax:<class>:<Z>")
    ap.add_argument("--train-frames", type=int, default=1 << 20)
    ap.add_argument("--eval-frames", type=int, default=1 << 18)
    ap.add_argument("--ebn0", default="1:6:0.25", help="start:stop:step in dB")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--train-ebn0", default="1:4", help="lo:hi, per-frame uniform training Eb/N0 in dB")
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--lr-final", type=float, default=None, help="cosine decay of the step size to this value")
    ap.add_argument("--tie", choices=["none", "layer"], default="none",
                    help="layer: one weight per (iteration, block row)")
    ap.add_argument("--iter-loss", choices=["uniform", "ramp", "early", "last"], default="uniform",
                    help="weights of the per-iteration losses in the objective")
    args = ap.parse_args()
    a, b, s = (float(x) for x in args.ebn0.split(":"))
    pts = list(np.round(np.arange(a, b + 1e-9, s), 4))
    lo, hi = (float(x) for x in args.train_ebn0.split(":"))
    hbm, Z = _code(args.code)
    r = compare(hbm, Z, args.train_frames, args.eval_frames, pts, args.seed, log_every=64, train_range=(lo, hi),
                lr=args.lr, lr_final=args.lr_final, tie=args.tie, iter_loss=args.iter_loss)
    r["code"] = args.code
    r.pop("w")
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
