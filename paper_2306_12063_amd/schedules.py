"""Decoder schedules and arithmetics side by side on one code: layered
versus flooding (Sec. 4: layering reduces the iterations needed), and FP32
NMS versus the fixed-point forms (int8 OMS; the paper's int16 Q_B = 10 with
wrap-around or saturation, Sec. 5). For each Eb/N0 point the same seeded
frames go through every selected decoder with early termination; reported
per decoder: FER (information bits), mean iterations, and the Eb/N0 at
FER = 1e-3. Throughput is timed at a fixed number of iterations with early
termination off.

    python -m paper_2306_12063_amd.schedules --code wifi:1/2:81
    python -m paper_2306_12063_amd.schedules --decoders layered_f32,q16_wrap,q16_sat
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from . import (ldpc_code_info, ldpc_decode_f32, ldpc_decode_flood_f32, ldpc_decode_flood_i8, ldpc_decode_i8,
               ldpc_decode_q16, ldpc_frame_stats, ldpc_quantize_i8, ldpc_quantize_q16)
from .learned import _code, ebn0_at_fer, make_frames


def _decoders(hbm, Z, T):
    # each decoder takes (FP32 LLRs, int8 LLRs, int16 Q_B = 10 LLRs, early termination)
    return {
        "q16_wrap": lambda l, q, q16, et: ldpc_decode_q16(hbm, Z, q16, max_iter=T, wq=12, wrap=True, early_term=et,
                                                          want_post=False),
        "q16_sat": lambda l, q, q16, et: ldpc_decode_q16(hbm, Z, q16, max_iter=T, wq=12, wrap=False, early_term=et,
                                                         want_post=False),
        **{n: (lambda f: (lambda l, q, q16, et: f(l, q, et)))(f) for n, f in _schedule_decoders(hbm, Z, T).items()},
    }


def _schedule_decoders(hbm, Z, T):
    return {
        "layered_f32": lambda l, q, et: ldpc_decode_f32(hbm, Z, l, max_iter=T, alpha=0.75, early_term=et,
                                                        want_post=False),
        "flooding_f32": lambda l, q, et: ldpc_decode_flood_f32(hbm, Z, l, max_iter=T, alpha=0.75, early_term=et,
                                                               want_post=False),
        "layered_i8": lambda l, q, et: ldpc_decode_i8(hbm, Z, q, max_iter=T, offset=1, early_term=et,
                                                      want_post=False),
        "flooding_i8": lambda l, q, et: ldpc_decode_flood_i8(hbm, Z, q, max_iter=T, offset=1, early_term=et,
                                                             want_post=False),
    }


def compare(hbm, Z, ebn0_list, frames, T=10, chunk=1 << 17, seed=5, device="cuda", names=None):
    K = ldpc_code_info(hbm, Z)["K"]
    decs = _decoders(hbm, Z, T)
    if names:
        decs = {n: decs[n] for n in names}
    sweep = {n: [] for n in decs}
    for pi, eb in enumerate(ebn0_list):
        cnt = {n: torch.zeros(4, dtype=torch.int64, device=device) for n in decs}
        done, ci = 0, 0
        while done < frames:
            F = min(chunk, frames - done)
            bits_in, _, llr = make_frames(hbm, Z, F, eb, seed * 7919 + pi * 104729 + ci, device)
            q = ldpc_quantize_i8(llr)
            q16 = ldpc_quantize_q16(llr)
            for n, d in decs.items():
                bits, _, iters, ok = d(llr, q, q16, True)
                ldpc_frame_stats(bits, bits_in, iters, ok, counters=cnt[n])
            done += F
            ci += 1
        for n in decs:
            c = cnt[n].cpu().numpy()
            sweep[n].append(dict(ebn0=float(eb), fer=c[1] / frames, ber=c[0] / (frames * K),
                                 mean_iters=c[2] / frames))
    # throughput at T fixed iterations
    F = 1 << 16
    _, _, llr = make_frames(hbm, Z, F, ebn0_list[len(ebn0_list) // 2], seed, device)
    q = ldpc_quantize_i8(llr)
    q16 = ldpc_quantize_q16(llr)
    speed = {}
    for n, d in decs.items():
        d(llr, q, q16, False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            d(llr, q, q16, False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        speed[n] = dict(ms=ms, gbit_s=F * K / (ms / 1e3) / 1e9)
    summary = {}
    for n, pts in sweep.items():
        e = ebn0_at_fer(pts)
        summary[n] = dict(ebn0_at_fer_1e3=e, gbit_s_fixed_iters=speed[n]["gbit_s"])
    for path in ("f32", "i8"):
        if f"layered_{path}" not in sweep or f"flooding_{path}" not in sweep:
            continue
        lay, fl = sweep[f"layered_{path}"], sweep[f"flooding_{path}"]
        e = summary[f"layered_{path}"]["ebn0_at_fer_1e3"]
        if e is not None:
            p = min(range(len(lay)), key=lambda k: abs(lay[k]["ebn0"] - e))
            summary[f"iterations_at_layered_1e3_{path}"] = dict(
                ebn0=lay[p]["ebn0"], layered=lay[p]["mean_iters"], flooding=fl[p]["mean_iters"])
    return dict(summary=summary, sweep=sweep, max_iter=T, frames=frames)


def main():
    ap = argparse.ArgumentParser(description="layered vs flooding min-sum on one GPU")
    ap.add_argument("--code", default="wifi:1/2:81", help="wifi:<rate>:<Z> or wimax:<class>:<Z>")
    ap.add_argument("--frames", type=int, default=1 << 19)
    ap.add_argument("--ebn0", default="1:4:0.25", help="start:stop:step in dB")
    ap.add_argument("--max-iter", type=int, default=10)
    ap.add_argument("--decoders", default="layered_f32,flooding_f32,layered_i8,flooding_i8",
                    help="comma-separated: layered_f32 flooding_f32 layered_i8 flooding_i8 q16_wrap q16_sat")
    args = ap.parse_args()
    a, b, s = (float(x) for x in args.ebn0.split(":"))
    pts = list(np.round(np.arange(a, b + 1e-9, s), 4))
    hbm, Z = _code(args.code)
    r = compare(hbm, Z, pts, args.frames, T=args.max_iter, names=args.decoders.split(","))
    r["code"] = args.code
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
