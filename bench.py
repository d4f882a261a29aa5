#!/usr/bin/env python3
"""Decoder throughput benchmark on one MI355X.

Workload: the Wi-Fi-shaped Z = 81 (N = 1944) codes at all four rates
(1/2, 2/3, 3/4, 5/6), 2^16 frames per launch, BPSK/AWGN frames at
Eb/N0 = 2 dB generated and encoded on the GPU before timing. One step decodes
every rate's batch twice -- FP32 normalised min-sum (alpha = 0.75) and the
saturating int8/int16 offset min-sum (offset 1) -- at a fixed 10 iterations
with early termination off, as the paper times its decoders. The reported
value is decoded information bits per second over the whole step.

Prints one JSON line. `--gpus` above 1 is refused: the benchmark runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "decoded info Gbit/s at 10 iters (FP32, int8); learned vs plain NMS FER=1e-3 Eb/N0"
Z = 81
ITERS = 10
EBN0_DB = 2.0
ALPHA = 0.75
OFFSET = 1
SEED = 2024
# VALU co-bound. Per edge and iteration the single-scan layered update needs:
# rebuild the old message (magnitude select, sign), Q = L - R_old, the running
# (min1, min2, argmin) update (three ops), the sign bit, the new message
# (magnitude select, sign) and L = Q + R: 10 operations per frame.
ALG_OPS_PER_EDGE_ITER = 10
# 32-bit VALU issue of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane
# operations per second; a packed 16-bit instruction does two frames' work,
# so the two-frames-per-lane fixed-point kernels are priced at twice that.
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
# LDS read peak: 256 CUs x 256 B/clk x 2.4 GHz. gfx950 reads twice CDNA3's
# 128 B/clk per CU: the LDS probe (ldpc_lds_probe) measures 144 TB/s, 92%
# of this figure and above the 128 B/clk one.
PEAK_LDS_GBS = 256 * 256 * 2.4e9 / 1e9


def lds_model_bytes(path, E, M, iters):
    """Algorithmic LDS bytes per frame of the layered single-scan method
    (Sec. 4) with the posteriors and the compressed row state on chip: each
    edge's posterior read and written once per iteration (4 B FP32, 2 B
    int16) and each row's compressed state (min1, min2, argmin, sign word)
    read and written once per iteration (16 B FP32, 8 B int8). The kernels
    here keep the row state in registers, so they move less than this."""
    bl, brow = (4, 16) if path == "f32" else (2, 8)
    return iters * (2 * bl * E + 2 * brow * M)


def hbm_model_bytes(path, N):
    """Algorithmic HBM bytes per frame: channel values in (4 B FP32, 1 B
    int8), hard bits (1 B each), the iteration count (4 B) and ok (1 B) out;
    posteriors are not written in the timed launches."""
    return N * (4 if path == "f32" else 1) + N + 4 + 1


def roofline_entry(lds_b, hbm_b, ops, ms, packed16, name):
    """Roofline of one kernel launch from its algorithmic bytes and
    operations and its average duration: the bound is the larger of the LDS
    and HBM fractions; VALU issue is reported beside it."""
    s = ms / 1e3
    lds_gbs, hbm_gbs = lds_b / s / 1e9, hbm_b / s / 1e9
    lds_f, hbm_f = lds_gbs / PEAK_LDS_GBS, hbm_gbs / PEAK_HBM_GBS
    vpeak = PEAK_VALU_TOPS * (2 if packed16 else 1)
    vt = ops / s / 1e12
    bound = "lds" if lds_f >= hbm_f else "hbm"
    return {"bound": bound, "achieved": round(lds_gbs if bound == "lds" else hbm_gbs, 1),
            "peak": round(PEAK_LDS_GBS if bound == "lds" else PEAK_HBM_GBS, 1), "unit": "GB/s",
            "frac": round(max(lds_f, hbm_f), 4), "kernel": name, "avg_ms": round(ms, 4),
            "alg_lds_bytes_per_launch": int(lds_b), "alg_hbm_bytes_per_launch": int(hbm_b),
            "lds_frac": round(lds_f, 4), "hbm_frac": round(hbm_f, 5),
            "valu": {"achieved": round(vt, 3), "peak": round(vpeak, 1), "unit": "T lane-ops/s",
                     "frac": round(vt / vpeak, 4), "alg_ops_per_launch": int(ops),
                     "ops_per_edge_iteration": ALG_OPS_PER_EDGE_ITER}}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=1 << 16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="use the default decode layout")
    ap.add_argument("--no-mixed-batch", action="store_true",
                    help="skip the secondary mixed-code batch measurement (114 codes, one persistent launch)")
    ap.add_argument("--batch-frames", type=int, default=1 << 18)
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the graph-replay timing of the mixed-code batch")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the Eb/N0 sweep with early termination and the small-code record")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-versus-plain Eb/N0 comparison (secondary record)")
    ap.add_argument("--learned-train-frames", type=int, default=1 << 21)
    ap.add_argument("--learned-eval-frames", type=int, default=1 << 20)
    ap.add_argument("--cpu-frames", type=int, default=4096,
                    help="frames per rate and path (and of the mixed batch) in the CPU-oracle baseline sample")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the oracle check of sampled frames of every timed launch")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this many MiB (a reference kernel "
                         "of known traffic for scaling hardware byte counters)")
    return ap.parse_args()


def progress(msg):
    """One line on stderr as each stage of the benchmark ends."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def source_sha(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2306_12063_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(kernel, sha):
    """The committed rocprofv3 counter summary of a kernel (HBM bytes per
    launch from FETCH_SIZE / WRITE_SIZE, LDS bytes per launch from the LDS
    instruction count), if it was taken on the current kernel source; else {}."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        rec = json.load(fh).get(kernel)
    if not rec or rec.get("source_sha") != sha:
        return {}
    return rec


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "unknown CPU")
    except OSError:
        return "unknown CPU"


def _oracle_jobs(sets):
    """(set name, decode of a frame-index chunk, frames, info bits) per set
    and path: C2 (the Z=81 rates), C1 (the Z=27 code), C3 (the mixed batch,
    each frame with its own code); FP32 NMS and int8 OMS."""
    import oracle
    jobs = []
    for st in sets:
        if st["kind"] == "single":
            for path in ("f32", "i8"):
                if path == "f32":
                    fn = lambda ix, st=st: oracle.decode_f32(st["hbm"], st["Z"], st["llr"][ix], max_iter=ITERS,
                                                             alpha=ALPHA, early_term=False)
                else:
                    fn = lambda ix, st=st: oracle.decode_i8(st["hbm"], st["Z"], st["q"][ix], max_iter=ITERS,
                                                            offset=OFFSET, early_term=False)
                jobs.append((st["name"], fn, len(st["llr"]), len(st["llr"]) * st["K"]))
        else:
            for path in ("f32", "i8"):
                def fn(ix, st=st, path=path):
                    for f in ix:
                        c = st["cid"][f]
                        _, Zc, h = st["codes"][c]
                        n = h.shape[1] * Zc
                        seg = st["llr"][st["off"][f]:st["off"][f] + n][None, :]
                        if path == "f32":
                            oracle.decode_f32(h, Zc, seg, max_iter=ITERS, alpha=ALPHA, early_term=False)
                        else:
                            oracle.decode_i8(h, Zc, oracle.quantize_i8(seg), max_iter=ITERS, offset=OFFSET,
                                             early_term=False)
                jobs.append((st["name"], fn, len(st["cid"]), int(st["kbits"])))
    return jobs


def cpu_baseline(sets):
    """Times the CPU oracle (test infrastructure, never tuned) on bounded
    samples of the workloads: one thread, then every host core the process
    may use (frame chunks over threads; ctypes releases the GIL). Info
    Gbit/s from wall time; frame generation is not timed."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle.build
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    # the GPU machine gives one GPU's job a share of 16 host cores
    threads = max(1, min(16, allowed))
    jobs = _oracle_jobs(sets)

    def run(nt):
        per = {}
        t_all = time.perf_counter()
        with ThreadPoolExecutor(max_workers=nt) as ex:
            for name, fn, nf, kb in jobs:
                t0 = time.perf_counter()
                chunks = [ix for ix in np.array_split(np.arange(nf), nt) if len(ix)]
                list(ex.map(fn, chunks))
                dt = time.perf_counter() - t0
                a = per.setdefault(name, [0, 0.0])
                a[0] += kb
                a[1] += dt
        wall = time.perf_counter() - t_all
        return {k: {"gbit_s": v[0] / v[1] / 1e9, "info_bits": v[0], "seconds": round(v[1], 2)}
                for k, v in per.items()}, wall

    one, w1 = run(1)
    progress(f"CPU oracle, one thread: {w1:.1f} s")
    many, wn = run(threads)
    progress(f"CPU oracle, {threads} threads: {wn:.1f} s")
    flags = " ".join(oracle.build.FLAGS)
    c2n = next(st for st in sets if st["name"] == "C2")
    return {"value": many["C2"]["gbit_s"], "unit": "Gbit/s", "cores": threads, "kind": "oracle",
            "sample": f"{_cpu_model()}; oracle built with gcc {flags}; C2 = first {len(c2n['llr'])} frames "
                      f"of each Z=81 rate at {EBN0_DB} dB, FP32 NMS and int8 OMS, {ITERS} fixed iterations, "
                      f"{threads} threads over frame chunks ({wn:.1f} s wall for all sets)",
            "nproc": os.cpu_count(), "affinity_cores": allowed, "cpu_model": _cpu_model(), "compiler_flags": flags,
            "one_thread": {k: round(v["gbit_s"], 6) for k, v in one.items()},
            "all_cores": {k: round(v["gbit_s"], 6) for k, v in many.items()},
            "sets": {"C1": "1000 frames of the Wi-Fi-shaped rate-1/2 Z=27 code (N=648) at 2 dB",
                     "C2": "a frame subset per Z=81 rate (1/2, 2/3, 3/4, 5/6) at 2 dB, FP32 and int8",
                     "C3": "the first frames of the 114-code mixed batch, each with its own code, FP32 and int8"},
            "seconds": {"one_thread": round(w1, 1), "all_cores": round(wn, 1)}}


def _batch_parity(codes, cid, off, llr_h, bits, iters, ok, path, et, idx):
    """Mismatching frames among `idx` of a batched decode: each frame decoded
    by the oracle with its own code from the same channel values."""
    import oracle
    bad = 0
    for f in idx:
        _, Zc, h = codes[cid[f]]
        n = h.shape[1] * Zc
        seg = llr_h[off[f]:off[f] + n][None, :]
        if path == "f32":
            wb, _, wi, wo = oracle.decode_f32(h, Zc, seg, max_iter=ITERS, alpha=ALPHA, early_term=et)
        else:
            wb, _, wi, wo = oracle.decode_i8(h, Zc, oracle.quantize_i8(seg), max_iter=ITERS, offset=OFFSET,
                                             early_term=et)
        same = (np.array_equal(bits[off[f]:off[f] + n], wb[0]) and int(iters[f]) == int(wi[0])
                and int(ok[f]) == int(wo[0]))
        bad += 0 if same else 1
    return bad


def mixed_batch(P, torch, dev, steps, frames, seed=SEED, graphs=True, parity=True, cpu_frames=0):
    """Frames of all 114 WiMAX-shaped codes (6 rate classes x Z = 24..96) in
    one persistent launch: code ids uniform, ragged lengths, Eb/N0 2 dB.
    Untimed: frame generation and the batch layout autotuner. Timed: `steps`
    FP32 and int8 decodes at 10 fixed iterations, then with early termination.
    After each timing, 40 sampled frames are checked against the oracle."""
    import synth
    codes = synth.wimax_code_set()
    cs = P.Codeset([(h, Z) for _, Z, h in codes])
    rng = np.random.default_rng(seed)
    cid = rng.integers(0, len(codes), frames).astype(np.int32)
    Ns = np.array([h.shape[1] * Z for _, Z, h in codes])
    Ks = np.array([(h.shape[1] - h.shape[0]) * Z for _, Z, h in codes])
    Es = np.array([int((h >= 0).sum()) * Z for _, Z, h in codes])
    off = np.zeros(frames, np.int64)
    off[1:] = np.cumsum(Ns[cid])[:-1]
    Ms = np.array([h.shape[0] * Z for _, Z, h in codes])
    total, kbits, edges = int(Ns[cid].sum()), int(Ks[cid].sum()), int(Es[cid].sum())
    d_off = torch.from_numpy(off).to(dev)
    d_cid = torch.from_numpy(cid).to(dev)
    llr = torch.empty(total, dtype=torch.float32, device=dev)
    for c in range(len(codes)):
        idx = np.flatnonzero(cid == c)
        if len(idx) == 0:
            continue
        _, Z, h = codes[c]
        N, K = h.shape[1] * Z, (h.shape[1] - h.shape[0]) * Z
        s2 = synth.sigma2_from_ebn0(EBN0_DB, K / N)
        cw = P.ldpc_encode(h, Z, P.ldpc_random_bits(seed + 10 * c, len(idx), K, device=dev))
        lc = P.ldpc_awgn_llr(seed + 10 * c + 1, cw, float(np.sqrt(s2)), 2.0 / s2)
        pos = (d_off[torch.from_numpy(idx).to(dev)][:, None] + torch.arange(N, device=dev)[None, :]).reshape(-1)
        llr[pos] = lc.reshape(-1)
    q = P.ldpc_quantize_i8(llr)
    work = torch.empty(cs.work_bytes(frames), dtype=torch.uint8, device=dev)
    bits = torch.empty(total, dtype=torch.uint8, device=dev)
    iters = torch.empty(frames, dtype=torch.int32, device=dev)
    ok = torch.empty(frames, dtype=torch.uint8, device=dev)
    layouts = {"f32": cs.autotune("f32", d_cid, d_off, llr, max_iter=ITERS, work=work),
               "i8": cs.autotune("i8", d_cid, d_off, q, max_iter=ITERS, work=work)}
    res = {}
    stream = torch.cuda.current_stream()
    llr_h = llr.cpu().numpy() if (parity or cpu_frames) else None
    rng_p = np.random.default_rng(seed + 1)
    par = {"frames": 0, "mismatches": 0}
    for path in ("f32", "i8"):
        for et in (False, True):
            def run():
                if path == "f32":
                    cs.decode_f32(d_cid, d_off, llr, max_iter=ITERS, alpha=ALPHA, early_term=et, bits=bits,
                                  iters=iters, ok=ok, work=work, want_post=False)
                else:
                    cs.decode_i8(d_cid, d_off, q, max_iter=ITERS, offset=OFFSET, early_term=et, bits=bits,
                                 iters=iters, ok=ok, work=work, want_post=False)
            run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                run()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            key = f"{path}{'_et' if et else ''}"
            res[key] = {"ms": round(ms, 4), "gbit_s": round(kbits / (ms / 1e3) / 1e9, 3),
                        "mean_iters": round(float(iters.float().mean()), 3),
                        "fer_syndrome": round(1.0 - float(ok.float().mean()), 4)}
            if not et:
                lds_b = float(sum(lds_model_bytes(path, int(Es[c]), int(Ms[c]), ITERS) * n
                                  for c, n in enumerate(np.bincount(cid, minlength=len(codes)))))
                hbm_b = float(sum(hbm_model_bytes(path, int(Ns[c])) * n
                                  for c, n in enumerate(np.bincount(cid, minlength=len(codes)))))
                res[key]["roofline"] = roofline_entry(lds_b, hbm_b, ALG_OPS_PER_EDGE_ITER * edges * ITERS, ms,
                                                      path == "i8", f"ldpc_batch_decode ({path}, with the five "
                                                      f"grouping kernels of the call)")
            if parity:
                idx = np.concatenate([[0, frames - 1], rng_p.choice(frames, 38, replace=False)])
                bad = _batch_parity(codes, cid, off, llr_h, bits.cpu().numpy(), iters.cpu().numpy(),
                                    ok.cpu().numpy(), path, et, idx)
                res[key]["parity"] = {"frames": len(idx), "mismatches": bad}
                par["frames"] += len(idx)
                par["mismatches"] += bad
    # The fixed-iteration decodes captured once each in a HIP graph (the six
    # stream-ordered kernels of a batched decode) and replayed; every replay
    # must reproduce the eager result.
    graph = {}
    for path in (("f32", "i8") if graphs else ()):
        def run_g():
            if path == "f32":
                cs.decode_f32(d_cid, d_off, llr, max_iter=ITERS, alpha=ALPHA, early_term=False, bits=bits,
                              iters=iters, ok=ok, work=work, want_post=False)
            else:
                cs.decode_i8(d_cid, d_off, q, max_iter=ITERS, offset=OFFSET, early_term=False, bits=bits,
                             iters=iters, ok=ok, work=work, want_post=False)
        run_g()
        torch.cuda.synchronize()
        ref = bits.clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):   # warm-up on the capture stream
            run_g()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            run_g()
        bits.zero_()
        g.replay()
        torch.cuda.synchronize()
        same = bool(torch.equal(bits, ref))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        same = same and bool(torch.equal(bits, ref))
        ms = e0.elapsed_time(e1) / steps
        graph[path] = {"ms": round(ms, 4), "gbit_s": round(kbits / (ms / 1e3) / 1e9, 3), "replays_equal_eager": same}
        del g
    if graphs:
        res["graph_replay"] = graph
    if parity:
        res["parity"] = par
    host = None
    if cpu_frames:
        n = min(cpu_frames, frames)
        end = int(off[n - 1] + Ns[cid[n - 1]])
        host = {"name": "C3", "kind": "batch", "codes": codes, "cid": cid[:n], "off": off[:n], "llr": llr_h[:end],
                "kbits": int(Ks[cid[:n]].sum())}
    return host, {"workload": f"114 WiMAX-shaped synthetic codes (rate classes 1/2 2/3A 2/3B 3/4A 3/4B 5/6, "
                        f"Z=24..96, N=576..2304), {frames} frames with uniform code ids in one persistent "
                        f"launch, Eb/N0={EBN0_DB} dB, FP32 NMS alpha={ALPHA} / int8 OMS offset={OFFSET} (two frames "
                        f"per lane in packed FP16), "
                        f"{ITERS} iterations (fixed; _et: early termination)",
            "info_bits": kbits, "layouts": layouts, **res}


def _frames_at(P, hbm, Zc, F, ebn0, seed, dev):
    """info, channel LLRs and their int8 quantisation for F seeded frames."""
    import synth
    info = P.ldpc_code_info(hbm, Zc)
    s2 = synth.sigma2_from_ebn0(ebn0, info["K"] / info["N"])
    bits_in = P.ldpc_random_bits(seed, F, info["K"], device=dev)
    llr = P.ldpc_awgn_llr(seed + 1, P.ldpc_encode(hbm, Zc, bits_in), float(np.sqrt(s2)), 2.0 / s2)
    return bits_in, llr, P.ldpc_quantize_i8(llr)


def _decode_stats(P, torch, run, bits_in, reps):
    """Runs the decode `run` reps times (HIP events around them) and counts
    the last result's errors: (ms per decode, FER, mean iterations)."""
    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        out = run()
    e1.record()
    bits, _, iters, ok = out
    cnt = P.ldpc_frame_stats(bits, bits_in, iters, ok)
    torch.cuda.synchronize()
    c = cnt.cpu().numpy()
    F = bits.shape[0]
    return e0.elapsed_time(e1) / reps, c[1] / F, c[2] / F


def et_sweep(P, torch, dev, frames):
    """Untimed record: the Z=81 codes over Eb/N0 0..5 dB (step 0.5) with
    early termination on (at most 10 iterations): per rate and path, the frame
    error rate, mean iterations and decoded information Gbit/s."""
    import synth
    pts = [0.5 * k for k in range(11)]
    out = {}
    for rate in synth.WIFI_RATES:
        h = synth.wifi_code(rate, Z)
        K = P.ldpc_code_info(h, Z)["K"]
        rows = {"f32": [], "i8": []}
        for k, eb in enumerate(pts):
            bits_in, llr, q = _frames_at(P, h, Z, frames, eb, SEED + 100 * k, dev)
            for path in ("f32", "i8"):
                if path == "f32":
                    run = lambda: P.ldpc_decode_f32(h, Z, llr, max_iter=ITERS, alpha=ALPHA, early_term=True,
                                                    want_post=False)
                else:
                    run = lambda: P.ldpc_decode_i8(h, Z, q, max_iter=ITERS, offset=OFFSET, early_term=True,
                                                   want_post=False)
                ms, fer, it = _decode_stats(P, torch, run, bits_in, 2)
                rows[path].append({"ebn0": eb, "fer": round(float(fer), 6), "mean_iters": round(float(it), 3),
                                   "gbit_s": round(frames * K / (ms / 1e3) / 1e9, 2)})
        out[rate] = rows
    return {"workload": f"Wi-Fi-shaped synthetic codes, Z={Z}, {frames} frames per point, Eb/N0 0..5 dB step "
                        f"0.5, FP32 NMS alpha={ALPHA} and int8 OMS offset={OFFSET}, at most {ITERS} iterations "
                        f"with early termination", "points": out}


def _small_code_host(h, Zs, llr, K):
    import oracle
    l = llr.cpu().numpy()
    return {"name": "C1", "kind": "single", "hbm": h, "Z": Zs, "K": K, "llr": l, "q": oracle.quantize_i8(l)}


def small_code(P, torch, dev):
    """Untimed record: the small Wi-Fi-shaped rate-1/2 code at Z=27 (N=648),
    1000 frames at 2 dB, FP32 NMS with early termination (latency-bound: few
    workgroups), on the layout the tuner picks for 1000 frames."""
    import synth
    Zs, F = 27, 1000
    h = synth.wifi_code("1/2", Zs)
    K = P.ldpc_code_info(h, Zs)["K"]
    bits_in, llr, _ = _frames_at(P, h, Zs, F, EBN0_DB, SEED + 7, dev)
    lay = P.ldpc_autotune_decode(h, Zs, path="f32", max_iter=ITERS, F=F)   # tuned for this small batch
    run = lambda: P.ldpc_decode_f32(h, Zs, llr, max_iter=ITERS, alpha=ALPHA, early_term=True, want_post=False)
    ms, fer, it = _decode_stats(P, torch, run, bits_in, 20)
    return _small_code_host(h, Zs, llr, K), {"workload": f"Wi-Fi-shaped synthetic rate-1/2 code, Z={Zs} (N=648), {F} frames at {EBN0_DB} dB, FP32 "
                        f"NMS alpha={ALPHA}, at most {ITERS} iterations with early termination",
            "ms": round(ms, 4), "gbit_s": round(F * K / (ms / 1e3) / 1e9, 3), "fer": round(float(fer), 5),
            "mean_iters": round(float(it), 3), "layout": {k: lay[k] for k in ("G", "KF", "threads", "hoist", "waves")}}


def learned_gain(train_frames, eval_frames, parity=True):
    """The metric's second part, untimed: Eb/N0 where the first-pass frame
    error rate crosses 1e-3 for plain NMS (alpha 0.75) and for the learned
    per-(iteration, block row, block column) weights, FP32 and int8 (weights
    in 1/16 steps), and each form's mean iterations at plain NMS's 1e-3
    point, on the WiMAX-shaped rate-1/2 code at Z=96 (N=2304) and the
    Wi-Fi-shaped rate-5/6 code at Z=81 (N=1944), beside the Wi-Fi-shaped
    rate-1/2 Z=81 training code. Training on the GPU through the library's
    forward and adjoint kernels: fresh frames at Eb/N0 uniform over the
    code's waterfall, batch 4096, Adam from 1e-2 with a cosine decay to
    1e-3, per-iteration BCE weighted toward early iterations (T - t).
    Evaluation: every decoder on the same frames (graph-replayed sweep
    chunks), early termination on, 10 iterations, each form on the decode
    layout that runs its sweep workload fastest (timed at the middle point)."""
    import synth
    from paper_2306_12063_amd import learned
    rnd = lambda v, n=3: None if v is None else round(float(v), n)
    cases = [("wimax_1/2_z96", "WiMAX-shaped synthetic rate-1/2 code", synth.wimax_code("1/2", 96), 96, (1.5, 3.5),
              [round(1.8 + 0.1 * k, 2) for k in range(15)]),
             ("wifi_5/6_z81", "Wi-Fi-shaped synthetic rate-5/6 code", synth.wifi_code("5/6", 81), 81, (3.8, 5.4),
              [round(4.1 + 0.1 * k, 2) for k in range(11)]),
             ("wifi_1/2_z81", "Wi-Fi-shaped synthetic rate-1/2 code (the training configuration's code)",
              synth.wifi_code("1/2", 81), 81, (1.3, 3.1), [round(1.6 + 0.1 * k, 2) for k in range(13)])]
    out = {}
    for name, what, hbm, Zl, tr, pts in cases:
        r = learned.compare(hbm, Zl, train_frames=train_frames, eval_frames=eval_frames, ebn0_list=pts, seed=1,
                            train_range=tr, lr=1e-2, lr_final=1e-3, iter_loss="early")
        sm = r["summary"]
        progress(f"learned {name}: trained and evaluated")
        par = _learned_parity(hbm, Zl, r["w"], pts[len(pts) // 2]) if parity else None
        out[name] = {
            "workload": f"{what}, Z={Zl} (N={hbm.shape[1] * Zl}); training on {train_frames} fresh frames "
                        f"(Eb/N0 uniform {tr[0]:g}-{tr[1]:g} dB), evaluation on {eval_frames} frames per point at "
                        f"{pts[0]}..{pts[-1]} dB step 0.1, 10 iterations with early termination",
            "train_seconds": rnd(r["train_seconds"], 2),
            "loss_first_last": [rnd(r["loss_first"], 5), rnd(r["loss_last"], 5)],
            "ebn0_at_fer_1e3_db": {k: rnd(v["ebn0_at_fer_1e3"]) for k, v in sm.items()},
            "gain_db": {k: rnd(v["gain_db"]) for k, v in sm.items() if k != "plain_nms_f32"},
            "mean_iters_at_plain_point": {k: rnd(v["mean_iters_at_plain_point"]) for k, v in sm.items()},
            "iter_reduction": {k: rnd(v.get("iter_reduction")) for k, v in sm.items() if k != "plain_nms_f32"},
            "decode_gbit_s": {k: rnd(v["gbit_s"], 2) for k, v in sm.items()},
            "decode_vs_plain": {k: rnd(v["gbit_s"] / sm["plain_nms_f32"]["gbit_s"]) for k, v in sm.items()
                                if k != "plain_nms_f32"},
            "decode_layouts": r["layouts"]}
        if par is not None:
            out[name]["parity"] = par
    return out


def _learned_parity(hbm, Zl, w, ebn0, F=64):
    """The learned FP32 and int8 decoders at the trained weights (the forms
    the comparison timed, early termination on) against the oracle with the
    same weight tables, on F fresh frames at a sweep point."""
    import torch
    import oracle
    import paper_2306_12063_amd as P
    from paper_2306_12063_amd import learned
    from paper_2306_12063_amd.nms import quantize_weights
    _, _, llr = learned.make_frames(hbm, Zl, F, ebn0, 99991)
    q = P.ldpc_quantize_i8(llr)
    wq = quantize_weights(w)
    g32 = P.ldpc_decode_f32(hbm, Zl, llr, max_iter=ITERS, w=w, early_term=True, want_post=False)
    g8 = P.ldpc_decode_i8(hbm, Zl, q, max_iter=ITERS, wq_table=wq, early_term=True, want_post=False)
    torch.cuda.synchronize()
    lh, qh, wh, wqh = llr.cpu().numpy(), q.cpu().numpy(), w.cpu().numpy(), wq.cpu().numpy()
    w32 = oracle.decode_f32(hbm, Zl, lh, max_iter=ITERS, early_term=True, w=wh)
    w8 = oracle.decode_i8(hbm, Zl, qh, max_iter=ITERS, wq_table=wqh, early_term=True)
    bad = 0
    for got, want in ((g32, w32), (g8, w8)):
        gb, gi, go = got[0].cpu().numpy(), got[2].cpu().numpy(), got[3].cpu().numpy()
        rows = (np.any(gb != want[0], axis=1) | (gi != want[2]) | (go != want[3]))
        bad += int(rows.sum())
    return {"frames": 2 * F, "mismatches": bad,
            "int8_weights_equal_oracle_quantiser": bool(np.array_equal(wqh, oracle.quantize_weights(wh)))}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(frames are independent: a multi-GPU run would give each GPU a share of the frames and add up the "
              "error and iteration counters)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2306_12063_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    F = args.frames
    cases = []
    for rate in synth.WIFI_RATES:
        h = synth.wifi_code(rate, Z)
        info = P.ldpc_code_info(h, Z)
        N, K, E, M = info["N"], info["K"], info["E"], info["M"]
        s2 = synth.sigma2_from_ebn0(EBN0_DB, K / N)
        bits_in = P.ldpc_random_bits(SEED, F, K, device=dev)
        cw = P.ldpc_encode(h, Z, bits_in)
        llr = P.ldpc_awgn_llr(SEED + 1, cw, float(np.sqrt(s2)), 2.0 / s2)
        q = P.ldpc_quantize_i8(llr)
        del bits_in, cw
        for path in ("f32", "i8"):
            cases.append(dict(rate=rate, path=path, hbm=h, N=N, K=K, E=E, M=M, llr=llr, q=q,
                              bits=torch.empty((F, N), dtype=torch.uint8, device=dev),
                              iters=torch.empty(F, dtype=torch.int32, device=dev),
                              ok=torch.empty(F, dtype=torch.uint8, device=dev)))
    torch.cuda.synchronize()
    # Untimed: pick each code's fastest decode layout (frames per workgroup and
    # per thread, register variant) with the library's autotuner.
    layouts = {}
    if not args.no_autotune:
        for c in cases:
            cfg = P.ldpc_autotune_decode(c["hbm"], Z, path=c["path"], max_iter=ITERS, F=min(F, 16384))
            layouts[f"{c['path']} {c['rate']}"] = {k: cfg[k] for k in ("G", "KF", "threads", "hoist", "h2", "waves")}
    torch.cuda.synchronize()
    progress("frames generated, decode layouts tuned")

    def launch(c):
        if c["path"] == "f32":
            P.ldpc_decode_f32(c["hbm"], Z, c["llr"], max_iter=ITERS, alpha=ALPHA, early_term=False,
                              bits=c["bits"], iters=c["iters"], ok=c["ok"], want_post=False)
        else:
            P.ldpc_decode_i8(c["hbm"], Z, c["q"], max_iter=ITERS, offset=OFFSET, early_term=False,
                             bits=c["bits"], iters=c["iters"], ok=c["ok"], want_post=False)

    for _ in range(args.warmup):
        for c in cases:
            launch(c)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cases]
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for j, c in enumerate(cases):
            ev[s][j][0].record(stream)
            launch(c)
            ev[s][j][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    progress(f"timed region: {wall:.3f} s")
    info_bits = args.steps * sum(F * c["K"] for c in cases)
    value = info_bits / wall / 1e9
    sha = source_sha("jit_decode.hip", "jit_h2.hip", "jit.cpp")
    per = []
    for j, c in enumerate(cases):
        ms = float(np.mean([ev[s][j][0].elapsed_time(ev[s][j][1]) for s in range(args.steps)]))
        lay = layouts.get(f"{c['path']} {c['rate']}", {})
        kpath = "i8h2" if lay.get("h2") else c["path"]
        name = f"ldpc_decode_{kpath}_z{Z}_mb{c['hbm'].shape[0]}_nb24"
        rl = roofline_entry(F * lds_model_bytes(c["path"], c["E"], c["M"], ITERS),
                            F * hbm_model_bytes(c["path"], c["N"]), ALG_OPS_PER_EDGE_ITER * c["E"] * ITERS * F,
                            ms, bool(lay.get("h2")), name)
        rec = measured_counters(f"decode_{c['path']} rate {c['rate']}", sha)
        rl["traffic"] = rec.get("hbm_bytes_per_launch")
        if rec.get("lds_bytes_per_launch"):
            rl["lds_bytes_measured_per_launch"] = rec["lds_bytes_per_launch"]
            rl["lds_measured_frac"] = round(rec["lds_bytes_per_launch"] / (ms / 1e3) / 1e9 / PEAK_LDS_GBS, 4)
        per.append(dict(case=f"{c['path']} {c['rate']}", ms=ms, gbit_s=F * c["K"] / (ms / 1e3) / 1e9, roofline=rl))

    # Parity of what was timed: the last timed launch of every (rate, path)
    # against the oracle on sampled frames (the first, the last and 62 drawn
    # at random), same channel values and settings.
    parity = None
    if not args.no_parity:
        import oracle
        rng_p = np.random.default_rng(SEED + 5)
        parity = {"frames": 0, "mismatches": 0, "per_case": {}}
        for c in cases:
            idx = np.concatenate([[0, F - 1], rng_p.choice(np.arange(1, F - 1), 62, replace=False)])
            ti = torch.from_numpy(idx).to(dev)
            gb, gi, go = (c[k].index_select(0, ti).cpu().numpy() for k in ("bits", "iters", "ok"))
            if c["path"] == "f32":
                wb, _, wi, wo = oracle.decode_f32(c["hbm"], Z, c["llr"].index_select(0, ti).cpu().numpy(),
                                                  max_iter=ITERS, alpha=ALPHA, early_term=False)
            else:
                wb, _, wi, wo = oracle.decode_i8(c["hbm"], Z, c["q"].index_select(0, ti).cpu().numpy(),
                                                 max_iter=ITERS, offset=OFFSET, early_term=False)
            bad = int((np.any(gb != wb, axis=1) | (gi != wi) | (go != wo)).sum())
            parity["per_case"][f"{c['path']} {c['rate']}"] = bad
            parity["frames"] += len(idx)
            parity["mismatches"] += bad

        progress(f"oracle parity of the timed launches: {parity['mismatches']} of {parity['frames']} frames differ")

    # Secondary, untimed in the headline: the same launches writing their
    # posteriors too (ldpc_decode_* specify them; the paper's throughput counts
    # decoded data bits only).
    with_post = {}
    for c in cases:
        post = torch.empty((F, c["N"]), dtype=torch.float32 if c["path"] == "f32" else torch.int16, device=dev)
        def launch_p(c=c, post=post):
            if c["path"] == "f32":
                P.ldpc_decode_f32(c["hbm"], Z, c["llr"], max_iter=ITERS, alpha=ALPHA, early_term=False,
                                  bits=c["bits"], post=post, iters=c["iters"], ok=c["ok"])
            else:
                P.ldpc_decode_i8(c["hbm"], Z, c["q"], max_iter=ITERS, offset=OFFSET, early_term=False,
                                 bits=c["bits"], post=post, iters=c["iters"], ok=c["ok"])
        launch_p()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            launch_p()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        with_post[f"{c['path']} {c['rate']}"] = {"ms": round(ms, 4), "gbit_s": round(F * c["K"] / (ms / 1e3) / 1e9, 2)}
        del post

    # measured LDS read bandwidth of this device (16-byte reads, every CU busy)
    blocks, rounds = 2048, 2048
    probe_out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    P.ldpc_lds_probe(blocks, rounds, out=probe_out)
    torch.cuda.synchronize()
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    for _ in range(3):
        P.ldpc_lds_probe(blocks, rounds, out=probe_out)
    p1.record(stream)
    torch.cuda.synchronize()
    lds_probe_gbs = blocks * 256 * rounds * 128 / (p0.elapsed_time(p1) / 3 / 1e3) / 1e9
    # the dominant kernel: the longest launch of the step
    dom = max(per, key=lambda p: p["ms"])
    roofline = dict(dom["roofline"])
    roofline["case"] = dom["case"]
    roofline["lds_probe_gbs"] = round(lds_probe_gbs, 1)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+i8", "data": "synthetic",
        "config": {"workload": f"Wi-Fi-shaped synthetic QC-LDPC codes, Z=81 (N=1944), rates 1/2 2/3 3/4 5/6; "
                               f"{F} frames per rate at Eb/N0={EBN0_DB} dB; FP32 NMS alpha={ALPHA} and "
                               f"int8 OMS offset={OFFSET}; {ITERS} fixed iterations, early termination off",
                   "frames_per_launch": F, "iterations": ITERS, "parallelism": "single GPU",
                   "layouts": layouts},
        "roofline": roofline,
        "parity": parity,
        "per_kernel": [{"case": p["case"], "ms": round(p["ms"], 4), "gbit_s": round(p["gbit_s"], 2),
                        "kernel": p["roofline"]["kernel"], "lds_frac": p["roofline"]["lds_frac"],
                        "hbm_frac": p["roofline"]["hbm_frac"], "valu_frac": p["roofline"]["valu"]["frac"],
                        "traffic": p["roofline"]["traffic"]} for p in per],
        "with_posteriors": with_post,
    }
    cpu_sets = []
    if not args.no_cpu_baseline:
        nf = min(args.cpu_frames, F)
        for c in cases:
            if c["path"] == "f32":
                cpu_sets.append({"name": "C2", "kind": "single", "hbm": c["hbm"], "Z": Z, "K": c["K"],
                                 "llr": c["llr"][:nf].cpu().numpy(), "q": c["q"][:nf].cpu().numpy()})
    if not args.no_mixed_batch:
        host, out["mixed_batch"] = mixed_batch(P, torch, dev, args.steps, args.batch_frames,
                                               graphs=not args.no_graph, parity=not args.no_parity,
                                               cpu_frames=0 if args.no_cpu_baseline else args.cpu_frames)
        if host is not None:
            cpu_sets.append(host)
        progress("mixed batch done")
    if not args.no_sweep:
        out["et_sweep"] = et_sweep(P, torch, dev, F)
        host, out["small_code"] = small_code(P, torch, dev)
        progress("early-termination sweep and small code done")
        if not args.no_cpu_baseline:
            cpu_sets.append(host)
    if not args.no_learned:
        out["learned"] = learned_gain(args.learned_train_frames, args.learned_eval_frames,
                                      parity=not args.no_parity)
        progress("learned-versus-plain comparison done")
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_reference"] = {"bytes_read": src.numel() * 4, "bytes_written": dst.numel() * 4}
        del src, dst
    if cpu_sets:
        out["cpu_baseline"] = cpu_baseline(cpu_sets)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
