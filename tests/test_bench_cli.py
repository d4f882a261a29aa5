"""bench.py's command-line contract that needs no GPU: it runs on one GPU and
refuses a multi-GPU request with a message instead of starting."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_exits_with_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1",
                          "--warmup", "0"], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode != 0
    msg = out.stdout + out.stderr
    assert "one GPU" in msg and "--gpus 2" in msg, msg


def test_roofline_entry_takes_the_larger_fraction():
    sys.path.insert(0, ROOT)
    import bench
    # 1 ms launches: LDS bytes at 10% of the LDS peak, HBM at 20% of 8 TB/s
    r = bench.roofline_entry(0.1 * bench.PEAK_LDS_GBS * 1e6, 0.2 * 8000.0 * 1e6, 1e9, 1.0, False, "k")
    assert r["bound"] == "hbm" and abs(r["frac"] - 0.2) < 1e-9 and abs(r["lds_frac"] - 0.1) < 1e-9
    r = bench.roofline_entry(0.3 * bench.PEAK_LDS_GBS * 1e6, 0.2 * 8000.0 * 1e6, 1e9, 1.0, True, "k")
    assert r["bound"] == "lds" and r["unit"] == "GB/s" and abs(r["frac"] - 0.3) < 1e-9
    # a packed 16-bit kernel is priced at twice the 32-bit VALU issue rate
    assert r["valu"]["peak"] == round(2 * bench.PEAK_VALU_TOPS, 1)
    # per-frame LDS model of the method: each edge's posterior read and
    # written per iteration, each row's state read and written: T (2 b_L E + 2 b_row M)
    assert bench.lds_model_bytes("f32", 100, 10, 10) == 10 * (2 * 4 * 100 + 2 * 16 * 10)
    assert bench.lds_model_bytes("i8", 100, 10, 10) == 10 * (2 * 2 * 100 + 2 * 8 * 10)


def test_cpu_baseline_runs_the_oracle_on_every_set():
    # the baseline leg on tiny sets (CPU only): one thread and all cores,
    # each set's info bits counted
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    import oracle
    import synth
    h27 = synth.wifi_code("1/2", 27)
    _, _, l27 = oracle.llr_frames(h27, 27, 6, 2.0, 3)
    h81 = synth.wifi_code("5/6", 81)
    _, _, l81 = oracle.llr_frames(h81, 81, 5, 2.0, 4)
    codes = synth.wimax_code_set()[:3]
    Ns = [h.shape[1] * z for _, z, h in codes]
    cid = np.array([0, 2, 1, 2], np.int32)
    off = np.cumsum([0] + [Ns[c] for c in cid[:-1]]).astype(np.int64)
    llr = np.zeros(int(off[-1] + Ns[cid[-1]]), np.float32)
    kb = sum((h.shape[1] - h.shape[0]) * z for c in cid for _, z, h in [codes[c]])
    sets = [{"name": "C2", "kind": "single", "hbm": h81, "Z": 81, "K": 1620, "llr": l81, "q": oracle.quantize_i8(l81)},
            {"name": "C1", "kind": "single", "hbm": h27, "Z": 27, "K": 324, "llr": l27, "q": oracle.quantize_i8(l27)},
            {"name": "C3", "kind": "batch", "codes": codes, "cid": cid, "off": off, "llr": llr, "kbits": kb}]
    r = bench.cpu_baseline(sets)
    assert r["kind"] == "oracle" and r["value"] > 0 and r["cores"] >= 1
    for part in ("one_thread", "all_cores"):
        assert set(r[part]) == {"C1", "C2", "C3"} and all(v > 0 for v in r[part].values())
    assert "-O3" in r["compiler_flags"] and "-ffp-contract=off" in r["compiler_flags"]
