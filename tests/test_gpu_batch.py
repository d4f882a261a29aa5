"""GPU parity of the batched persistent decoder on a ragged mix of codes
(WiMAX-shaped, 6 rate classes x 19 expansion factors): every frame must
decode exactly as the oracle decodes it with its own code; the decode must
also replay exactly from a captured graph."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2306_12063_amd as P

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def wimax_set():
    codes = synth.wimax_code_set()
    return codes, P.Codeset([(h, Z) for _, Z, h in codes])


def _ragged(codes, F, ebn0, seed, frames_per_code=None):
    rng = np.random.default_rng(seed)
    cid = rng.integers(0, len(codes), F).astype(np.int32)
    Ns = np.array([h.shape[1] * Z for _, Z, h in codes])
    off = np.zeros(F, np.int64)
    off[1:] = np.cumsum(Ns[cid])[:-1]
    total = int(Ns[cid].sum())
    llr = np.zeros(total, np.float32)
    per = {}
    for c in np.unique(cid):
        idx = np.flatnonzero(cid == c)
        _, Z, h = codes[c]
        _, _, l = oracle.llr_frames(h, Z, len(idx), ebn0, seed + 31 * int(c))
        N = Ns[c]
        for k, f in enumerate(idx):
            llr[off[f]:off[f] + N] = l[k]
        per[int(c)] = (idx, l)
    return cid, off, llr, total, per


def test_codeset_classes(wimax_set):
    codes, cs = wimax_set
    assert cs.n == 114
    assert cs.info[0]["nclass"] == 6
    for c, (cls, Z, h) in enumerate(codes):
        assert cs.info[c]["N"] == 24 * Z and cs.info[c]["G"] == min(64, 256 // Z)


@pytest.mark.parametrize("path", ["f32", "i8"])
@pytest.mark.parametrize("et", [True, False])
def test_batch_matches_oracle(wimax_set, path, et):
    codes, cs = wimax_set
    F = 400
    cid, off, llr, total, per = _ragged(codes, F, 2.0, 5)
    d = lambda x: torch.from_numpy(x).to(DEV)
    if path == "f32":
        bits, post, iters, ok = cs.decode_f32(d(cid), d(off), d(llr), max_iter=8, alpha=0.75, early_term=et)
    else:
        q = oracle.quantize_i8(llr)
        bits, post, iters, ok = cs.decode_i8(d(cid), d(off), d(q), max_iter=8, offset=1, early_term=et)
    torch.cuda.synchronize()
    bits, post, iters, ok = (t.cpu().numpy() for t in (bits, post, iters, ok))
    for c, (idx, l) in per.items():
        _, Z, h = codes[c]
        N = 24 * Z
        if path == "f32":
            wb, wp, wi, wo = oracle.decode_f32(h, Z, l, max_iter=8, alpha=0.75, early_term=et)
        else:
            wb, wp, wi, wo = oracle.decode_i8(h, Z, oracle.quantize_i8(l), max_iter=8, offset=1, early_term=et)
        for k, f in enumerate(idx):
            assert np.array_equal(bits[off[f]:off[f] + N], wb[k]), (c, f)
            assert np.array_equal(post[off[f]:off[f] + N], wp[k]), (c, f)
        assert np.array_equal(iters[idx], wi) and np.array_equal(ok[idx], wo), c


def test_batch_graph_replay(wimax_set):
    codes, cs = wimax_set
    F = 300
    cid, off, llr, total, per = _ragged(codes, F, 1.5, 9)
    d_cid, d_off, d_llr = (torch.from_numpy(x).to(DEV) for x in (cid, off, llr))
    work = torch.empty(cs.work_bytes(F), dtype=torch.uint8, device=DEV)
    out = [torch.empty(total, dtype=torch.uint8, device=DEV), torch.empty(total, dtype=torch.float32, device=DEV),
           torch.empty(F, dtype=torch.int32, device=DEV), torch.empty(F, dtype=torch.uint8, device=DEV)]
    eager = [t.clone() for t in cs.decode_f32(d_cid, d_off, d_llr, max_iter=10, work=work)]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):       # warm up on the capture stream
        cs.decode_f32(d_cid, d_off, d_llr, max_iter=10, bits=out[0], post=out[1], iters=out[2], ok=out[3], work=work)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cs.decode_f32(d_cid, d_off, d_llr, max_iter=10, bits=out[0], post=out[1], iters=out[2], ok=out[3], work=work)
    for rep in range(3):
        for t in out:
            t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, eager):
            assert torch.equal(a, b), rep
        # unrelated eager work between replays
        cs.decode_i8(d_cid, d_off, torch.zeros(total, dtype=torch.int8, device=DEV), max_iter=2)
        torch.cuda.synchronize()


def test_batch_full_size_sampled(wimax_set):
    # 2^18 frames with uniformly drawn code ids in one persistent launch,
    # FP32 and int8; the oracle checks a sample of frames.
    codes, cs = wimax_set
    F = 1 << 18
    rng = np.random.default_rng(3)
    cid = rng.integers(0, len(codes), F).astype(np.int32)
    Ns = np.array([h.shape[1] * Z for _, Z, h in codes])
    off = np.zeros(F, np.int64)
    off[1:] = np.cumsum(Ns[cid])[:-1]
    total = int(Ns[cid].sum())
    llr = torch.empty(total, dtype=torch.float32, device=DEV)
    d_off = torch.from_numpy(off).to(DEV)
    for c in range(len(codes)):
        idx = np.flatnonzero(cid == c)
        if len(idx) == 0:
            continue
        _, Z, h = codes[c]
        N, K = 24 * Z, (24 - h.shape[0]) * Z
        s2 = synth.sigma2_from_ebn0(2.0, K / N)
        cw = P.ldpc_encode(h, Z, P.ldpc_random_bits(100 + c, len(idx), K))
        l = P.ldpc_awgn_llr(200 + c, cw, float(np.sqrt(s2)), 2.0 / s2)
        pos = (d_off[torch.from_numpy(idx).to(DEV)][:, None] + torch.arange(N, device=DEV)[None, :]).reshape(-1)
        llr[pos] = l.reshape(-1)
    bits, post, iters, ok = cs.decode_f32(torch.from_numpy(cid).to(DEV), d_off, llr, max_iter=10, early_term=False)
    torch.cuda.synchronize()
    sample = rng.choice(F, 40, replace=False)
    lh = llr.cpu().numpy()
    bh, ph, ih = bits.cpu().numpy(), post.cpu().numpy(), iters.cpu().numpy()
    for f in sample:
        _, Z, h = codes[cid[f]]
        N = 24 * Z
        wb, wp, wi, _ = oracle.decode_f32(h, Z, lh[off[f]:off[f] + N][None], max_iter=10, early_term=False)
        assert np.array_equal(bh[off[f]:off[f] + N], wb[0]) and np.array_equal(ph[off[f]:off[f] + N], wp[0])
        assert ih[f] == wi[0]
    # the int8 path (two frames per lane in packed FP16) on the same frames
    q = P.ldpc_quantize_i8(llr)
    bits, post, iters, ok = cs.decode_i8(torch.from_numpy(cid).to(DEV), d_off, q, max_iter=10, offset=1,
                                         early_term=False)
    torch.cuda.synchronize()
    qh, bh, ph, ih, oh = (t.cpu().numpy() for t in (q, bits, post, iters, ok))
    for f in np.concatenate([[0, F - 1], rng.choice(F, 38, replace=False)]):
        _, Z, h = codes[cid[f]]
        N = 24 * Z
        wb, wp, wi, wo = oracle.decode_i8(h, Z, qh[off[f]:off[f] + N][None], max_iter=10, offset=1, early_term=False)
        assert np.array_equal(bh[off[f]:off[f] + N], wb[0]) and np.array_equal(ph[off[f]:off[f] + N], wp[0])
        assert ih[f] == wi[0] and oh[f] == wo[0]


def test_batch_autotune_keeps_parity():
    # the tuner rebuilds the code set's tables for each layout; the chosen
    # layout must still decode every frame exactly as the oracle does
    all_codes = synth.wimax_code_set()
    codes = [all_codes[k] for k in range(0, len(all_codes), 10)]
    cs = P.Codeset([(h, Z) for _, Z, h in codes])
    F = 160
    cid, off, llr, total, per = _ragged(codes, F, 2.5, 17)
    d = lambda x: torch.from_numpy(x).to(DEV)
    q = oracle.quantize_i8(llr)
    for path in ("f32", "i8"):
        src = d(llr) if path == "f32" else d(q)
        cfg = cs.autotune(path, d(cid), d(off), src, max_iter=6)
        assert cfg["threads"] in (192, 256, 384, 512) and cfg["divisor"] in (1, 2) and cfg["ms"] > 0
        if path == "f32":
            bits, post, iters, ok = cs.decode_f32(d(cid), d(off), src, max_iter=6, alpha=0.75, early_term=True)
        else:
            bits, post, iters, ok = cs.decode_i8(d(cid), d(off), src, max_iter=6, offset=1, early_term=True)
        torch.cuda.synchronize()
        bits, post, iters = bits.cpu().numpy(), post.cpu().numpy(), iters.cpu().numpy()
        for c, (idx, l) in per.items():
            _, Z, h = codes[c]
            N = 24 * Z
            if path == "f32":
                wb, wp, wi, _ = oracle.decode_f32(h, Z, l, max_iter=6, alpha=0.75, early_term=True)
            else:
                wb, wp, wi, _ = oracle.decode_i8(h, Z, oracle.quantize_i8(l), max_iter=6, offset=1, early_term=True)
            for k, f in enumerate(idx):
                assert np.array_equal(bits[off[f]:off[f] + N], wb[k]) and np.array_equal(post[off[f]:off[f] + N], wp[k])
            assert np.array_equal(iters[idx], wi)


@pytest.mark.parametrize("path", ["f32", "i8"])
def test_batch_grouping_one_dominant_code(path):
    # Frames of a batch are grouped by code in per-workgroup LDS counts with
    # one global count per code and workgroup: here most of 9000 frames (three
    # such workgroups) share one code, some carry invalid code ids and a few
    # offsets that would reach outside the buffers (those frames are not
    # decoded: iters -1, ok 0, bits and posteriors untouched), and one code
    # has N < 256, so a thread's share of a work item spans several frames.
    codes = [("1/2", 8, synth.wimax_code("1/2", 8, seed=4)), ("5/6", 24, synth.wimax_code("5/6", 24, seed=5)),
             ("3/4A", 52, synth.wimax_code("3/4A", 52, seed=6))]
    cs = P.Codeset([(h, Z) for _, Z, h in codes])
    F = 9000
    rng = np.random.default_rng(21)
    cid = np.where(rng.random(F) < 0.9, 1, rng.integers(-1, 4, F)).astype(np.int32)   # -1 and 3 are invalid
    Ns = np.array([24 * Z for _, Z, _ in codes])
    Nf = np.array([Ns[c] if 0 <= c < 3 else 16 for c in cid])
    off = np.zeros(F, np.int64)
    off[1:] = np.cumsum(Nf)[:-1]
    total = int(Nf.sum())
    llr = np.zeros(total, np.float32)
    per = {}
    for c in range(3):
        idx = np.flatnonzero(cid == c)
        _, Z, h = codes[c]
        _, _, l = oracle.llr_frames(h, Z, len(idx), 2.5, 40 + c)
        for k, f in enumerate(idx):
            llr[off[f]:off[f] + Ns[c]] = l[k]
        per[c] = (idx, l)
    # frames of valid codes whose offsets leave the buffers (checked on the
    # device against the element count the binding passes)
    moved = {}
    for f, o in zip(per[1][0][[3, 50, 400, 2000, 5000]], (-1, -int(Ns[1]), total - int(Ns[1]) + 1, total, 1 << 40)):
        moved[int(f)] = int(off[f])
        off[f] = o
    d = lambda x: torch.from_numpy(x).to(DEV)
    bits = torch.full((total,), 7, dtype=torch.uint8, device=DEV)
    iters = torch.full((F,), -5, dtype=torch.int32, device=DEV)
    ok = torch.full((F,), 9, dtype=torch.uint8, device=DEV)
    if path == "f32":
        bits, post, iters, ok = cs.decode_f32(d(cid), d(off), d(llr), max_iter=6, alpha=0.75, early_term=True,
                                              bits=bits, iters=iters, ok=ok)
    else:
        bits, post, iters, ok = cs.decode_i8(d(cid), d(off), d(oracle.quantize_i8(llr)), max_iter=6, offset=1,
                                             early_term=True, bits=bits, iters=iters, ok=ok)
    torch.cuda.synchronize()
    bits, post, iters, ok = bits.cpu().numpy(), post.cpu().numpy(), iters.cpu().numpy(), ok.cpu().numpy()
    for c, (idx, l) in per.items():
        _, Z, h = codes[c]
        if path == "f32":
            wb, wp, wi, wo = oracle.decode_f32(h, Z, l, max_iter=6, alpha=0.75, early_term=True)
        else:
            wb, wp, wi, wo = oracle.decode_i8(h, Z, oracle.quantize_i8(l), max_iter=6, offset=1, early_term=True)
        for k, f in enumerate(idx):
            if int(f) in moved:
                continue
            s = slice(off[f], off[f] + Ns[c])
            assert np.array_equal(bits[s], wb[k]) and np.array_equal(post[s], wp[k]) and iters[f] == wi[k], (c, f)
            assert ok[f] == wo[k]
    bad = np.flatnonzero((cid < 0) | (cid >= 3))
    assert len(bad) > 0
    for f in bad:
        assert iters[f] == -1 and ok[f] == 0 and np.all(bits[off[f]:off[f] + 16] == 7)
    for f, o in moved.items():
        assert iters[f] == -1 and ok[f] == 0 and np.all(bits[o:o + Ns[1]] == 7), f


@pytest.mark.parametrize("packed", [True, False])
@pytest.mark.parametrize("wq", [0, 12])
def test_batch_i8_forms(monkeypatch, packed, wq):
    # the fixed-point batch with two frames per lane in packed FP16 (default
    # for these codes, column weight <= 15) and, with LDPC_BATCH_H2=0 at
    # code-set creation, one frame per lane (the form used for codes of
    # larger column weight); offset (wq = 0) and weight wq/16 magnitudes
    if not packed:
        monkeypatch.setenv("LDPC_BATCH_H2", "0")
    all_codes = synth.wimax_code_set()
    codes = [all_codes[k] for k in range(3, len(all_codes), 9)]
    cs = P.Codeset([(h, Z) for _, Z, h in codes])
    F = 150
    cid, off, llr, total, per = _ragged(codes, F, 2.0, 23)
    q = oracle.quantize_i8(llr)
    d = lambda x: torch.from_numpy(x).to(DEV)
    for et in (True, False):
        bits, post, iters, ok = cs.decode_i8(d(cid), d(off), d(q), max_iter=7, offset=1, wq=wq, early_term=et)
        torch.cuda.synchronize()
        bits, post, iters = bits.cpu().numpy(), post.cpu().numpy(), iters.cpu().numpy()
        for c, (idx, l) in per.items():
            _, Z, h = codes[c]
            wb, wp, wi, _ = oracle.decode_i8(h, Z, oracle.quantize_i8(l), max_iter=7, offset=1, wq=wq,
                                             early_term=et)
            for k, f in enumerate(idx):
                s = slice(off[f], off[f] + 24 * Z)
                assert np.array_equal(bits[s], wb[k]) and np.array_equal(post[s], wp[k]) and iters[f] == wi[k]


@pytest.mark.parametrize("with_heavy", [False, True])
def test_batch_mixed_families(with_heavy):
    # Wi-Fi-shaped Z=81 codes and WiMAX-shaped codes in one code set (four
    # structure classes); with a code of column weight 16 added, the int8
    # batch must leave packed FP16 for the whole set (one frame per lane).
    codes = [("wifi 1/2", 81, synth.wifi_code("1/2", 81)), ("wifi 5/6", 81, synth.wifi_code("5/6", 81)),
             ("wimax 2/3B", 40, synth.wimax_code("2/3B", 40))]
    if with_heavy:
        codes.append(("weight 16", 32, synth.heavy_column_code(16, 16, 32, 66)))
    cs = P.Codeset([(h, Z) for _, Z, h in codes])
    assert cs.info[0]["nclass"] == len(codes)
    F = 240
    rng = np.random.default_rng(8)
    cid = rng.integers(0, len(codes), F).astype(np.int32)
    Ns = np.array([24 * Z for _, Z, _ in codes])
    off = np.zeros(F, np.int64)
    off[1:] = np.cumsum(Ns[cid])[:-1]
    llr = np.zeros(int(Ns[cid].sum()), np.float32)
    per = {}
    for c in range(len(codes)):
        idx = np.flatnonzero(cid == c)
        l = synth.zero_word_llr(Ns[c], len(idx), 90 + c, sigma=0.85)
        for k, f in enumerate(idx):
            llr[off[f]:off[f] + Ns[c]] = l[k]
        per[c] = (idx, l)
    d = lambda x: torch.from_numpy(x).to(DEV)
    for path in ("f32", "i8"):
        if path == "f32":
            bits, post, iters, ok = cs.decode_f32(d(cid), d(off), d(llr), max_iter=8, alpha=0.75, early_term=True)
        else:
            bits, post, iters, ok = cs.decode_i8(d(cid), d(off), d(oracle.quantize_i8(llr)), max_iter=8, offset=1,
                                                 early_term=True)
        torch.cuda.synchronize()
        bits, post, iters = bits.cpu().numpy(), post.cpu().numpy(), iters.cpu().numpy()
        for c, (idx, l) in per.items():
            _, Z, h = codes[c]
            if path == "f32":
                wb, wp, wi, _ = oracle.decode_f32(h, Z, l, max_iter=8, alpha=0.75, early_term=True)
            else:
                wb, wp, wi, _ = oracle.decode_i8(h, Z, oracle.quantize_i8(l), max_iter=8, offset=1, early_term=True)
            for k, f in enumerate(idx):
                s = slice(off[f], off[f] + Ns[c])
                assert np.array_equal(bits[s], wb[k]) and np.array_equal(post[s], wp[k]) and iters[f] == wi[k], \
                    (path, codes[c][0], f)


def test_batch_at_size_limits():
    # codes at the kernels' limits (Z = 256, 32 block columns; 16 block rows,
    # or a block row of check degree 26) beside a small code in one code set
    codes = [("16 rows", 256, synth.limit_code(16, 32, 256, 18, 6, 86)),
             ("degree 26", 256, synth.limit_code(6, 32, 256, 26, 6, 76)),
             ("wifi 1/2", 27, synth.wifi_code("1/2", 27))]
    cs = P.Codeset([(h, Z) for _, Z, h in codes])
    F = 30
    rng = np.random.default_rng(12)
    cid = rng.integers(0, len(codes), F).astype(np.int32)
    Ns = np.array([h.shape[1] * Z for _, Z, h in codes])
    off = np.zeros(F, np.int64)
    off[1:] = np.cumsum(Ns[cid])[:-1]
    llr = np.zeros(int(Ns[cid].sum()), np.float32)
    per = {}
    for c in range(len(codes)):
        idx = np.flatnonzero(cid == c)
        _, Z, h = codes[c]
        _, _, l = oracle.llr_frames(h, Z, len(idx), 3.0, 95 + c)
        for k, f in enumerate(idx):
            llr[off[f]:off[f] + Ns[c]] = l[k]
        per[c] = (idx, l)
    d = lambda x: torch.from_numpy(x).to(DEV)
    for path in ("f32", "i8"):
        if path == "f32":
            bits, post, iters, ok = cs.decode_f32(d(cid), d(off), d(llr), max_iter=6, alpha=0.75, early_term=True)
        else:
            bits, post, iters, ok = cs.decode_i8(d(cid), d(off), d(oracle.quantize_i8(llr)), max_iter=6, offset=1,
                                                 early_term=True)
        torch.cuda.synchronize()
        bits, post, iters = bits.cpu().numpy(), post.cpu().numpy(), iters.cpu().numpy()
        for c, (idx, l) in per.items():
            _, Z, h = codes[c]
            if path == "f32":
                wb, wp, wi, _ = oracle.decode_f32(h, Z, l, max_iter=6, alpha=0.75, early_term=True)
            else:
                wb, wp, wi, _ = oracle.decode_i8(h, Z, oracle.quantize_i8(l), max_iter=6, offset=1, early_term=True)
            for k, f in enumerate(idx):
                s = slice(off[f], off[f] + Ns[c])
                assert np.array_equal(bits[s], wb[k]) and np.array_equal(post[s], wp[k]) and iters[f] == wi[k], \
                    (path, codes[c][0], f)
