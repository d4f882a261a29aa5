"""Every layout the autotuners may keep is exact against the oracle.

The decode autotuner chooses, per code and arithmetic path, among layouts
(frames per workgroup and per thread, hoisted gather addresses, two frames
per lane in packed FP16, an occupancy hint that may spill a few registers);
the batch autotuner among six persistent-kernel layouts. The choice depends
on timings, so each candidate is installed explicitly here
(ldpc_set_decode_layout, Codeset.set_layout) and must give the oracle's
bits, posteriors, iteration counts and ok flags exactly, with early
termination on and off (the layouts change the launch, never the
arithmetic of Sec. 4, eqs. 20-23)."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2306_12063_amd as P

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


CODES = [("wifi", r, 81) for r in synth.WIFI_RATES] + [("wimax", "1/2", 96), ("wifi", "1/2", 27)]


@pytest.mark.parametrize("path", ["f32", "i8"])
@pytest.mark.parametrize("code", CODES, ids=lambda c: f"{c[0]}-{c[1]}-z{c[2]}")
def test_every_decode_layout_exact(code, path):
    kind, rate, Z = code
    h = synth.wifi_code(rate, Z) if kind == "wifi" else synth.wimax_code(rate, Z)
    _, _, llr = oracle.llr_frames(h, Z, 131, 1.5, 23)   # 131 frames: ragged last workgroup for every layout
    q = oracle.quantize_i8(llr)
    layouts = P.ldpc_decode_layouts(h, Z, path)
    assert layouts, "the tuner has no candidate"
    if path == "i8":
        assert any(l["h2"] for l in layouts), "packed-FP16 layouts missing"
    want = {}
    for et in (True, False):
        if path == "f32":
            want[et] = oracle.decode_f32(h, Z, llr, max_iter=10, alpha=0.75, early_term=et)
        else:
            want[et] = oracle.decode_i8(h, Z, q, max_iter=10, offset=1, early_term=et)
    try:
        for lay in layouts:
            P.ldpc_set_decode_layout(h, Z, path, lay)
            for et in (True, False):
                if path == "f32":
                    got = P.ldpc_decode_f32(h, Z, _gpu(llr), max_iter=10, alpha=0.75, early_term=et)
                else:
                    got = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=10, offset=1, early_term=et)
                torch.cuda.synchronize()
                for g, w, what in zip(got, want[et], ("bits", "posteriors", "iterations", "ok")):
                    assert np.array_equal(g.cpu().numpy(), w), (lay, et, what)
    finally:
        P.ldpc_set_decode_layout(h, Z, path, None)


@pytest.mark.parametrize("path", ["f32w", "i8w"])
@pytest.mark.parametrize("code", [("wifi", "1/2", 81), ("wifi", "5/6", 81), ("wimax", "1/2", 96)],
                         ids=lambda c: f"{c[0]}-{c[1]}-z{c[2]}")
def test_every_weighted_layout_exact(code, path):
    """The layouts the tuner times for the kernels with a weight table (FP32
    weights; int8 weights in 1/16 steps, one or two frames per lane), each
    installed as the tuned one: bit-exact against the oracle with the same
    table."""
    kind, rate, Z = code
    h = synth.wifi_code(rate, Z) if kind == "wifi" else synth.wimax_code(rate, Z)
    _, _, llr = oracle.llr_frames(h, Z, 67, 1.5, 29)
    q = oracle.quantize_i8(llr)
    rng = np.random.default_rng(5)
    w = rng.uniform(0.5, 1.0, (10,) + h.shape).astype(np.float32)
    wq = oracle.quantize_weights(w)
    layouts = P.ldpc_decode_layouts(h, Z, path)
    assert layouts
    # the int8 table runs two frames per lane in packed FP16 too; FP32 never does
    assert any(l["h2"] for l in layouts) == (path == "i8w")
    want = {et: (oracle.decode_f32(h, Z, llr, max_iter=10, early_term=et, w=w) if path == "f32w" else
                 oracle.decode_i8(h, Z, q, max_iter=10, wq_table=wq, early_term=et)) for et in (True, False)}
    try:
        for lay in layouts:
            P.ldpc_set_decode_layout(h, Z, path, lay)
            for et in (True, False):
                if path == "f32w":
                    got = P.ldpc_decode_f32(h, Z, _gpu(llr), max_iter=10, w=_gpu(w), early_term=et)
                else:
                    got = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=10, wq_table=_gpu(wq), early_term=et)
                torch.cuda.synchronize()
                for g, ww, what in zip(got, want[et], ("bits", "posteriors", "iterations", "ok")):
                    assert np.array_equal(g.cpu().numpy(), ww), (lay, et, what)
    finally:
        P.ldpc_set_decode_layout(h, Z, path, None)


def test_set_layout_validation():
    h = synth.wifi_code("1/2", 81)
    lay = P.ldpc_decode_layouts(h, 81, "f32")[0]
    for bad in ({**lay, "threads": lay["threads"] + 64}, {**lay, "FWp": lay["FWp"] + 1}, {**lay, "hoist": 13},
                {**lay, "waves": 2}, {**lay, "h2": 1}):
        with pytest.raises(P.LdpcError):
            P.ldpc_set_decode_layout(h, 81, "f32", bad)
    with pytest.raises(P.LdpcError):
        P.ldpc_set_decode_layout(h, 81, "i8", {**lay, "G": 40})
    h2lay = next(l for l in P.ldpc_decode_layouts(h, 81, "i8") if l["h2"])
    with pytest.raises(P.LdpcError):   # no packed FP16 on the FP32 table path
        P.ldpc_set_decode_layout(h, 81, "f32w", h2lay)
    P.ldpc_set_decode_layout(h, 81, "i8w", h2lay)
    P.ldpc_set_decode_layout(h, 81, "i8w", None)
    P.ldpc_set_decode_layout(h, 81, "f32", None)


@pytest.fixture(scope="module")
def wimax_set():
    codes = synth.wimax_code_set()
    return codes, P.Codeset([(h, Z) for _, Z, h in codes])


BATCH_LAYOUTS = [(256, 1), (192, 1), (384, 1), (512, 1), (256, 2), (512, 2)]


@pytest.mark.parametrize("path", ["f32", "i8"])
def test_every_batch_layout_exact(wimax_set, path):
    codes, cs = wimax_set
    F = 300
    rng = np.random.default_rng(41)
    cid = rng.integers(0, len(codes), F).astype(np.int32)
    Ns = np.array([h.shape[1] * Z for _, Z, h in codes])
    off = np.zeros(F, np.int64)
    off[1:] = np.cumsum(Ns[cid])[:-1]
    llr = np.zeros(int(Ns[cid].sum()), np.float32)
    per = {}
    for c in np.unique(cid):
        idx = np.flatnonzero(cid == c)
        _, Z, h = codes[c]
        _, _, l = oracle.llr_frames(h, Z, len(idx), 2.0, 300 + int(c))
        for k, f in enumerate(idx):
            llr[off[f]:off[f] + Ns[c]] = l[k]
        per[int(c)] = (idx, l)
    q = oracle.quantize_i8(llr)
    want = {}
    for c, (idx, l) in per.items():
        _, Z, h = codes[c]
        for et in (True, False):
            if path == "f32":
                want[c, et] = oracle.decode_f32(h, Z, l, max_iter=8, alpha=0.75, early_term=et)
            else:
                want[c, et] = oracle.decode_i8(h, Z, oracle.quantize_i8(l), max_iter=8, offset=1, early_term=et)
    d_cid, d_off = _gpu(cid), _gpu(off)
    try:
        for threads, div in BATCH_LAYOUTS:
            cs.set_layout(path, threads, div)
            for et in (True, False):
                if path == "f32":
                    out = cs.decode_f32(d_cid, d_off, _gpu(llr), max_iter=8, alpha=0.75, early_term=et)
                else:
                    out = cs.decode_i8(d_cid, d_off, _gpu(q), max_iter=8, offset=1, early_term=et)
                torch.cuda.synchronize()
                bits, post, iters, ok = (t.cpu().numpy() for t in out)
                for c, (idx, _) in per.items():
                    wb, wp, wi, wo = want[c, et]
                    N = Ns[c]
                    for k, f in enumerate(idx):
                        s = slice(off[f], off[f] + N)
                        assert np.array_equal(bits[s], wb[k]) and np.array_equal(post[s], wp[k]), \
                            (threads, div, et, c, f)
                    assert np.array_equal(iters[idx], wi) and np.array_equal(ok[idx], wo), (threads, div, et, c)
    finally:
        cs.set_layout(path, 256, 1)


def test_batch_layout_validation(wimax_set):
    _, cs = wimax_set
    for threads, div in ((128, 1), (192, 2), (320, 1), (1024, 1)):
        with pytest.raises(P.LdpcError):
            cs.set_layout("f32", threads, div)
    # a code wider than 192 threads cannot take the 192-thread layout
    wide = P.Codeset([(synth.wifi_code("5/6", 224), 224)])
    with pytest.raises(P.LdpcError):
        wide.set_layout("f32", 192, 1)
    wide.set_layout("f32", 256, 1)
