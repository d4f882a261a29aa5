"""GPU parity of the layered decoders against the CPU oracle.

Bar: FP32 hard bits, iteration counts and ok flags exactly equal; FP32
posteriors within 1e-5 relative (compared by value, so +0 and -0 agree);
fixed point bit-exact. All inputs come from the seeded generator and the
oracle's own encoder and channel."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2306_12063_amd as P

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _frames(hbm, Z, F, ebn0, seed):
    info, cw, llr = oracle.llr_frames(hbm, Z, F, ebn0, seed)
    return info, cw, llr


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _assert_f32_parity(got, want, rtol=1e-5):
    gb, gp, gi, go = (t.cpu().numpy() if t is not None else None for t in got)
    wb, wp, wi, wo = want
    assert np.array_equal(gi, wi), f"iterations differ on {np.sum(gi != wi)} frames"
    assert np.array_equal(go, wo), "ok flags differ"
    assert np.array_equal(gb, wb), f"hard bits differ on {np.sum(np.any(gb != wb, axis=1))} frames"
    if gp is not None:
        np.testing.assert_allclose(gp, wp, rtol=rtol, atol=0)
    return gp, wp


def _decode_f32_both(h, Z, llr, **kw):
    got = P.ldpc_decode_f32(h, Z, _gpu(llr), **kw)
    torch.cuda.synchronize()
    want = oracle.decode_f32(h, Z, llr, **{k: v for k, v in kw.items()})
    return got, want


@pytest.mark.parametrize("early_term", [True, False])
def test_wifi_rate_half_z27(early_term):
    # 1000 frames of the rate-1/2, Z = 27 Wi-Fi-shaped code at Eb/N0 = 2 dB.
    h = synth.wifi_code("1/2", 27)
    _, _, llr = _frames(h, 27, 1000, 2.0, 1)
    got, want = _decode_f32_both(h, 27, llr, max_iter=10, alpha=0.75, early_term=early_term)
    gp, wp = _assert_f32_parity(got, want)
    assert np.array_equal(gp, wp)   # no rounding-order freedom: bit-identical


@pytest.mark.parametrize("rate", list(synth.WIFI_RATES))
@pytest.mark.parametrize("ebn0", [0.5, 2.5])
def test_wifi_z81_all_rates(rate, ebn0):
    h = synth.wifi_code(rate, 81)
    _, _, llr = _frames(h, 81, 131, ebn0, 7)         # 131 frames: several workgroups and a ragged tail
    got, want = _decode_f32_both(h, 81, llr, max_iter=10, alpha=0.75, early_term=True)
    gp, wp = _assert_f32_parity(got, want)
    assert np.array_equal(gp, wp)


@pytest.mark.parametrize("cls", list(synth.WIMAX_CLASSES))
@pytest.mark.parametrize("Z", [24, 52, 96])
def test_wimax_shapes(cls, Z):
    h = synth.wimax_code(cls, Z)
    _, _, llr = _frames(h, Z, 37, 2.0, Z)
    got, want = _decode_f32_both(h, Z, llr, max_iter=8, alpha=0.8125, early_term=True)
    gp, wp = _assert_f32_parity(got, want)
    assert np.array_equal(gp, wp)


@pytest.mark.parametrize("F", [1, 2, 5, 7, 13])
def test_ragged_batches(F):
    h = synth.wifi_code("3/4", 81)
    _, _, llr = _frames(h, 81, F, 1.0, 100 + F)
    got, want = _decode_f32_both(h, 81, llr, max_iter=10, alpha=0.75, early_term=True)
    _assert_f32_parity(got, want)


def test_empty_batch_is_noop():
    h = synth.wifi_code("1/2", 27)
    llr = torch.zeros((0, 648), dtype=torch.float32, device=DEV)
    bits, post, iters, ok = P.ldpc_decode_f32(h, 27, llr)
    assert bits.shape == (0, 648) and iters.shape == (0,)


def test_edge_values():
    # zeros, negative zeros, huge and tiny magnitudes, all-zero frames
    h = synth.wifi_code("2/3", 27)
    rng = np.random.default_rng(5)
    llr = rng.normal(0.5, 2.0, (24, 648)).astype(np.float32)
    llr[0] = 0.0
    llr[1] = -0.0
    llr[2, ::3] = 0.0
    llr[3, ::5] = -0.0
    llr[4] *= 1e30
    llr[5] *= 1e-30
    llr[6, ::2] = np.float32(3.0e38)
    llr[7] = np.where(rng.random(648) < 0.5, 1.0, -1.0)
    for et in (True, False):
        got, want = _decode_f32_both(h, 27, llr, max_iter=6, alpha=0.75, early_term=et)
        _assert_f32_parity(got, want)


@pytest.mark.parametrize("max_iter", [1, 2, 25])
def test_iteration_limits(max_iter):
    h = synth.wifi_code("1/2", 81)
    _, _, llr = _frames(h, 81, 40, 1.2, 3)
    got, want = _decode_f32_both(h, 81, llr, max_iter=max_iter, alpha=0.75, early_term=True)
    _assert_f32_parity(got, want)


def test_learned_weight_table():
    h = synth.wifi_code("1/2", 81)
    _, _, llr = _frames(h, 81, 60, 1.5, 9)
    rng = np.random.default_rng(2)
    w = rng.uniform(0.4, 1.1, (10,) + h.shape).astype(np.float32)
    got = P.ldpc_decode_f32(h, 81, _gpu(llr), max_iter=10, early_term=True, w=_gpu(w))
    torch.cuda.synchronize()
    want = oracle.decode_f32(h, 81, llr, max_iter=10, early_term=True, w=w)
    gp, wp = _assert_f32_parity(got, want)
    assert np.array_equal(gp, wp)


def test_noiseless_decodes_in_one_iteration():
    h = synth.wifi_code("5/6", 81)
    _, K, _ = synth.code_dims(h, 81)
    cw = oracle.encode(h, 81, synth.info_bits(64, K, 4))
    llr = ((1.0 - 2.0 * cw) * 3.0).astype(np.float32)
    bits, _, iters, ok = P.ldpc_decode_f32(h, 81, _gpu(llr))
    assert np.array_equal(bits.cpu().numpy(), cw)
    assert (iters.cpu().numpy() == 1).all() and (ok.cpu().numpy() == 1).all()


def test_deterministic():
    h = synth.wifi_code("1/2", 81)
    _, _, llr = _frames(h, 81, 300, 1.5, 11)
    x = _gpu(llr)
    a = P.ldpc_decode_f32(h, 81, x, early_term=True)
    b = P.ldpc_decode_f32(h, 81, x, early_term=True)
    for u, v in zip(a, b):
        assert torch.equal(u, v)


# ---------------------------------------------------------------- fixed point

def _assert_exact(got, want):
    for name, g, w in zip(("bits", "post", "iters", "ok"), got, want):
        g = g.cpu().numpy()
        assert np.array_equal(g, w), f"{name} differs"


def test_register_fitted_layouts():
    # the WiMAX-shaped rate-1/2 code at Z = 96 is where untuned and weighted
    # layouts are re-derived from the kernels' registers (FP32 weight table:
    # 6 block rows hoisted at three waves; int8 table and the packed int8
    # default: 3): bit-exact, with early termination on and off
    h = synth.wimax_code("1/2", 96)
    Z, T = 96, 10
    _, _, llr = oracle.llr_frames(h, Z, 40, 1.8, 91)
    q = oracle.quantize_i8(llr)
    rng = np.random.default_rng(92)
    w = (0.75 + 0.1 * rng.uniform(-1, 1, (T,) + h.shape)).astype(np.float32)
    wt = rng.integers(8, 17, (T,) + h.shape).astype(np.uint8)
    for et in (True, False):
        got = P.ldpc_decode_f32(h, Z, _gpu(llr), max_iter=T, early_term=et, w=_gpu(w))
        torch.cuda.synchronize()
        _assert_f32_parity(got, oracle.decode_f32(h, Z, llr, max_iter=T, early_term=et, w=w))
        got = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=T, wq_table=_gpu(wt), early_term=et)
        torch.cuda.synchronize()
        _assert_exact(got, oracle.decode_i8(h, Z, q, max_iter=T, wq_table=wt, early_term=et))
        got = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=T, offset=1, early_term=et)
        torch.cuda.synchronize()
        _assert_exact(got, oracle.decode_i8(h, Z, q, max_iter=T, offset=1, early_term=et))


@pytest.mark.parametrize("rate", list(synth.WIFI_RATES))
@pytest.mark.parametrize("mode", [dict(offset=1, wq=0), dict(offset=0, wq=12), dict(offset=2, wq=0)])
def test_int8_bit_exact(rate, mode):
    h = synth.wifi_code(rate, 81)
    _, _, llr = _frames(h, 81, 97, 1.8, 21)
    q = oracle.quantize_i8(llr)
    for et in (True, False):
        got = P.ldpc_decode_i8(h, 81, _gpu(q), max_iter=10, early_term=et, **mode)
        torch.cuda.synchronize()
        want = oracle.decode_i8(h, 81, q, max_iter=10, early_term=et, **mode)
        _assert_exact(got, want)


def test_int8_weight_table_and_extremes():
    h = synth.wifi_code("1/2", 27)
    _, _, llr = _frames(h, 27, 50, 1.0, 5)
    q = oracle.quantize_i8(llr, 8.0)          # many clipped +-127 values
    q[0] = 0
    q[1] = 127
    q[2] = -127
    rng = np.random.default_rng(1)
    wt = rng.integers(0, 32, (10,) + h.shape).astype(np.uint8)
    got = P.ldpc_decode_i8(h, 27, _gpu(q), max_iter=10, wq_table=_gpu(wt), early_term=True)
    torch.cuda.synchronize()
    want = oracle.decode_i8(h, 27, q, max_iter=10, wq_table=wt, early_term=True)
    _assert_exact(got, want)


@pytest.mark.parametrize("cls,Z", [("1/2", 24), ("2/3B", 60), ("5/6", 96), ("3/4A", 44)])
def test_int8_wimax(cls, Z):
    h = synth.wimax_code(cls, Z)
    _, _, llr = _frames(h, Z, 29, 2.5, 3)
    q = oracle.quantize_i8(llr)
    got = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=10, offset=1, early_term=True)
    torch.cuda.synchronize()
    _assert_exact(got, oracle.decode_i8(h, Z, q, max_iter=10, offset=1, early_term=True))


@pytest.mark.parametrize("rate", ["1/2", "5/6"])
def test_autotuned_layouts_stay_exact(rate):
    # The autotuner may pick any layout (frames per workgroup and thread,
    # register variant); results must not change.
    h = synth.wifi_code(rate, 81)
    _, _, llr = _frames(h, 81, 211, 1.5, 17)
    q = oracle.quantize_i8(llr)
    try:
        for path in ("f32", "i8"):
            cfg = P.ldpc_autotune_decode(h, 81, path=path, max_iter=10, F=2048)
            assert cfg["G"] >= 1 and cfg["KF"] >= 1 and cfg["ms"] > 0
        got = P.ldpc_decode_f32(h, 81, _gpu(llr), max_iter=10, early_term=True)
        torch.cuda.synchronize()
        gp, wp = _assert_f32_parity(got, oracle.decode_f32(h, 81, llr, max_iter=10, early_term=True))
        assert np.array_equal(gp, wp)
        got = P.ldpc_decode_i8(h, 81, _gpu(q), max_iter=10, offset=1, early_term=True)
        torch.cuda.synchronize()
        _assert_exact(got, oracle.decode_i8(h, 81, q, max_iter=10, offset=1, early_term=True))
    finally:
        P.ldpc_cache_clear()


# ------------------------------------------------------- full-size, sampled

@pytest.mark.parametrize("rate", list(synth.WIFI_RATES))
def test_full_batch_sampled(rate):
    # The benchmark's launch: 2^16 frames of a Z = 81 code at a fixed 10
    # iterations. The oracle checks a random sample of the frames.
    h = synth.wifi_code(rate, 81)
    N, K, _ = synth.code_dims(h, 81)
    F = 1 << 16
    seed = 42
    info = P.ldpc_random_bits(seed, F, K)
    cw = P.ldpc_encode(h, 81, info)
    s2 = synth.sigma2_from_ebn0(2.0, K / N)
    llr = P.ldpc_awgn_llr(seed, cw, np.sqrt(s2), 2.0 / s2)
    bits, post, iters, ok = P.ldpc_decode_f32(h, 81, llr, max_iter=10, early_term=False)
    q = P.ldpc_quantize_i8(llr)
    bq, pq, iq, oq = P.ldpc_decode_i8(h, 81, q, max_iter=10, offset=1, early_term=False)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(F, 48, replace=False))
    idx = np.concatenate([idx, [0, F - 1]])
    tidx = torch.from_numpy(idx).to(DEV)
    l_s = llr[tidx].cpu().numpy()
    want = oracle.decode_f32(h, 81, l_s, max_iter=10, early_term=False)
    got = tuple(t[tidx] for t in (bits, post, iters, ok))
    gp, wp = _assert_f32_parity(got, want)
    assert np.array_equal(gp, wp)
    q_s = q[tidx].cpu().numpy()
    assert np.array_equal(q_s, oracle.quantize_i8(l_s))
    want_q = oracle.decode_i8(h, 81, q_s, max_iter=10, offset=1, early_term=False)
    _assert_exact(tuple(t[tidx] for t in (bq, pq, iq, oq)), want_q)


@pytest.mark.parametrize("rate,Z", [("1/2", 27), ("5/6", 81), ("2/3", 81)])
def test_precompiled_kernels_match_oracle(rate, Z, monkeypatch):
    # LDPC_JIT=0 selects the precompiled per-shape kernels instead of the
    # run-time specialised ones (the library reads the switch on every call)
    monkeypatch.setenv("LDPC_JIT", "0")
    h = synth.wifi_code(rate, Z)
    _, _, llr = _frames(h, Z, 77, 2.5 if rate == "1/2" else 4.0, 23)
    for et in (True, False):
        got, want = _decode_f32_both(h, Z, llr, max_iter=8, alpha=0.75, early_term=et)
        gp, wp = _assert_f32_parity(got, want)
        assert np.array_equal(gp, wp)
        q = oracle.quantize_i8(llr)
        gb, gpost, gi, go = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=8, offset=1, early_term=et)
        wb, wpost, wi, wo = oracle.decode_i8(h, Z, q, max_iter=8, offset=1, early_term=et)
        torch.cuda.synchronize()
        assert np.array_equal(gb.cpu().numpy(), wb) and np.array_equal(gpost.cpu().numpy(), wpost)
        assert np.array_equal(gi.cpu().numpy(), wi) and np.array_equal(go.cpu().numpy(), wo)


@pytest.mark.parametrize("Mb,heavy", [(15, 15), (16, 16)])
def test_int8_column_weight_boundary(Mb, heavy):
    # Column weight 15 keeps every fixed-point value below 2048 (exact in
    # FP16: the two-frames-per-lane kernel); weight 16 must fall back to one
    # frame per lane. Both must be bit-exact against the oracle.
    Z = 32
    h = synth.heavy_column_code(Mb, heavy, Z, 50 + Mb)
    q = oracle.quantize_i8(synth.zero_word_llr(24 * Z, 37, 60 + Mb))
    try:
        for et in (True, False):
            got = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=12, offset=1, early_term=et)
            torch.cuda.synchronize()
            _assert_exact(got, oracle.decode_i8(h, Z, q, max_iter=12, offset=1, early_term=et))
        # untuned, the weight-15 code ran two frames per lane; the tuner may
        # choose either kernel for it, never the packed one for weight 16
        cfg = P.ldpc_autotune_decode(h, Z, path="i8", max_iter=4, F=1024)
        if heavy > 15:
            assert cfg["h2"] == 0
        got = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=12, offset=1, early_term=True)
        torch.cuda.synchronize()
        _assert_exact(got, oracle.decode_i8(h, Z, q, max_iter=12, offset=1, early_term=True))
    finally:
        P.ldpc_cache_clear()


@pytest.mark.parametrize("Mb,deg0", [(16, 18), (6, 26)])
def test_decoders_at_size_limits(Mb, deg0):
    # 32 block columns and Z = 256 (N = 8192, one frame per workgroup), with
    # 16 block rows or a block row of the maximum check degree 26; 5 frames
    Z = 256
    h = synth.limit_code(Mb, 32, Z, deg0, 6, 70 + Mb)
    _, _, llr = oracle.llr_frames(h, Z, 5, 2.0 if Mb == 16 else 4.0, 80 + Mb)
    q = oracle.quantize_i8(llr)
    for et in (True, False):
        got = P.ldpc_decode_f32(h, Z, _gpu(llr), max_iter=6, alpha=0.75, early_term=et)
        torch.cuda.synchronize()
        _assert_f32_parity(got, oracle.decode_f32(h, Z, llr, max_iter=6, alpha=0.75, early_term=et))
        got = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=6, offset=1, early_term=et)
        torch.cuda.synchronize()
        _assert_exact(got, oracle.decode_i8(h, Z, q, max_iter=6, offset=1, early_term=et))
