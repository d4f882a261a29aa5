"""Pins for the oracle's layered min-sum decoders (Sec. 4, eqs. 17-23).

The decoders are checked against: the check-node rule evaluated by sorting
(not by the oracle's per-edge loop), noiseless decoding, the exact
max-marginals of tree codes, exhaustive ML on tiny loopy codes, codeword-flip
and scale symmetries, and the integer/float special case."""
import numpy as np
import pytest

import oracle
import synth
from helpers import codebook, dense_h, max_marginals, ml_decode, syndrome


def _check_node_sorted(q, alpha_mag):
    """Messages of one check by sorting: every edge gets the smallest |q| of
    the others, which is min1 except at the (first) argmin, which gets min2;
    its sign is the product of the other signs, with sgn(-0) = +1."""
    a = np.abs(q)
    order = np.argsort(a, kind="stable")
    m = np.full(q.shape, a[order[0]])
    m[order[0]] = a[order[1]]
    neg = (q < 0)
    total = np.bitwise_xor.reduce(neg.astype(np.int64))
    sign = np.where((total ^ neg.astype(np.int64)) == 1, -1, 1)
    return sign, alpha_mag(m)


@pytest.mark.parametrize("d", [2, 3, 7, 20])
def test_single_check_float(d):
    # One check of degree d (Z = 1, one block row): after one iteration the
    # posterior is llr + message (eqs. 20, 23). Inputs include ties, zeros
    # and negative zeros.
    rng = np.random.default_rng(d)
    F = 200
    llr = rng.normal(0, 2, (F, d)).astype(np.float32)
    llr[::7, 0] = llr[::7, 1]                     # exact ties
    llr[::5, d - 1] = -llr[::5, 0]                # opposite-sign ties
    llr[::11, 0] = 0.0
    llr[::13, d // 2] = -0.0
    h = np.zeros((1, d), np.int16)
    alpha = np.float32(0.75)
    _, post, iters, _ = oracle.decode_f32(h, 1, llr, max_iter=1, alpha=alpha, early_term=False)
    assert (iters == 1).all()
    for f in range(F):
        sign, mag = _check_node_sorted(llr[f], lambda m: alpha * m.astype(np.float32))
        expect = llr[f] + (sign * mag).astype(np.float32)
        assert np.array_equal(post[f], expect), f


def test_single_check_negative_zero_is_positive():
    # sgn(-0.0) = +1: a -0.0 among the other edges does not flip the sign.
    h = np.zeros((1, 3), np.int16)
    llr = np.array([[-0.0, 2.0, 3.0]], np.float32)
    _, post, _, _ = oracle.decode_f32(h, 1, llr, max_iter=1, alpha=1.0, early_term=False)
    # edge 1: others are (-0.0, 3) -> min 0, sign +; edge 2: others (-0.0, 2) -> 0, +
    # edge 0: others (2, 3) -> +2
    assert post[0].tolist() == [2.0, 2.0, 3.0]
    llr = np.array([[-1e-30, 2.0, 3.0]], np.float32)
    _, post, _, _ = oracle.decode_f32(h, 1, llr, max_iter=1, alpha=1.0, early_term=False)
    assert post[0, 1] == np.float32(2.0) - np.float32(1e-30)


@pytest.mark.parametrize("mode", ["oms0", "oms1", "oms3", "wq12", "wq16", "wq31"])
def test_single_check_int(mode):
    d = 9
    rng = np.random.default_rng(42)
    F = 300
    llr = rng.integers(-127, 128, (F, d)).astype(np.int8)
    llr[::3, 2] = llr[::3, 5]
    llr[::4, 1] = 0
    h = np.zeros((1, d), np.int16)
    if mode.startswith("oms"):
        off = int(mode[3:])
        kw = dict(offset=off, wq=0)
        rule = lambda m: np.maximum(m - off, 0)
    else:
        wq = int(mode[2:])
        kw = dict(offset=0, wq=wq)
        rule = lambda m: np.minimum(127, (wq * m + 8) >> 4)
    _, post, _, _ = oracle.decode_i8(h, 1, llr, max_iter=1, early_term=False, **kw)
    for f in range(F):
        q = llr[f].astype(np.int64)
        sign, mag = _check_node_sorted(q, lambda m: rule(np.minimum(m, 127)))
        assert np.array_equal(post[f], q + sign * mag), f


def test_single_check_int_weight_table():
    # A weight table holds 1/16-step weights per (iteration, block row,
    # block column); an entry of 0 is weight 0 (no message), never the
    # offset rule, and the offset argument is unused.
    d = 6
    rng = np.random.default_rng(8)
    llr = rng.integers(-127, 128, (100, d)).astype(np.int8)
    h = np.zeros((1, d), np.int16)
    wt = np.array([[[0, 3, 16, 31, 12, 7]]], np.uint8)
    _, post, _, _ = oracle.decode_i8(h, 1, llr, max_iter=1, offset=5, wq=0, wq_table=wt, early_term=False)
    for f in range(100):
        q = llr[f].astype(np.int64)
        sign, m = _check_node_sorted(q, lambda m: np.minimum(m, 127))
        mag = np.minimum(127, (wt[0, 0].astype(np.int64) * m + 8) >> 4)
        assert np.array_equal(post[f], q + sign * mag), f
    assert (post[:, 0] == llr[:, 0]).all()


@pytest.mark.parametrize("rate", list(synth.WIFI_RATES))
def test_noiseless_one_iteration(rate):
    h = synth.wifi_code(rate, 27)
    N, K, _ = synth.code_dims(h, 27)
    info = synth.info_bits(20, K, seed=9)
    cw = oracle.encode(h, 27, info)
    llr = ((1.0 - 2.0 * cw) * 2.5).astype(np.float32)
    for dec in (oracle.decode_f32, oracle.decode_f64):
        bits, post, iters, ok = dec(h, 27, llr, max_iter=10, alpha=0.75, early_term=True)
        assert np.array_equal(bits, cw) and (iters == 1).all() and ok.all()
    q = oracle.quantize_i8(llr)
    bits, _, iters, ok = oracle.decode_i8(h, 27, q, max_iter=10, offset=1)
    assert np.array_equal(bits, cw) and (iters == 1).all() and ok.all()


def _tree_code(Z):
    # Two block rows sharing one block column: every lifted component is
    # two checks of degree 3 joined through one variable, i.e. a tree.
    return np.array([[1 % Z, 0, 2 % Z, -1, -1], [-1, -1, 1 % Z, 3 % Z, 0]], np.int16)


@pytest.mark.parametrize("Z", [1, 2, 4])
def test_tree_code_max_marginals(Z):
    # On a cycle-free graph min-sum with unit weight computes the exact
    # max-product posteriors, and its hard decision is the ML codeword.
    h = _tree_code(Z)
    H = dense_h(h, Z)
    C = codebook(H)
    rng = np.random.default_rng(Z)
    F = 64
    llr64 = rng.normal(0.8, 1.5, (F, H.shape[1]))
    _, post64, _, _ = oracle.decode_f64(h, Z, llr64, max_iter=6, alpha=1.0, early_term=False)
    exact = max_marginals(C, llr64)
    np.testing.assert_allclose(post64, exact, rtol=1e-12, atol=1e-12)
    llr32 = llr64.astype(np.float32)
    bits, post32, _, _ = oracle.decode_f32(h, Z, llr32, max_iter=6, alpha=1.0, early_term=False)
    np.testing.assert_allclose(post32, max_marginals(C, llr32.astype(np.float64)), rtol=1e-5, atol=1e-5)
    ml = ml_decode(C, llr32.astype(np.float64))
    assert np.array_equal(bits, ml)


def test_tiny_loopy_code_against_ml():
    # A small QC code with cycles: min-sum is not ML, but its decoded words
    # with a zero syndrome are codewords, and at high SNR it agrees with ML
    # on nearly every frame.
    h = np.array([[0, 1, 2, 0, -1, -1], [2, -1, 0, -1, 0, 1], [-1, 0, 1, 1, 2, 0]], np.int16)
    Z = 3
    H = dense_h(h, Z)
    C = codebook(H)
    assert len(C) >= 2
    rng = np.random.default_rng(0)
    F = 2000
    cw = C[rng.integers(0, len(C), F)]
    sigma2 = 0.25
    llr = (((1.0 - 2.0 * cw) + rng.normal(0, np.sqrt(sigma2), cw.shape)) * 2 / sigma2).astype(np.float32)
    bits, _, _, ok = oracle.decode_f32(h, Z, llr, max_iter=20, alpha=1.0, early_term=True)
    assert not syndrome(H, bits[ok == 1]).any()
    ml = ml_decode(C, llr.astype(np.float64))
    agree = np.all(bits == ml, axis=1).mean()
    assert agree >= 0.99, agree
    fer_ms = np.any(bits != cw, axis=1).mean()
    fer_ml = np.any(ml != cw, axis=1).mean()
    assert fer_ms >= fer_ml - 3 * np.sqrt(fer_ml * (1 - fer_ml) / F + 1e-12)


def _frames(rate, Z, F, ebn0, seed):
    h = synth.wifi_code(rate, Z)
    info, cw, llr = oracle.llr_frames(h, Z, F, ebn0, seed)
    return h, info, cw, llr


@pytest.mark.parametrize("dec,dt", [(oracle.decode_f32, np.float32), (oracle.decode_f64, np.float64)])
def test_codeword_flip_symmetry(dec, dt):
    # Negating the LLRs of the ones of any codeword c' negates every value the
    # decoder computes on those positions (each check has even parity over
    # c'), so L' = L * (1 - 2c') exactly, unless a zero posterior occurs.
    h, info, cw, llr = _frames("1/2", 27, 60, 1.5, 21)
    llr = llr.astype(dt)
    other = oracle.encode(h, 27, synth.info_bits(60, 12 * 27, seed=77))
    flip = (1 - 2 * other.astype(np.int64)).astype(dt)
    b1, p1, i1, o1 = dec(h, 27, llr, max_iter=10, alpha=0.75, early_term=True)
    b2, p2, i2, o2 = dec(h, 27, llr * flip, max_iter=10, alpha=0.75, early_term=True)
    clean = ~np.any(p1 == 0, axis=1)
    assert clean.sum() >= 55
    assert np.array_equal(p2[clean], (p1 * flip)[clean])
    assert np.array_equal(b2[clean], (b1 ^ other)[clean])
    assert np.array_equal(i2, i1) and np.array_equal(o2, o1)


def test_scale_invariance_unit_weight():
    # With weight 1 every operation commutes with multiplication by 2^k.
    h, info, cw, llr = _frames("3/4", 27, 40, 3.0, 5)
    for k in (-3, 4):
        s = np.float32(2.0 ** k)
        b1, p1, i1, _ = oracle.decode_f32(h, 27, llr, max_iter=10, alpha=1.0, early_term=True)
        b2, p2, i2, _ = oracle.decode_f32(h, 27, llr * s, max_iter=10, alpha=1.0, early_term=True)
        assert np.array_equal(p2, p1 * s) and np.array_equal(b1, b2) and np.array_equal(i1, i2)


@pytest.mark.parametrize("max_iter", [1, 2])
def test_int_equals_float_on_small_integers(max_iter):
    # |q| <= 10 and column weight <= 12 keep every |Q| <= 120 in the first two
    # iterations, so neither the 127 clip nor int16 saturation is reached and
    # integer arithmetic is exact: the integer decoder with weight 16/16 (or
    # offset 0) must equal the float decoder with weight 1.
    h = synth.wifi_code("1/2", 27)
    assert (h >= 0).sum(axis=0).max() <= 12
    rng = np.random.default_rng(3)
    q = rng.integers(-10, 11, (50, 24 * 27)).astype(np.int8)
    bf, pf, itf, okf = oracle.decode_f32(h, 27, q.astype(np.float32), max_iter=max_iter, alpha=1.0,
                                         early_term=False)
    for kw in (dict(offset=0, wq=0), dict(offset=0, wq=16)):
        bi, pi, iti, oki = oracle.decode_i8(h, 27, q, max_iter=max_iter, early_term=False, **kw)
        assert np.array_equal(pi.astype(np.float32), pf)
        assert np.array_equal(bi, bf) and np.array_equal(oki, okf)


def test_weight_table_of_constant_alpha_equals_plain():
    h, info, cw, llr = _frames("2/3", 27, 30, 2.0, 8)
    Mb, Nb = h.shape
    w = np.full((10, Mb, Nb), 0.75, np.float32)
    a = oracle.decode_f32(h, 27, llr, max_iter=10, alpha=0.75, early_term=True)
    b = oracle.decode_f32(h, 27, llr, max_iter=10, alpha=0.0, early_term=True, w=w)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    wq = np.full((10, Mb, Nb), 12, np.uint8)
    q = oracle.quantize_i8(llr)
    a = oracle.decode_i8(h, 27, q, max_iter=10, offset=0, wq=12)
    b = oracle.decode_i8(h, 27, q, max_iter=10, offset=0, wq=0, wq_table=wq)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_early_termination_conventions():
    h, info, cw, llr = _frames("1/2", 27, 100, 2.5, 4)
    b_et, p_et, i_et, ok_et = oracle.decode_f32(h, 27, llr, max_iter=10, early_term=True)
    b_fx, p_fx, i_fx, ok_fx = oracle.decode_f32(h, 27, llr, max_iter=10, early_term=False)
    assert (i_fx == 10).all()
    assert (i_et >= 1).all() and (i_et <= 10).all()
    H = dense_h(h, 27)
    # ok is exactly the zero-syndrome test of the returned hard bits
    assert np.array_equal(ok_et, (~syndrome(H, b_et).any(axis=1)).astype(np.uint8))
    assert np.array_equal(ok_fx, (~syndrome(H, b_fx).any(axis=1)).astype(np.uint8))
    # a frame that stopped at iteration k returns the state after k iterations
    for k in range(1, 11):
        sel = (i_et == k) & (ok_et == 1)
        if sel.any():
            _, pk, _, _ = oracle.decode_f32(h, 27, llr[sel], max_iter=k, early_term=False)
            assert np.array_equal(pk, p_et[sel])
    # bits are the hard decisions of eq. 21 (zero decodes to 1)
    assert np.array_equal(b_fx, (p_fx <= 0).astype(np.uint8))


def test_float_and_double_agree_on_decisions():
    h, info, cw, llr = _frames("5/6", 27, 200, 4.0, 12)
    b32, _, i32, _ = oracle.decode_f32(h, 27, llr, max_iter=10)
    b64, _, i64, _ = oracle.decode_f64(h, 27, llr.astype(np.float64), max_iter=10)
    assert (np.all(b32 == b64, axis=1)).mean() > 0.97
    assert (i32 == i64).mean() > 0.97


def test_decoder_rejects_bad_input():
    h = synth.wifi_code("1/2", 27)
    llr = np.zeros((1, 648), np.float32)
    with pytest.raises(oracle.OracleError):
        oracle.decode_f32(h, 27, llr, max_iter=0)
    g = np.full((2, 4), -1, np.int16)
    g[0, 0] = 0
    g[0, 1] = 0
    g[1, 2] = 0          # a check row of degree 1
    with pytest.raises(oracle.OracleError):
        oracle.decode_f32(g, 3, np.zeros((1, 12), np.float32))


def test_decoding_gain_is_monotone_in_snr():
    h = synth.wifi_code("1/2", 27)
    fers, its = [], []
    for eb in (0.5, 1.5, 2.5, 3.5):
        _, info, cw, llr = _frames("1/2", 27, 300, eb, 31)
        b, _, it, _ = oracle.decode_f32(h, 27, llr)
        fers.append(np.any(b[:, :324] != info, axis=1).mean())
        its.append(it.mean())
    assert all(a >= b for a, b in zip(fers, fers[1:]))
    assert all(a >= b for a, b in zip(its, its[1:]))
