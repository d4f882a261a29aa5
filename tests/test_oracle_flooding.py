"""Pins of the oracle's flooding (two-phase) min-sum decoders (Sec. 4,
eqs. 18-23 without layering) against things the schedule fixes: where no
two block rows share a column the layered and flooding schedules perform
the same operations; on a cycle-free graph min-sum computes the exact
max-product posteriors; noiseless frames stop after one iteration; the
codeword-flip symmetry; the integer path equals the float path on small
integers with unit weight."""
import numpy as np
import pytest

import oracle
import synth
from helpers import codebook, dense_h, max_marginals

RNG = np.random.default_rng(1234)


def _int_llr(F, N, lim):
    # integer-valued LLRs: with alpha = 0.75 every quantity stays a short
    # dyadic fraction, so double arithmetic is exact
    v = RNG.integers(-lim, lim + 1, (F, N)).astype(np.float64)
    v[v == 0] = 1.0
    return v


@pytest.mark.parametrize("h,Z", [
    (np.array([[0, 3, 1, 4, 2]], np.int16), 5),                                    # one block row
    (np.array([[0, 1, 2, -1, -1, -1], [-1, -1, -1, 1, 0, 2]], np.int16), 4),       # disjoint columns
    (np.array([[2, -1, 0, -1, 1, -1, -1], [-1, 1, -1, 0, -1, 2, 0]], np.int16), 3),
])
def test_flooding_equals_layered_when_rows_share_no_column(h, Z):
    llr = _int_llr(40, h.shape[1] * Z, 6)
    for it, et in ((1, False), (4, False), (10, True)):
        a = oracle.decode_f64(h, Z, llr, max_iter=it, alpha=0.75, early_term=et)
        b = oracle.decode_flood_f64(h, Z, llr, max_iter=it, alpha=0.75, early_term=et)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    q = np.clip(llr * 3, -127, 127).astype(np.int8)
    for wq, off in ((0, 1), (12, 0)):
        a = oracle.decode_i8(h, Z, q, max_iter=6, offset=off, wq=wq, early_term=False)
        b = oracle.decode_flood_i8(h, Z, q, max_iter=6, offset=off, wq=wq, early_term=False)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_flooding_differs_from_layered_when_rows_share_columns():
    # a control for the test above: with shared columns the schedules differ
    h = synth.wifi_code("1/2", 27)
    _, _, llr = oracle.llr_frames(h, 27, 30, 1.5, 3)
    a = oracle.decode_f32(h, 27, llr, max_iter=3, early_term=False)
    b = oracle.decode_flood_f32(h, 27, llr, max_iter=3, early_term=False)
    assert not np.array_equal(a[1], b[1])


@pytest.mark.parametrize("Z", [1, 2, 4])
def test_flooding_tree_code_max_marginals(Z):
    h = np.array([[1 % Z, 0, 2 % Z, -1, -1], [-1, -1, 1 % Z, 3 % Z, 0]], np.int16)
    H = dense_h(h, Z)
    C = codebook(H)
    llr = RNG.normal(0.8, 1.5, (64, H.shape[1]))
    _, post, _, _ = oracle.decode_flood_f64(h, Z, llr, max_iter=8, alpha=1.0, early_term=False)
    np.testing.assert_allclose(post, max_marginals(C, llr), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("rate", list(synth.WIFI_RATES))
def test_flooding_noiseless_one_iteration(rate):
    h = synth.wifi_code(rate, 27)
    _, K, _ = synth.code_dims(h, 27)
    cw = oracle.encode(h, 27, synth.info_bits(16, K, seed=4))
    llr = ((1.0 - 2.0 * cw) * 2.5).astype(np.float32)
    bits, _, iters, ok = oracle.decode_flood_f32(h, 27, llr, max_iter=10)
    assert np.array_equal(bits, cw) and (iters == 1).all() and ok.all()
    bits, _, iters, ok = oracle.decode_flood_i8(h, 27, oracle.quantize_i8(llr), max_iter=10)
    assert np.array_equal(bits, cw) and (iters == 1).all() and ok.all()


def test_flooding_codeword_flip_symmetry():
    h = synth.wifi_code("2/3", 27)
    _, _, llr = oracle.llr_frames(h, 27, 50, 2.5, 8)
    other = oracle.encode(h, 27, synth.info_bits(50, 16 * 27, seed=5))
    flip = (1 - 2 * other.astype(np.int64)).astype(np.float32)
    b1, p1, i1, o1 = oracle.decode_flood_f32(h, 27, llr, max_iter=12)
    b2, p2, i2, o2 = oracle.decode_flood_f32(h, 27, llr * flip, max_iter=12)
    clean = ~np.any(p1 == 0, axis=1)
    assert clean.sum() >= 45
    assert np.array_equal(p2[clean], (p1 * flip)[clean])
    assert np.array_equal(b2[clean], (b1 ^ other)[clean])
    assert np.array_equal(i2, i1) and np.array_equal(o2, o1)


def test_flooding_int_equals_float_on_small_integers():
    # wq = 16 is weight 1; with |q| <= 3 and two iterations no magnitude
    # reaches the int8 clip, so the integer decoder is the float one
    h = synth.wifi_code("3/4", 27)
    q = RNG.integers(-3, 4, (30, 24 * 27)).astype(np.int8)
    a = oracle.decode_flood_i8(h, 27, q, max_iter=2, wq=16, early_term=False)
    b = oracle.decode_flood_f64(h, 27, q.astype(np.float64), max_iter=2, alpha=1.0, early_term=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1].astype(np.float64), b[1])
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_layered_converges_in_fewer_iterations():
    # Sec. 4: the layered schedule reduces the iterations needed; on the same
    # frames its mean iteration count is lower and it fails no more often
    h = synth.wifi_code("1/2", 27)
    _, _, llr = oracle.llr_frames(h, 27, 300, 2.0, 12)
    _, _, il, ol = oracle.decode_f32(h, 27, llr, max_iter=20)
    _, _, iff, of = oracle.decode_flood_f32(h, 27, llr, max_iter=20)
    assert il.mean() < 0.8 * iff.mean()
    assert ol.sum() >= of.sum()


def test_flooding_rejects_bad_input():
    h = synth.wifi_code("1/2", 27)
    with pytest.raises(Exception):
        oracle.decode_flood_f32(h, 27, np.zeros((2, 100), np.float32))
    with pytest.raises(Exception):
        oracle.decode_flood_i8(h, 27, np.zeros((2, 648), np.int8), offset=200)
