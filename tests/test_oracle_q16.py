"""Pins of the oracle's int16 Q_B-bit decoder (the paper's own fixed point,
Sec. 5: wrap-around int16 arithmetic, and its saturating twin): a single
check in closed form (the two smallest magnitudes by sorting, wrap-around by
numpy's int16 conversion), equality with the float decoder on small integers
at unit weight, equality with the int8 decoder where no int8 clip is
reachable, noiseless frames, the quantiser against numpy."""
import numpy as np
import pytest

import oracle
import synth

RNG = np.random.default_rng(77)


def _single_check(d):
    return np.zeros((1, d), np.int16)        # one check row of degree d (Z = 1)


def _closed_form(L, wq, wrap):
    L = L.astype(np.int64)
    a = np.abs(L)
    srt = np.sort(a, axis=1)
    m1, m2 = srt[:, :1], srt[:, 1:2]
    first = np.argmin(a, axis=1)[:, None] == np.arange(L.shape[1])[None, :]
    m = np.where(first, m2, m1)                      # min over the other edges
    neg_all = (np.sum(L < 0, axis=1, keepdims=True) % 2).astype(bool)
    neg = neg_all ^ (L < 0)                           # product of the other signs
    mag = (wq * m + 8) >> 4
    R = np.where(neg, -mag, mag)
    if wrap:
        return (R.astype(np.int16).astype(np.int64) + L).astype(np.int16)
    sat = lambda x: np.clip(x, -32767, 32767)
    return sat(sat(R) + L).astype(np.int16)


@pytest.mark.parametrize("wrap", [True, False])
@pytest.mark.parametrize("wq", [16, 12, 7])
def test_single_check_closed_form(wrap, wq):
    for d in (2, 3, 7, 20):
        L = RNG.integers(-32767, 32768, (200, d)).astype(np.int16)
        L[:20] = RNG.integers(-1023, 1024, (20, d))
        L[20:30] = 30000                                   # overflows when added
        L[30:40, 0] = L[30:40, 1]                          # ties of the minimum
        _, post, _, _ = oracle.decode_q16(_single_check(d), 1, L, max_iter=1, wq=wq, wrap=wrap,
                                          early_term=False)
        assert np.array_equal(post, _closed_form(L, wq, wrap)), d


def test_unit_weight_equals_float_on_small_integers():
    h = synth.wifi_code("1/2", 27)
    q = RNG.integers(-6, 7, (30, 648)).astype(np.int16)
    for wrap in (True, False):
        a = oracle.decode_q16(h, 27, q, max_iter=4, wq=16, wrap=wrap, early_term=False)
        b = oracle.decode_f64(h, 27, q.astype(np.float64), max_iter=4, alpha=1.0, early_term=False)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1].astype(np.float64), b[1])
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_equals_int8_decoder_without_clipping():
    # wq = 12 in both; |q| <= 2 and two iterations keep every |Q| below the
    # int8 decoder's clip of 127, where the two definitions coincide
    h = synth.wifi_code("2/3", 27)
    q = RNG.integers(-2, 3, (40, 648)).astype(np.int8)
    a = oracle.decode_q16(h, 27, q.astype(np.int16), max_iter=2, wq=12, early_term=False)
    b = oracle.decode_i8(h, 27, q, max_iter=2, wq=12, early_term=False)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("wrap", [True, False])
def test_noiseless_one_iteration(wrap):
    h = synth.wifi_code("3/4", 27)
    _, K, _ = synth.code_dims(h, 27)
    cw = oracle.encode(h, 27, synth.info_bits(12, K, seed=3))
    q = oracle.quantize_q16(((1.0 - 2.0 * cw) * 2.5).astype(np.float32))
    bits, _, iters, ok = oracle.decode_q16(h, 27, q, wrap=wrap)
    assert np.array_equal(bits, cw) and (iters == 1).all() and ok.all()


def test_quantizer_matches_numpy():
    x = np.concatenate([RNG.normal(0, 30, 5000), [0.5 / 16, 1.5 / 16, -2.5 / 16, 1e9, -1e9, 63.9, 64.0]])
    x = x.astype(np.float32)
    want = np.clip(np.rint(np.float32(16.0) * x), -1023, 1023).astype(np.int16)
    assert np.array_equal(oracle.quantize_q16(x), want)
    assert np.array_equal(oracle.quantize_q16(x, scale=4.0, qmax=127),
                          np.clip(np.rint(np.float32(4.0) * x), -127, 127).astype(np.int16))


def test_wrap_around_flips_signs_where_saturation_holds():
    # noiseless frames at +-30000 (far beyond Q_B = 10, so the first update
    # exceeds 16 bits): wrap-around turns the posteriors' signs and the
    # decode fails, the saturating twin keeps them and decodes
    h = synth.wifi_code("1/2", 27)
    _, K, _ = synth.code_dims(h, 27)
    cw = oracle.encode(h, 27, synth.info_bits(8, K, seed=6))
    q = ((1 - 2 * cw.astype(np.int64)) * 30000).astype(np.int16)
    bs, ps, its, os_ = oracle.decode_q16(h, 27, q, max_iter=5, wrap=False)
    assert np.array_equal(bs, cw) and os_.all() and (its == 1).all()
    assert np.abs(ps.astype(np.int64)).max() == 32767
    bw, pw, _, ow = oracle.decode_q16(h, 27, q, max_iter=5, wrap=True)
    assert not ow.any() and not np.array_equal(bw, cw)


def test_q_b_range_has_headroom_at_practical_snr():
    # Sec. 5: with Q_B = 10 inside int16 overflow is rare; at 1-6 dB with
    # weight 0.75 and 10 iterations the two arithmetics agree on every frame
    h = synth.wifi_code("1/2", 27)
    for eb in (1.0, 3.0, 6.0):
        _, _, llr = oracle.llr_frames(h, 27, 40, eb, 2)
        q = oracle.quantize_q16(llr)
        a = oracle.decode_q16(h, 27, q, max_iter=10, wrap=True, early_term=False)
        b = oracle.decode_q16(h, 27, q, max_iter=10, wrap=False, early_term=False)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert np.abs(a[1].astype(np.int64)).max() < 32767
