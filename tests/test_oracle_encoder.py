"""Pins for the oracle's direct encoder (Sec. 2, eqs. 8-15) and the code
parameters of Tab. 1 / Tab. 2. Everything here is checked against GF(2)
linear algebra written independently in tests/helpers.py."""
import numpy as np
import pytest

import oracle
import synth
from helpers import dense_h, gf2_encode, syndrome

WIFI = [(r, 27) for r in synth.WIFI_RATES] + [("1/2", 54), ("5/6", 81)]
WIMAX = [(c, z) for c in synth.WIMAX_CLASSES for z in (24, 52, 96)]


@pytest.mark.parametrize("rate,Z", WIFI)
def test_wifi_codewords_satisfy_parity(rate, Z):
    h = synth.wifi_code(rate, Z)
    N, K, _ = synth.code_dims(h, Z)
    info = synth.info_bits(16, K, seed=3)
    cw = oracle.encode(h, Z, info)
    assert not syndrome(dense_h(h, Z), cw).any()
    assert np.array_equal(cw[:, :K], info)      # systematic, eq. 1


@pytest.mark.parametrize("cls,Z", WIMAX)
def test_wimax_codewords_satisfy_parity(cls, Z):
    h = synth.wimax_code(cls, Z)
    N, K, _ = synth.code_dims(h, Z)
    info = synth.info_bits(8, K, seed=5)
    cw = oracle.encode(h, Z, info)
    assert not syndrome(dense_h(h, Z), cw).any()


@pytest.mark.parametrize("rate,Z", [("1/2", 27), ("2/3", 27), ("3/4", 27), ("5/6", 27), ("1/2", 8)])
def test_encoder_equals_gaussian_elimination(rate, Z):
    # H2 (the expanded [h_b | H_b2']) is invertible, so the parity is unique:
    # the direct encoder must equal textbook elimination bit for bit.
    h = synth.wifi_code(rate, Z, seed=11)
    _, K, _ = synth.code_dims(h, Z)
    info = synth.info_bits(12, K, seed=2)
    assert np.array_equal(oracle.encode(h, Z, info), gf2_encode(h, Z, info))


def test_encoder_linear():
    h = synth.wifi_code("2/3", 27)
    _, K, _ = synth.code_dims(h, 27)
    a = synth.info_bits(10, K, seed=1)
    b = synth.info_bits(10, K, seed=2)
    ea, eb, eab = (oracle.encode(h, 27, x) for x in (a, b, a ^ b))
    assert np.array_equal(eab, ea ^ eb)
    assert not oracle.encode(h, 27, np.zeros_like(a)).any()


def test_eq7_parity_structure(golden):
    # The paper's example H_b2 (eq. 7) with y = 2 and h_b(y) = 80, under a
    # random 6 x 18 information part at Z = 96.
    hb2 = np.array(golden("eq7_hb2.txt"), dtype=np.int16)
    assert hb2.shape == (6, 6)
    rng = np.random.default_rng(7)
    h1 = np.where(rng.random((6, 18)) < 0.7, rng.integers(0, 96, (6, 18)), -1).astype(np.int16)
    h = np.concatenate([h1, hb2], axis=1)
    info = rng.integers(0, 2, (6, 18 * 96)).astype(np.uint8)
    cw = oracle.encode(h, 96, info)
    assert not syndrome(dense_h(h, 96), cw).any()
    assert np.array_equal(cw, gf2_encode(h, 96, info))


def _broken(h, fn):
    g = h.copy()
    fn(g)
    return g


@pytest.mark.parametrize("mutate", [
    lambda g: g.__setitem__((0, 12), 5),        # paired h_b values differ
    lambda g: g.__setitem__((5, 12), -1),       # h_b has no entry y
    lambda g: g.__setitem__((3, 12), 2),        # h_b has two middle entries
    lambda g: g.__setitem__((0, 13), 1),        # staircase shift not zero
    lambda g: g.__setitem__((4, 13), 0),        # extra block in the staircase
])
def test_encoder_rejects_wrong_structure(mutate):
    h = synth.wifi_code("1/2", 27)
    g = _broken(h, mutate)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.encode(g, 27, np.zeros((1, 12 * 27), np.uint8))
    assert ei.value.code == oracle.ORC_ESTRUCT


def test_shift_out_of_range_is_invalid():
    h = synth.wifi_code("1/2", 27)
    h[0, 0] = 27
    with pytest.raises(oracle.OracleError) as ei:
        oracle.encode(h, 27, np.zeros((1, 12 * 27), np.uint8))
    assert ei.value.code == oracle.ORC_EINVAL


def test_tab1_wifi_parameters(golden):
    # Tab. 1: N = 24 Z and K = R N for the four rates.
    for N, Z, *Ks in golden("tab1_wifi.txt"):
        assert N == 24 * Z
        for rate, K in zip(synth.WIFI_RATES, Ks):
            h = synth.wifi_code(rate, Z)
            assert synth.code_dims(h, Z)[:2] == (N, K)


def test_tab2_wimax_parameters(golden):
    # Tab. 2: N = 24 Z, K in bytes = R N / 8, for all 19 expansion factors.
    rows = golden("tab2_wimax.txt")
    assert [r[1] for r in rows] == list(synth.WIMAX_Z)
    cls_for_rate = ["1/2", "2/3A", "3/4A", "5/6"]
    for N, Z, *Kbytes in rows:
        for cls, Kb in zip(cls_for_rate, Kbytes):
            h = synth.wimax_code(cls, Z)
            n, k, _ = synth.code_dims(h, Z)
            assert (n, k) == (N, 8 * Kb)


def test_code_edges_counts():
    h = synth.wifi_code("5/6", 81)
    E, dmax = oracle.code_edges(h, 81)
    assert E == int((h >= 0).sum()) * 81
    assert dmax == 20   # the paper's maximum check degree for R = 5/6 (Sec. 4)
