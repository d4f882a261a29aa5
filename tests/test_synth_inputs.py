"""The synthetic codes that stand in for the standards' base matrices (which
are not available) have the shapes the workloads are defined by: the
802.11ax shape of Tab. 1 (24 block columns, M_b = 12/8/6/4 for rates
1/2..5/6, Z = 27/54/81) and the 802.16 shape of Tab. 2 (6 rate classes, Z
= 24..96 in steps of 4), dual-diagonal parity parts that the direct encoder
of Sec. 2 accepts, every shift in [-1, Z-1] and every check row of degree at
least 2. Host-only (ldpc_code_info needs no GPU)."""
import numpy as np
import pytest

import synth
import paper_2306_12063_amd as P


def _check_code(h, Z, Mb):
    assert h.dtype == np.int16 and h.shape == (Mb, 24)
    assert ((h == -1) | ((h >= 0) & (h < Z))).all()
    assert ((h >= 0).sum(axis=1) >= 2).all()
    info = P.ldpc_code_info(h, Z)
    assert info["N"] == 24 * Z and info["K"] == (24 - Mb) * Z and info["M"] == Mb * Z
    assert info["E"] == int((h >= 0).sum()) * Z
    assert 0 < info["enc_y"] < Mb - 1   # directly encodable: h_b has its third entry inside
    # parity part: h_b (column K_b) then the zero-shift staircase
    Kb = 24 - Mb
    hb = h[:, Kb]
    assert hb[0] >= 0 and hb[0] == hb[Mb - 1] and (hb >= 0).sum() == 3
    stair = h[:, Kb + 1:]
    for r in range(Mb):
        for c in range(Mb - 1):
            assert stair[r, c] == (0 if r in (c, c + 1) else -1)


@pytest.mark.parametrize("rate", list(synth.WIFI_RATES))
@pytest.mark.parametrize("Z", [27, 54, 81])
def test_wifi_shaped_codes(rate, Z):
    _check_code(synth.wifi_code(rate, Z), Z, synth.WIFI_RATES[rate])


def test_wimax_shaped_code_set():
    codes = synth.wimax_code_set()
    assert len(codes) == 114
    assert sorted({c for c, _, _ in codes}) == sorted(synth.WIMAX_CLASSES)
    assert sorted({Z for _, Z, _ in codes}) == list(range(24, 97, 4))
    for cls, Z, h in codes:
        _check_code(h, Z, synth.WIMAX_CLASSES[cls])
    N = np.array([h.shape[1] * Z for _, Z, h in codes])
    R = np.array([(h.shape[1] - h.shape[0]) / h.shape[1] for _, _, h in codes])
    assert N.min() == 576 and N.max() == 2304 and N.mean() == 1440
    assert abs(R.mean() - 0.6944) < 1e-3
    # classes A and B of a rate are different codes of the same shape
    for rate in ("2/3", "3/4"):
        a, b = synth.wimax_code(rate + "A", 96), synth.wimax_code(rate + "B", 96)
        assert a.shape == b.shape and not np.array_equal(a, b)


def test_codes_are_deterministic():
    assert np.array_equal(synth.wifi_code("2/3", 81), synth.wifi_code("2/3", 81))
    assert not np.array_equal(synth.wifi_code("2/3", 81, seed=1), synth.wifi_code("2/3", 81, seed=2))
