"""GPU parity of the paper's int16 Q_B-bit fixed-point decoder (wrap-around
and saturating) and its quantiser against the oracle: bit-exact."""
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


def _both(h, Z, q, **kw):
    got = [t.cpu().numpy() for t in P.ldpc_decode_q16(h, Z, _gpu(q), **kw)]
    want = oracle.decode_q16(h, Z, q, **kw)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    return got


def test_quantizer_bit_exact():
    x = np.random.default_rng(1).normal(0, 25, 100003).astype(np.float32)
    x[:6] = [0.5 / 16, 1.5 / 16, -2.5 / 16, 1e9, -1e9, -0.0]
    got = P.ldpc_quantize_q16(_gpu(x)).cpu().numpy()
    assert np.array_equal(got, oracle.quantize_q16(x))


@pytest.mark.parametrize("rate", list(synth.WIFI_RATES))
@pytest.mark.parametrize("wrap", [True, False])
def test_q16_z81(rate, wrap):
    h = synth.wifi_code(rate, 81)
    eb = {"1/2": 1.75, "2/3": 2.5, "3/4": 3.0, "5/6": 3.75}[rate]
    _, _, llr = oracle.llr_frames(h, 81, 97, eb, 3)
    q = oracle.quantize_q16(llr)
    _both(h, 81, q, max_iter=10, wq=12, wrap=wrap, early_term=True)
    _both(h, 81, q, max_iter=7, wq=16, wrap=wrap, early_term=False)


@pytest.mark.parametrize("wrap", [True, False])
def test_q16_overflow_beyond_16_bits(wrap):
    # values near the int16 limit: wrap-around and saturation take effect
    h = synth.wifi_code("1/2", 27)
    _, cw, llr = oracle.llr_frames(h, 27, 64, 3.0, 4)
    q = np.clip(np.rint(llr * 2000), -32767, 32767).astype(np.int16)
    _both(h, 27, q, max_iter=8, wq=31, wrap=wrap, early_term=False)
    _both(h, 27, q, max_iter=8, wq=12, wrap=wrap, early_term=True)


@pytest.mark.parametrize("cls,Z", [("1/2", 96), ("3/4A", 52)])
def test_q16_wimax(cls, Z):
    h = synth.wimax_code(cls, Z)
    _, _, llr = oracle.llr_frames(h, Z, 41, 2.5, 6)
    _both(h, Z, oracle.quantize_q16(llr), max_iter=10, wq=12, wrap=True, early_term=True)


@pytest.mark.parametrize("F", [1, 3, 4])
def test_q16_ragged(F):
    h = synth.wifi_code("5/6", 27)
    _, _, llr = oracle.llr_frames(h, 27, F, 4.0, 10 + F)
    _both(h, 27, oracle.quantize_q16(llr), max_iter=6, wq=12, wrap=True, early_term=True)
