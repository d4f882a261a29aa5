"""Statistical behaviour of the GPU decoders on seeded Monte-Carlo frames of
the Wi-Fi-shaped rate-1/2 Z = 81 code (library frame generation, early
termination, at most 10 iterations): the frame error rate and the mean
iteration count fall as Eb/N0 rises (each step by more than three binomial
standard deviations), and the fixed-point decoder (int8 LLRs at scale 4,
offset min-sum, offset 1) needs at most a few tenths of a dB more than FP32
normalised min-sum for a FER of 1e-2 (the paper puts its own fixed point at
about 0.1 dB behind, Sec. 6)."""
import math

import numpy as np
import pytest
import torch

import synth
import paper_2306_12063_amd as P
from paper_2306_12063_amd.learned import ebn0_at_fer

pytestmark = pytest.mark.gpu
DEV = "cuda"
F = 1 << 15
POINTS = (1.0, 1.5, 2.0, 2.5, 3.0)


def _sweep(path):
    h, Z = synth.wifi_code("1/2", 81), 81
    info = P.ldpc_code_info(h, Z)
    K, N = info["K"], info["N"]
    out = []
    for j, ebn0 in enumerate(POINTS):
        s2 = synth.sigma2_from_ebn0(ebn0, K / N)
        bits_in = P.ldpc_random_bits(1000 + j, F, K, device=DEV)
        llr = P.ldpc_awgn_llr(2000 + j, P.ldpc_encode(h, Z, bits_in), float(np.sqrt(s2)), 2.0 / s2)
        if path == "f32":
            bits, _, iters, ok = P.ldpc_decode_f32(h, Z, llr, max_iter=10, alpha=0.75, early_term=True,
                                                  want_post=False)
        else:
            bits, _, iters, ok = P.ldpc_decode_i8(h, Z, P.ldpc_quantize_i8(llr), max_iter=10, offset=1,
                                                 early_term=True, want_post=False)
        c = P.ldpc_frame_stats(bits, bits_in, iters, ok).cpu().numpy()
        out.append({"ebn0": ebn0, "fer": c[1] / F, "iters": c[2] / F})
    return out


def _sd(a, b):
    # standard deviation of the difference of two binomial frame error rates
    return math.sqrt(a * (1 - a) / F + b * (1 - b) / F)


@pytest.mark.parametrize("path", ["f32", "i8"])
def test_fer_and_iterations_fall_with_snr(path):
    pts = _sweep(path)
    for a, b in zip(pts, pts[1:]):
        if a["fer"] * F >= 20:     # enough errors to resolve the step: a significant fall
            assert a["fer"] - b["fer"] > 3 * _sd(a["fer"], b["fer"]), (path, a, b)
        else:                      # a handful of errors: at least no significant rise
            assert b["fer"] - a["fer"] <= 3 * _sd(a["fer"], b["fer"]) + 3 / F, (path, a, b)
        assert a["iters"] > b["iters"], (path, a, b)
    assert pts[0]["fer"] > 0.5 and pts[-1]["fer"] < 1e-3, (path, pts)


def test_fixed_point_loss_is_small():
    e32 = ebn0_at_fer(_sweep("f32"), target=1e-2)
    e8 = ebn0_at_fer(_sweep("i8"), target=1e-2)
    assert e32 is not None and e8 is not None
    assert -0.1 <= e8 - e32 <= 0.4, (e32, e8)
