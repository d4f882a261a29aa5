"""What the trained weights gain: on the WiMAX-shaped rate-1/2 code
(Z = 96, N = 2304) the learned normalised min-sum, trained by the library's
forward and adjoint kernels on AWGN frames at 1-4 dB, must reach a clearly
lower frame error rate than plain normalised min-sum (alpha = 0.75) at the
same Eb/N0, in FP32 and in int8 with 1/16-step weights."""
import numpy as np
import pytest
import torch

import synth
import paper_2306_12063_amd as P
from paper_2306_12063_amd import learned

pytestmark = pytest.mark.gpu


def test_learned_weights_lower_fer():
    hbm, Z = synth.wimax_code("1/2", 96), 96
    torch.manual_seed(0)
    w, hist = learned.train(hbm, Z, frames=1 << 19, seed=3, lr_final=1e-3)
    assert np.mean(hist[-8:]) < hist[0]            # the objective went down
    decs = learned.decoders(hbm, Z, w)
    res = learned.sweep(hbm, Z, decs, [2.25], 1 << 17, seed=11)
    plain = res["plain_nms_f32"][0]["fer"]
    f32 = res["learned_f32"][0]["fer"]
    i8 = res["learned_i8"][0]["fer"]
    # at 2.25 dB plain NMS fails on ~0.4% of the frames (~600 of 2^17)
    assert plain > 1e-3
    assert f32 < 0.5 * plain and i8 < 0.5 * plain, (plain, f32, i8)
