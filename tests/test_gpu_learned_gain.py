"""What the trained weights gain, by the criterion the learned decoder is
held to: learned normalised min-sum (per-iteration, per-block-row,
per-block-column weights, trained by the library's forward and adjoint
kernels on AWGN frames over the code's waterfall) must reach plain
normalised min-sum's (alpha = 0.75) frame error rate of 1e-3 at least
0.2 dB earlier, or with at least 25% fewer mean iterations, in FP32 and in
int8 with 1/16-step weights. Met on the WiMAX-shaped rate-1/2 code (Z = 96,
N = 2304). On the Wi-Fi-shaped rate-5/6 code (Z = 81, N = 1944) the gain
is smaller; it is held to a positive margin."""
import pytest
import torch

import synth
from paper_2306_12063_amd import learned

pytestmark = pytest.mark.gpu


def _compare(hbm, Z, train_range, pts):
    torch.manual_seed(0)
    r = learned.compare(hbm, Z, train_frames=1 << 20, eval_frames=1 << 18, ebn0_list=pts, seed=3,
                        train_range=train_range, lr=1e-2, lr_final=1e-3, iter_loss="early")
    assert r["loss_last"] < r["loss_first"]        # the objective went down
    return r["summary"]


def _criterion(s):
    gain = s["gain_db"]
    fewer = s.get("iter_reduction")
    return (gain is not None and gain >= 0.2) or (fewer is not None and fewer >= 0.25)


def test_learned_meets_criterion_wimax():
    sm = _compare(synth.wimax_code("1/2", 96), 96, (1.5, 3.5), [round(1.8 + 0.1 * k, 2) for k in range(14)])
    assert sm["plain_nms_f32"]["ebn0_at_fer_1e3"] is not None
    for form in ("learned_f32", "learned_i8"):
        assert _criterion(sm[form]), (form, sm[form], sm["plain_nms_f32"])


def test_learned_gains_wifi_rate56():
    sm = _compare(synth.wifi_code("5/6", 81), 81, (3.8, 5.4), [round(4.1 + 0.1 * k, 2) for k in range(11)])
    for form in ("learned_f32", "learned_i8"):
        g = sm[form]["gain_db"]
        assert g is not None and g >= 0.05, (form, sm[form], sm["plain_nms_f32"])
