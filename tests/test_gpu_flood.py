"""GPU parity of the flooding (two-phase) min-sum decoder against the
oracle's flooding decoder: FP32 hard bits, posteriors, iteration counts and
ok flags identical; fixed point bit-exact."""
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


def _f32(h, Z, llr, **kw):
    got = [t.cpu().numpy() for t in P.ldpc_decode_flood_f32(h, Z, _gpu(llr), **kw)]
    want = oracle.decode_flood_f32(h, Z, llr, **kw)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    return got


def _i8(h, Z, q, **kw):
    got = [t.cpu().numpy() for t in P.ldpc_decode_flood_i8(h, Z, _gpu(q), **kw)]
    want = oracle.decode_flood_i8(h, Z, q, **kw)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    return got


@pytest.mark.parametrize("et", [True, False])
def test_flood_z27_rate_half(et):
    h = synth.wifi_code("1/2", 27)
    _, _, llr = oracle.llr_frames(h, 27, 1000, 2.0, 1)
    _f32(h, 27, llr, max_iter=10, alpha=0.75, early_term=et)


@pytest.mark.parametrize("rate", list(synth.WIFI_RATES))
def test_flood_z81_all_rates(rate):
    h = synth.wifi_code(rate, 81)
    eb = {"1/2": 1.75, "2/3": 2.5, "3/4": 3.0, "5/6": 3.75}[rate]
    _, _, llr = oracle.llr_frames(h, 81, 131, eb, 5)
    _f32(h, 81, llr, max_iter=12, alpha=0.75, early_term=True)
    q = oracle.quantize_i8(llr)
    _i8(h, 81, q, max_iter=12, offset=1, early_term=True)
    _i8(h, 81, q, max_iter=6, wq=12, early_term=False)


@pytest.mark.parametrize("cls,Z", [("1/2", 96), ("2/3B", 44), ("5/6", 24)])
def test_flood_wimax_shapes(cls, Z):
    h = synth.wimax_code(cls, Z)
    _, _, llr = oracle.llr_frames(h, Z, 37, 2.5, 9)
    _f32(h, Z, llr, max_iter=10, alpha=0.75, early_term=True)
    _i8(h, Z, oracle.quantize_i8(llr), max_iter=10, offset=1, early_term=True)


@pytest.mark.parametrize("F", [1, 2, 5, 7])
def test_flood_ragged(F):
    h = synth.wifi_code("3/4", 27)
    _, _, llr = oracle.llr_frames(h, 27, F, 3.0, F)
    _f32(h, 27, llr, max_iter=8, alpha=0.75, early_term=True)


def test_flood_empty_and_noiseless():
    h = synth.wifi_code("2/3", 27)
    e = P.ldpc_decode_flood_f32(h, 27, torch.zeros((0, 648), dtype=torch.float32, device=DEV))
    assert e[0].shape == (0, 648)
    _, K, _ = synth.code_dims(h, 27)
    cw = oracle.encode(h, 27, synth.info_bits(9, K, seed=2))
    llr = ((1.0 - 2.0 * cw) * 3.0).astype(np.float32)
    bits, _, iters, ok = _f32(h, 27, llr, max_iter=10)
    assert np.array_equal(bits, cw) and (iters == 1).all() and ok.all()


def test_flood_full_batch_sampled():
    h = synth.wifi_code("1/2", 81)
    F = 1 << 16
    info = P.ldpc_code_info(h, 81)
    s2 = synth.sigma2_from_ebn0(2.0, info["K"] / info["N"])
    cw = P.ldpc_encode(h, 81, P.ldpc_random_bits(31, F, info["K"], device=DEV))
    llr = P.ldpc_awgn_llr(32, cw, float(np.sqrt(s2)), 2.0 / s2)
    bits, post, iters, ok = P.ldpc_decode_flood_f32(h, 81, llr, max_iter=10, early_term=False)
    torch.cuda.synchronize()
    idx = np.random.default_rng(0).choice(F, 30, replace=False)
    lh = llr[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    wb, wp, wi, wo = oracle.decode_flood_f32(h, 81, lh, max_iter=10, early_term=False)
    sel = torch.from_numpy(idx).to(DEV)
    assert np.array_equal(bits[sel].cpu().numpy(), wb) and np.array_equal(post[sel].cpu().numpy(), wp)
    assert np.array_equal(iters[sel].cpu().numpy(), wi) and np.array_equal(ok[sel].cpu().numpy(), wo)
