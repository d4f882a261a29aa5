"""GPU parity of the evaluation pipeline: per-frame channel noise levels,
decoding statistics, and the fallback re-decode of failed frames."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2306_12063_amd as P
from paper_2306_12063_amd import learned

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def test_awgn_per_frame_sigma():
    F, N, seed = 12, 648, 5
    cw = (np.arange(F * N).reshape(F, N) % 5 == 1).astype(np.uint8)
    e = np.linspace(0.5, 5.0, F)
    s2 = 1.0 / (2 * 0.5 * 10 ** (e / 10))
    sig, sc = np.sqrt(s2).astype(np.float32), (2 / s2).astype(np.float32)
    got = P.ldpc_awgn_llr(seed, _gpu(cw), _gpu(sig), _gpu(sc)).cpu().numpy()
    z = oracle.frame_noise(seed, F, N).astype(np.float32)
    for f in range(F):
        want = oracle.channel(cw[f:f + 1], z[f:f + 1], sig[f], sc[f])[0]
        np.testing.assert_allclose(got[f], want, rtol=2e-6, atol=1e-5 * float(sc[f]) * float(sig[f]))


def test_frame_stats_counts():
    rng = np.random.default_rng(0)
    F, N, K = 300, 1944, 972
    info = rng.integers(0, 2, (F, K), dtype=np.uint8)
    bits = rng.integers(0, 2, (F, N), dtype=np.uint8)
    bits[:100, :K] = info[:100]                     # 100 error-free frames
    bits[100:110, :K] = info[100:110]
    bits[100:110, 5] ^= 1                           # one bit error each
    iters = rng.integers(1, 11, F).astype(np.int32)
    ok = (rng.random(F) < 0.7).astype(np.uint8)
    c = P.ldpc_frame_stats(_gpu(bits), _gpu(info), _gpu(iters), _gpu(ok)).cpu().numpy()
    be = (bits[:, :K] != info).sum()
    fe = np.any(bits[:, :K] != info, axis=1).sum()
    assert c.tolist() == [be, fe, iters.sum(), (ok == 0).sum()]
    c2 = P.ldpc_frame_stats(_gpu(bits), _gpu(info), counters=torch.from_numpy(c).to(DEV)).cpu().numpy()
    assert c2[0] == 2 * be and c2[1] == 2 * fe and c2[2] == iters.sum()


@pytest.mark.parametrize("rate,ebn0", [("1/2", 1.5), ("5/6", 3.5)])
def test_fallback_f32_matches_direct_decode(rate, ebn0):
    h = synth.wifi_code(rate, 81)
    _, cw, llr = oracle.llr_frames(h, 81, 97, ebn0, 3)
    d = _gpu(llr)
    bits, post, iters, ok = P.ldpc_decode_f32(h, 81, d, max_iter=2, alpha=0.75, early_term=True)
    first = [t.clone() for t in (bits, post, iters, ok)]
    P.ldpc_fallback_f32(h, 81, d, bits, iters, ok, post=post, max_iter=20, alpha=0.75)
    torch.cuda.synchronize()
    ok1 = first[3].cpu().numpy()
    assert (ok1 == 0).sum() >= 5                       # the test exercises the fallback
    wb, wp, wi, wo = oracle.decode_f32(h, 81, llr, max_iter=20, alpha=0.75, early_term=True)
    fail = ok1 == 0
    g = [t.cpu().numpy() for t in (bits, post, iters, ok)]
    f0 = [t.cpu().numpy() for t in first]
    for k, want in enumerate((wb, wp, wi, wo)):
        assert np.array_equal(g[k][fail], want[fail])
        assert np.array_equal(g[k][~fail], f0[k][~fail])


def test_fallback_i8_and_no_failures():
    h = synth.wifi_code("2/3", 27)
    _, cw, llr = oracle.llr_frames(h, 27, 60, 2.0, 9)
    q = oracle.quantize_i8(llr)
    dq = _gpu(q)
    bits, post, iters, ok = P.ldpc_decode_i8(h, 27, dq, max_iter=1, offset=1, early_term=True)
    ok1 = ok.cpu().numpy().copy()
    b1 = bits.cpu().numpy().copy()
    P.ldpc_fallback_i8(h, 27, dq, bits, iters, ok, post=post, max_iter=20, wq=12)
    torch.cuda.synchronize()
    wb, wp, wi, wo = oracle.decode_i8(h, 27, q, max_iter=20, offset=0, wq=12, early_term=True)
    fail = ok1 == 0
    assert fail.sum() >= 5
    assert np.array_equal(bits.cpu().numpy()[fail], wb[fail])
    assert np.array_equal(post.cpu().numpy()[fail], wp[fail])
    assert np.array_equal(iters.cpu().numpy()[fail], wi[fail])
    assert np.array_equal(bits.cpu().numpy()[~fail], b1[~fail])
    # noiseless frames: nothing fails, nothing changes
    cw0 = oracle.encode(h, 27, synth.info_bits(20, 16 * 27, 1))
    l0 = _gpu(((1.0 - 2.0 * cw0) * 4).astype(np.float32))
    b, p, i, o = P.ldpc_decode_f32(h, 27, l0)
    before = [t.clone() for t in (b, p, i, o)]
    P.ldpc_fallback_f32(h, 27, l0, b, i, o, post=p)
    for x, y in zip((b, p, i, o), before):
        assert torch.equal(x, y)


def test_learned_pipeline_runs():
    h = synth.wifi_code("1/2", 27)
    w, hist = learned.train(h, 27, T=10, frames=4 * 1024, batch=1024, seed=3)
    assert w.shape == (10,) + h.shape and torch.isfinite(w).all() and len(hist) == 4
    res = learned.sweep(h, 27, learned.decoders(h, 27, w), [2.0, 4.0], frames=4096, chunk=2048)
    for name, pts in res.items():
        assert len(pts) == 2 and all(0.0 <= p["fer"] <= 1.0 for p in pts)
        assert pts[1]["fer"] <= pts[0]["fer"] + 0.02
        assert pts[0]["fer_fallback"] <= pts[0]["fer"] + 1e-12
