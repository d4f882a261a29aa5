"""The allocation-free batched decode (ldpc_decode_batch_f32_noalloc) gives
exactly what ldpc_decode_batch_f32 gives on the same frames: two calls in a
row, the second with fewer frames, so the second runs over the static
scratch the first left behind. Also its refusals: a batch beyond the
scratch, and a code set whose kernels are not loaded yet (both raised on
the host before anything is launched)."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2306_12063_amd as P

pytestmark = pytest.mark.gpu
DEV = "cuda"
MAX_FRAMES = 1 << 18


def _ragged(codes, F, ebn0, seed):
    rng = np.random.default_rng(seed)
    cid = rng.integers(0, len(codes), F).astype(np.int32)
    Ns = np.array([h.shape[1] * Z for _, Z, h in codes])
    off = np.zeros(F, np.int64)
    off[1:] = np.cumsum(Ns[cid])[:-1]
    llr = np.zeros(int(Ns[cid].sum()), np.float32)
    for c in np.unique(cid):
        idx = np.flatnonzero(cid == c)
        _, Z, h = codes[c]
        _, _, l = oracle.llr_frames(h, Z, len(idx), ebn0, seed + 17 * int(c))
        for k, f in enumerate(idx):
            llr[off[f]:off[f] + Ns[c]] = l[k]
    return cid, off, llr


@pytest.fixture(scope="module")
def wimax_set():
    codes = synth.wimax_code_set()
    return codes, P.Codeset([(h, Z) for _, Z, h in codes])


def test_noalloc_equals_batch_decode_twice(wimax_set):
    codes, cs = wimax_set
    d = lambda x: torch.from_numpy(x).to(DEV)
    for F, seed, et in ((3000, 71, True), (700, 72, False)):
        cid, off, llr = _ragged(codes, F, 2.0, seed)
        dc, do, dl = d(cid), d(off), d(llr)
        want = cs.decode_f32(dc, do, dl, max_iter=10, alpha=0.75, early_term=et)
        torch.cuda.synchronize()
        bits = torch.full((llr.size,), 7, dtype=torch.uint8, device=DEV)
        post = torch.full((llr.size,), 1234.5, dtype=torch.float32, device=DEV)
        iters = torch.full((F,), -5, dtype=torch.int32, device=DEV)
        ok = torch.full((F,), 9, dtype=torch.uint8, device=DEV)
        cs.decode_f32_noalloc(dc, do, dl, bits, iters, post=post, ok=ok, max_iter=10, alpha=0.75, early_term=et)
        torch.cuda.synchronize()
        for g, w, what in zip((bits, post, iters, ok), want, ("bits", "posteriors", "iterations", "ok")):
            assert torch.equal(g, w), (F, what)
        # and the first and last frames against the oracle directly
        for f in (0, F - 1):
            _, Z, h = codes[cid[f]]
            n = h.shape[1] * Z
            wb, wp, wi, wo = oracle.decode_f32(h, Z, llr[off[f]:off[f] + n][None, :], max_iter=10, alpha=0.75,
                                               early_term=et)
            assert np.array_equal(bits[off[f]:off[f] + n].cpu().numpy(), wb[0]), (F, f)
            assert np.array_equal(post[off[f]:off[f] + n].cpu().numpy(), wp[0]), (F, f)
            assert int(iters[f]) == int(wi[0]) and int(ok[f]) == int(wo[0]), (F, f)


def test_noalloc_refusals(wimax_set):
    codes, cs = wimax_set
    # more frames than the static scratch holds: refused on the host
    F = MAX_FRAMES + 1
    cid = torch.zeros(F, dtype=torch.int32, device=DEV)
    off = torch.zeros(F, dtype=torch.int64, device=DEV)
    llr = torch.zeros(576, dtype=torch.float32, device=DEV)
    bits = torch.zeros(576, dtype=torch.uint8, device=DEV)
    iters = torch.zeros(F, dtype=torch.int32, device=DEV)
    with pytest.raises(P.LdpcError) as e:
        cs.decode_f32_noalloc(cid, off, llr, bits, iters)
    assert e.value.code == P.LDPC_ERANGE
    # a code set no call has loaded kernels for yet: refused, nothing loaded
    fresh = P.Codeset([(synth.wifi_code("2/3", 40), 40), (synth.wifi_code("2/3", 44), 44)])
    F = 4
    cid = torch.zeros(F, dtype=torch.int32, device=DEV)
    off = torch.arange(F, dtype=torch.int64, device=DEV) * 960
    llr = torch.ones(F * 960, dtype=torch.float32, device=DEV)
    bits = torch.zeros(F * 960, dtype=torch.uint8, device=DEV)
    iters = torch.zeros(F, dtype=torch.int32, device=DEV)
    with pytest.raises(P.LdpcError) as e:
        fresh.decode_f32_noalloc(cid, off, llr, bits, iters)
    assert e.value.code == P.LDPC_ERANGE and "not loaded" in str(e.value)
    # after one ordinary decode the same call runs and agrees with it
    want = fresh.decode_f32(cid, off, llr, max_iter=5, early_term=True, want_post=False)
    fresh.decode_f32_noalloc(cid, off, llr, bits, iters, max_iter=5)
    torch.cuda.synchronize()
    assert torch.equal(bits, want[0]) and torch.equal(iters, want[2])
