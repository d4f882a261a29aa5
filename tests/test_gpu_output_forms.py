"""Output paths that the benchmark workloads never take. The decoders write
hard bits four per 32-bit store where N is a multiple of 4 and the word is
4-byte aligned, and one byte per store otherwise. These tests force the byte
paths (a code of odd length, a bits buffer one byte off alignment, batch
frames at offsets that are not multiples of 4) and hold them to the oracle
and to the aligned path: bits, iteration counts and ok flags exactly equal,
FP32 posteriors within 1e-5 relative, fixed point bit-exact, and no byte
outside a frame written."""
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


def _odd_code():
    # 4 x 9 base matrix at Z = 7: N = 63, K = 35 (encodable, dual-diagonal parity part)
    return synth.limit_code(4, 9, 7, 6, 4, 91), 7


def _check_f32(got, want):
    gb, gp, gi, go = (t.cpu().numpy() for t in got)
    wb, wp, wi, wo = want
    assert np.array_equal(gi, wi) and np.array_equal(go, wo)
    assert np.array_equal(gb, wb)
    np.testing.assert_allclose(gp, wp, rtol=1e-5, atol=0)


def _check_i8(got, want):
    for g, w in zip(got, want):
        assert np.array_equal(g.cpu().numpy(), w)


@pytest.mark.parametrize("et", [True, False])
def test_odd_length_code(et):
    h, Z = _odd_code()
    assert (h.shape[1] * Z) % 4 != 0
    _, _, llr = oracle.llr_frames(h, Z, 37, 2.5, 5)
    q = oracle.quantize_i8(llr)
    try:
        got = P.ldpc_decode_f32(h, Z, _gpu(llr), max_iter=8, alpha=0.75, early_term=et)
        torch.cuda.synchronize()
        _check_f32(got, oracle.decode_f32(h, Z, llr, max_iter=8, alpha=0.75, early_term=et))
        want = oracle.decode_i8(h, Z, q, max_iter=8, offset=1, early_term=et)
        # both fixed-point kernels: one frame per lane and two per lane
        lays = P.ldpc_decode_layouts(h, Z, "i8")
        picked = [next(l for l in lays if l["h2"] == k) for k in (0, 1)]
        for lay in picked:
            P.ldpc_set_decode_layout(h, Z, "i8", lay)
            got = P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=8, offset=1, early_term=et)
            torch.cuda.synchronize()
            _check_i8(got, want)
    finally:
        P.ldpc_cache_clear()


@pytest.mark.parametrize("path", ["f32", "i8"])
@pytest.mark.parametrize("et", [True, False])
def test_misaligned_bits_buffer(path, et):
    h, Z = synth.wifi_code("1/2", 27), 27
    F, N = 50, 24 * 27
    _, _, llr = oracle.llr_frames(h, Z, F, 2.0, 9)
    if path == "f32":
        run = lambda bits: P.ldpc_decode_f32(h, Z, _gpu(llr), max_iter=10, early_term=et, bits=bits)
        want = oracle.decode_f32(h, Z, llr, max_iter=10, alpha=0.75, early_term=et)
    else:
        q = oracle.quantize_i8(llr)
        run = lambda bits: P.ldpc_decode_i8(h, Z, _gpu(q), max_iter=10, offset=1, early_term=et, bits=bits)
        want = oracle.decode_i8(h, Z, q, max_iter=10, offset=1, early_term=et)
    buf = torch.full((F * N + 8,), 0xAA, dtype=torch.uint8, device=DEV)
    off = buf[1:1 + F * N].view(F, N)         # one byte past a 4-byte boundary
    assert off.data_ptr() % 4 == 1
    got_off = run(off)
    got_al = run(None)
    torch.cuda.synchronize()
    assert np.array_equal(off.cpu().numpy(), got_al[0].cpu().numpy())
    assert np.array_equal(off.cpu().numpy(), want[0])
    b = buf.cpu().numpy()
    assert b[0] == 0xAA and np.all(b[1 + F * N:] == 0xAA)   # nothing written outside


@pytest.mark.parametrize("path", ["f32", "i8"])
@pytest.mark.parametrize("et", [True, False])
def test_batch_frames_at_unaligned_offsets(path, et):
    # a small set with the odd-length code among WiMAX-shaped ones; frame f
    # starts (f mod 3) elements after the previous frame ends
    oh, oZ = _odd_code()
    codes = [(synth.wimax_code("1/2", 24), 24), (synth.wimax_code("5/6", 28), 28), (oh, oZ)]
    cs = P.Codeset(codes)
    F = 90
    rng = np.random.default_rng(4)
    cid = rng.integers(0, len(codes), F).astype(np.int32)
    Ns = np.array([h.shape[1] * Z for h, Z in codes])
    off = np.zeros(F, np.int64)
    end = 0
    for f in range(F):
        off[f] = end + f % 3
        end = off[f] + Ns[cid[f]]
    total = int(end)
    assert np.any(off % 4 != 0)
    llr = np.zeros(total, np.float32)
    per = {}
    for c in range(len(codes)):
        idx = np.flatnonzero(cid == c)
        h, Z = codes[c]
        _, _, l = oracle.llr_frames(h, Z, len(idx), 2.5, 40 + c)
        for k, f in enumerate(idx):
            llr[off[f]:off[f] + Ns[c]] = l[k]
        per[c] = (idx, l)
    d = lambda x: torch.from_numpy(x).to(DEV)
    bits = torch.full((total,), 0xAA, dtype=torch.uint8, device=DEV)
    if path == "f32":
        _, post, iters, ok = cs.decode_f32(d(cid), d(off), d(llr), max_iter=8, alpha=0.75, early_term=et, bits=bits)
    else:
        _, post, iters, ok = cs.decode_i8(d(cid), d(off), d(oracle.quantize_i8(llr)), max_iter=8, offset=1,
                                          early_term=et, bits=bits)
    torch.cuda.synchronize()
    bits, post, iters, ok = (t.cpu().numpy() for t in (bits, post, iters, ok))
    inside = np.zeros(total, bool)
    for c, (idx, l) in per.items():
        h, Z = codes[c]
        N = Ns[c]
        if path == "f32":
            wb, wp, wi, wo = oracle.decode_f32(h, Z, l, max_iter=8, alpha=0.75, early_term=et)
        else:
            wb, wp, wi, wo = oracle.decode_i8(h, Z, oracle.quantize_i8(l), max_iter=8, offset=1, early_term=et)
        for k, f in enumerate(idx):
            inside[off[f]:off[f] + N] = True
            assert np.array_equal(bits[off[f]:off[f] + N], wb[k]), (c, f)
            if path == "f32":
                np.testing.assert_allclose(post[off[f]:off[f] + N], wp[k], rtol=1e-5, atol=0)
            else:
                assert np.array_equal(post[off[f]:off[f] + N], wp[k]), (c, f)
        assert np.array_equal(iters[idx], wi) and np.array_equal(ok[idx], wo), c
    assert np.all(bits[~inside] == 0xAA)      # the gaps between frames are untouched
