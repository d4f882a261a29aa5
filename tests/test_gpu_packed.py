"""GPU parity of the packed-bit cyclic shift and packed direct encoder
(Sec. 3, bitmap encoder) against the oracle: byte-exact."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2306_12063_amd as P

pytestmark = pytest.mark.gpu
DEV = "cuda"
RNG = np.random.default_rng(9)


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _pack(bits):
    return np.packbits(bits.astype(np.uint8), axis=-1, bitorder="little")


@pytest.mark.parametrize("Z", [1, 7, 24, 27, 32, 33, 81, 96, 255, 256])
def test_shift_packed(Z):
    F = 300
    blocks = _pack(RNG.integers(0, 2, (F, Z)))
    for s in sorted({0, 1 % Z, Z // 3, Z - 1}):
        got = P.ldpc_shift_packed(_gpu(blocks), Z, s).cpu().numpy()
        assert np.array_equal(got, oracle.shift_packed(blocks, Z, s)), s


def test_shift_fig1_invariant():
    Z = 24
    blocks = _gpu(_pack(RNG.integers(0, 2, (64, Z))))
    o3, o11, o19 = (P.ldpc_shift_packed(blocks, Z, s).cpu().numpy() for s in (3, 11, 19))
    assert np.array_equal(o3[:, 1], o11[:, 0]) and np.array_equal(o3[:, 1], o19[:, 2])


@pytest.mark.parametrize("code", [("wifi", "1/2", 27), ("wifi", "2/3", 81), ("wifi", "5/6", 81),
                                  ("wimax", "1/2", 24), ("wimax", "2/3B", 44), ("wimax", "3/4A", 68),
                                  ("wimax", "5/6", 96)])
def test_encode_packed(code):
    kind, rate, Z = code
    h = synth.wifi_code(rate, Z) if kind == "wifi" else synth.wimax_code(rate, Z)
    N, K, _ = synth.code_dims(h, Z)
    F = 131
    info = synth.info_bits(F, K, seed=Z + 1)
    packed = _pack(info)
    if K % 8:
        packed[:, -1] |= np.uint8((0xff << (K % 8)) & 0xff)   # padding bits are ignored
    got = P.ldpc_encode_packed(h, Z, _gpu(packed)).cpu().numpy()
    assert np.array_equal(got, _pack(oracle.encode(h, Z, info)))
    assert np.array_equal(got, oracle.encode_packed(h, Z, packed))


def test_encode_packed_agrees_with_byte_encoder_at_scale():
    h = synth.wifi_code("1/2", 81)
    info_d = P.ldpc_code_info(h, 81)
    F = 1 << 16
    bits = P.ldpc_random_bits(3, F, info_d["K"], device=DEV)
    cw = P.ldpc_encode(h, 81, bits).cpu().numpy()
    packed = _gpu(_pack(bits.cpu().numpy()))
    got = P.ldpc_encode_packed(h, 81, packed).cpu().numpy()
    assert np.array_equal(got, _pack(cw))


@pytest.mark.parametrize("code", [("wifi", "1/2", 81), ("wimax", "5/6", 96), ("tiny", None, 3)])
def test_decode_packed_bits(code):
    # hard bits packed eight per byte equal the unpacked decode's bits, packed
    kind, rate, Z = code
    if kind == "tiny":
        h = np.array([[0, 1, 2, 0, -1], [2, -1, 0, 1, 0]], np.int16)   # N = 15: a partial last byte
        llr = RNG.normal(0.5, 2.0, (37, 15)).astype(np.float32)
    else:
        h = synth.wifi_code(rate, Z) if kind == "wifi" else synth.wimax_code(rate, Z)
        _, _, llr = oracle.llr_frames(h, Z, 37, 2.5, 4)
    for et in (True, False):
        b, _, it, ok = P.ldpc_decode_f32(h, Z, _gpu(llr), max_iter=7, early_term=et)
        bp, _, itp, okp = P.ldpc_decode_f32_packed(h, Z, _gpu(llr), max_iter=7, early_term=et)
        assert np.array_equal(bp.cpu().numpy(), _pack(b.cpu().numpy()))
        assert torch.equal(it, itp) and torch.equal(ok, okp)
        q = _gpu(oracle.quantize_i8(llr))
        b, _, it, _ = P.ldpc_decode_i8(h, Z, q, max_iter=7, offset=1, early_term=et)
        bp, post, itp, _ = P.ldpc_decode_i8_packed(h, Z, q, max_iter=7, offset=1, early_term=et, want_post=True)
        assert np.array_equal(bp.cpu().numpy(), _pack(b.cpu().numpy())) and torch.equal(it, itp)
        _, want_post, _, _ = oracle.decode_i8(h, Z, oracle.quantize_i8(llr), max_iter=7, offset=1, early_term=et)
        assert np.array_equal(post.cpu().numpy(), want_post)
