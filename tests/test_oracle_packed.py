"""Pins of the oracle's packed-bit routines (Sec. 3, bitmap encoder): the
packing agrees with numpy.packbits (little bit order); the packed cyclic
shift agrees with numpy.roll, composes, inverts, and shows Fig. 1's
observation that shifts congruent modulo the word size give the same words
at rotated positions; the packed encoder is the unpacked direct encoder."""
import numpy as np
import pytest

import oracle
import synth

RNG = np.random.default_rng(5)


def _pack(bits):
    return np.packbits(bits.astype(np.uint8), axis=-1, bitorder="little")


def _unpack(b, n):
    return np.unpackbits(b, axis=-1, bitorder="little", count=n)


@pytest.mark.parametrize("Z", [1, 7, 8, 24, 27, 32, 81, 96])
def test_shift_matches_roll(Z):
    bits = RNG.integers(0, 2, (20, Z)).astype(np.uint8)
    for s in sorted({0, 1 % Z, Z // 2, Z - 1}):
        got = _unpack(oracle.shift_packed(_pack(bits), Z, s), Z)
        assert np.array_equal(got, np.roll(bits, -s, axis=1)), s     # out[r] = in[(r + s) mod Z]


def test_shift_group_laws():
    Z = 81
    bits = _pack(RNG.integers(0, 2, (10, Z)))
    for s1, s2 in ((3, 11), (40, 60), (80, 80)):
        two = oracle.shift_packed(oracle.shift_packed(bits, Z, s1), Z, s2)
        assert np.array_equal(two, oracle.shift_packed(bits, Z, (s1 + s2) % Z))
        assert np.array_equal(oracle.shift_packed(oracle.shift_packed(bits, Z, s1), Z, (Z - s1) % Z), bits)


def test_fig1_shifts_congruent_modulo_word_size():
    # Z = 24, word = 8 bits: shifting by 3, 11 and 19 yields the same bytes at
    # positions rotated by one (Fig. 1; with the code's shift direction
    # out[r] = in[r + s], byte 1 of s = 3 equals byte 0 of s = 11 and byte 2
    # of s = 19)
    Z = 24
    blocks = _pack(RNG.integers(0, 2, (50, Z)))
    o3, o11, o19 = (oracle.shift_packed(blocks, Z, s) for s in (3, 11, 19))
    assert np.array_equal(o3[:, 1], o11[:, 0]) and np.array_equal(o3[:, 1], o19[:, 2])
    for i in range(3):
        assert np.array_equal(o11[:, i], o3[:, (i + 1) % 3])
        assert np.array_equal(o19[:, i], o3[:, (i + 2) % 3])


@pytest.mark.parametrize("code", [("wifi", "1/2", 27), ("wifi", "5/6", 81), ("wimax", "2/3A", 44),
                                  ("wimax", "1/2", 96)])
def test_packed_encoder_is_the_direct_encoder(code):
    kind, rate, Z = code
    h = synth.wifi_code(rate, Z) if kind == "wifi" else synth.wimax_code(rate, Z)
    N, K, _ = synth.code_dims(h, Z)
    info = synth.info_bits(12, K, seed=Z)
    cw = oracle.encode(h, Z, info)
    got = oracle.encode_packed(h, Z, _pack(info))
    assert got.shape == (12, (N + 7) // 8)
    assert np.array_equal(got, _pack(cw))
    assert np.array_equal(_unpack(got, N)[:, :K], info)


def test_packed_rejects_bad_shift():
    with pytest.raises(Exception):
        oracle.shift_packed(np.zeros((1, 3), np.uint8), 24, 24)
