"""Pins for the oracle's frame generation: Philox4x32-10 against its
published known-answer vectors, the BPSK/AWGN LLR statistics of eqs. (16)-(17)
and the int8 quantiser."""
import numpy as np
import pytest

import oracle
import synth

# Known-answer vectors of Philox4x32 with 10 rounds, as published with the
# generator (Salmon et al., SC'11, Random123): (counter, key) -> output.
PHILOX_KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


@pytest.mark.parametrize("ctr,key,out", PHILOX_KAT)
def test_philox_known_answers(ctr, key, out):
    assert oracle.philox4x32_10(ctr, key).tolist() == out


def test_frame_bits_uniform_and_distinct():
    b = oracle.frame_bits(12345, 64, 1000)
    assert abs(b.mean() - 0.5) < 0.01
    assert not np.array_equal(b[0], b[1])
    b2 = oracle.frame_bits(12346, 64, 1000)
    assert (b != b2).mean() > 0.45


def test_frame_noise_is_standard_normal():
    z = oracle.frame_noise(99, 32, 4096).ravel()
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.02
    # fourth moment of N(0,1) is 3
    assert abs((z ** 4).mean() - 3.0) < 0.1


def test_llr_consistency_condition():
    # eq. 17: LLR = 2 y / sigma^2 with y ~ N(1 - 2x, sigma^2) has mean
    # (1-2x) 2/sigma^2 and variance 4/sigma^2, i.e. var = 2 |mean|.
    s2 = synth.sigma2_from_ebn0(2.0, 0.5)
    cw = np.zeros((64, 2048), np.uint8)
    cw[:, 1::2] = 1
    z = oracle.frame_noise(7, 64, 2048).astype(np.float32)
    llr = oracle.channel(cw, z, np.sqrt(s2), 2.0 / s2).astype(np.float64)
    m0, m1 = llr[:, 0::2].mean(), llr[:, 1::2].mean()
    assert m0 == pytest.approx(2 / s2, rel=0.02) and m1 == pytest.approx(-2 / s2, rel=0.02)
    v = llr[:, 0::2].var()
    assert v == pytest.approx(4 / s2, rel=0.03)
    assert v == pytest.approx(2 * abs(m0), rel=0.04)


def test_quantizer_rounds_half_to_even_and_clips():
    llr = np.array([0.125, 0.375, -0.125, -0.375, 0.625, 31.6, 40.0, -40.0, -0.0, 1e-9, 31.875], np.float32)
    q = oracle.quantize_i8(llr, 4.0)
    assert q.tolist() == [0, 2, 0, -2, 2, 126, 127, -127, 0, 0, 127]
    big = np.linspace(-1000, 1000, 10001).astype(np.float32)
    qb = oracle.quantize_i8(big, 4.0)
    assert qb.min() == -127 and qb.max() == 127
    assert np.array_equal(oracle.quantize_i8(-big, 4.0), -qb)


def test_weight_quantizer_half_to_even_and_clamps():
    # wq = clamp(rint(16 w), 0, 31) (the fixed-point decoder's 1/16-step
    # normalisation): each case written out by hand from that definition.
    cases = [
        (0.75, 12),              # alpha = 0.75 is exactly 12/16
        (0.5 / 16, 0),           # 0.5 -> 0 (half to even)
        (1.5 / 16, 2),           # 1.5 -> 2
        (2.5 / 16, 2),           # 2.5 -> 2
        (3.5 / 16, 4),           # 3.5 -> 4
        (12.5 / 16, 12),         # 12.5 -> 12
        (13.5 / 16, 14),         # 13.5 -> 14
        (30.5 / 16, 30),         # 30.5 -> 30
        (31.5 / 16, 31),         # 31.5 -> 32, clamped to 31
        (1.9375, 31),            # 31 exactly
        (2.0, 31),               # 32 -> 31
        (1e30, 31),
        (float("inf"), 31),
        (-0.01, 0),              # -0.16 -> -0 -> 0
        (-0.5, 0),               # -8 -> 0
        (-0.0, 0),
        (float("-inf"), 0),
        (float("nan"), 0),
        (0.78, 12),              # 12.48 -> 12
        (0.79, 13),              # 12.64 -> 13
    ]
    w = np.array([c[0] for c in cases], np.float32)
    assert oracle.quantize_weights(w).tolist() == [c[1] for c in cases]


def test_weight_quantizer_matches_numpy_rint():
    # numpy's rint rounds half to even as well: the finite range agrees with
    # np.clip(np.rint(16 w), 0, 31) element by element
    w = np.linspace(-1.0, 3.0, 64000).astype(np.float32)
    want = np.clip(np.rint(np.float32(16.0) * w), 0, 31).astype(np.uint8)
    got = oracle.quantize_weights(w.reshape(16, -1)).ravel()
    assert np.array_equal(got, want)
    assert oracle.quantize_weights(w.reshape(16, -1)).shape == (16, 4000)
