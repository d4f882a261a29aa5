"""GPU parity of frame generation: Philox bits and the direct encoder are
bit-exact against the oracle; Box-Muller noise and the channel LLR agree
to FP32 rounding; the int8 quantiser is bit-exact on identical input."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2306_12063_amd as P

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_random_bits_bit_exact():
    for F, K, seed in ((5, 324, 1), (17, 1620, 0xDEADBEEF12345), (3, 1, 7), (2, 129, 9)):
        got = P.ldpc_random_bits(seed, F, K).cpu().numpy()
        assert np.array_equal(got, oracle.frame_bits(seed, F, K))


@pytest.mark.parametrize("code", [("wifi", r, z) for r in synth.WIFI_RATES for z in (27, 81)] +
                         [("wimax", c, z) for c in synth.WIMAX_CLASSES for z in (24, 76, 96)])
def test_encoder_bit_exact(code):
    kind, rate, Z = code
    h = synth.wifi_code(rate, Z) if kind == "wifi" else synth.wimax_code(rate, Z)
    N, K, _ = synth.code_dims(h, Z)
    info = synth.info_bits(37, K, seed=Z)
    got = P.ldpc_encode(h, Z, torch.from_numpy(info).to(DEV)).cpu().numpy()
    assert np.array_equal(got, oracle.encode(h, Z, info))


def test_encoder_large_batch_sampled():
    h = synth.wifi_code("1/2", 81)
    N, K, _ = synth.code_dims(h, 81)
    F = 1 << 16
    info = P.ldpc_random_bits(3, F, K)
    cw = P.ldpc_encode(h, 81, info).cpu().numpy()
    inf = info.cpu().numpy()
    idx = np.random.default_rng(0).choice(F, 64, replace=False)
    assert np.array_equal(cw[idx], oracle.encode(h, 81, inf[idx]))
    assert np.array_equal(oracle.syndrome_ok(h, 81, cw[idx]), np.ones(64, np.uint8))


def test_awgn_llr_matches_oracle():
    F, N, seed = 9, 1944, 77
    cw = (np.arange(F * N).reshape(F, N) % 3 == 0).astype(np.uint8)
    s2 = synth.sigma2_from_ebn0(1.0, 0.5)
    sigma, scale = np.float32(np.sqrt(s2)), np.float32(2.0 / s2)
    got = P.ldpc_awgn_llr(seed, torch.from_numpy(cw).to(DEV), sigma, scale).cpu().numpy()
    z = oracle.frame_noise(seed, F, N)                     # double precision
    want = oracle.channel(cw, z.astype(np.float32), sigma, scale)
    # float sqrt/log/cos on the GPU vs double on the host: a few ulp of z
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=2e-6 * float(scale) * float(sigma) * 4)
    zg = (got / scale - np.where(cw == 1, -1.0, 1.0)) / sigma
    assert abs(zg.mean()) < 0.03 and abs(zg.var() - 1.0) < 0.05


def test_quantizer_bit_exact():
    rng = np.random.default_rng(0)
    x = rng.normal(0, 20, 100000).astype(np.float32)
    x[:40] = np.arange(-20, 20) * 0.125          # exact halves after scaling by 4
    x[40:44] = [1e30, -1e30, -0.0, 0.0]
    got = P.ldpc_quantize_i8(torch.from_numpy(x).to(DEV), 4.0).cpu().numpy()
    assert np.array_equal(got, oracle.quantize_i8(x, 4.0))


@pytest.mark.parametrize("Mb,deg0", [(16, 18), (6, 26)])
def test_encoder_at_size_limits(Mb, deg0):
    # 32 block columns, Z = 256 (N = 8192); 16 block rows, or a block row of
    # the maximum check degree 26
    Z = 256
    h = synth.limit_code(Mb, 32, Z, deg0, 6, 70 + Mb)
    assert (h[0] >= 0).sum() == deg0
    K = (32 - Mb) * Z
    info = synth.info_bits(3, K, 71)
    got = P.ldpc_encode(h, Z, torch.from_numpy(info).to(DEV)).cpu().numpy()
    assert np.array_equal(got, oracle.encode(h, Z, info))


def test_lds_probe_reads_what_it_claims():
    # the bandwidth probe's checksum for a small launch, recomputed: thread t
    # folds words base + u*256 (u < 8) of buf[k] = (k, 3k, 5k, 7k), base
    # starting at t and advancing by 64 modulo 2048 each round
    blocks, rounds = 2, 5
    got = P.ldpc_lds_probe(blocks, rounds).cpu().numpy()
    k = np.arange(4096, dtype=np.uint64)
    buf = np.stack([k, 3 * k, 5 * k, 7 * k], axis=1).astype(np.uint32)
    want = np.zeros(blocks * 256, np.float32)
    for t in range(256):
        a0 = a1 = np.uint32(0)
        base = t
        for _ in range(rounds):
            for u in range(8):
                v = buf[base + u * 256]
                a0 ^= v[0] ^ v[1]
                a1 ^= v[2] ^ v[3]
            base = (base + 64) & 2047
        want[t] = want[256 + t] = np.float32(a0 ^ a1)
    assert np.array_equal(got, want)


def test_weight_quantizer_bit_exact():
    # the learned-weight quantiser (1/16 steps, half to even, clamp to
    # [0, 31], NaN -> 0) against the oracle on ties, clamps, specials and a
    # dense sweep, including a ragged tail of a 256-thread block
    special = np.array([0.75, 0.5 / 16, 1.5 / 16, 2.5 / 16, 31.5 / 16, 2.0, 1e30, np.inf, -np.inf, np.nan, -0.0,
                        -0.01, 0.78, 0.79], np.float32)
    sweep = np.linspace(-1.0, 3.0, 100003).astype(np.float32)
    for w in (special, sweep, sweep[:1], np.zeros(0, np.float32)):
        got = P.ldpc_quantize_weights(torch.from_numpy(w).to(DEV)).cpu().numpy()
        assert np.array_equal(got, oracle.quantize_weights(w))
