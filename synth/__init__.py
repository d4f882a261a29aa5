"""Seeded synthetic inputs: base matrices, information bits and Gaussian noise.

This module only draws random data. It holds none of the decoder's or the
encoder's arithmetic, so both the CPU oracle and the GPU path can consume
what it produces without sharing any of the method's code.

Base matrices follow the block shape of the paper's codes (Sec. 1, eq. 3 and
the example in eq. 7): an information part H_b1 of M_b x K_b circulants, a
weight-3 column h_b whose first and last entries are equal and which has one
more non-negative entry at row y, and a staircase H_b2' of zero shifts. The
standards' shift tables are not reproduced; shifts and the positions of the
information-part circulants are drawn from a splitmix64 stream instead.
Entry -1 is a zero block, s >= 0 is the identity cyclically shifted by s.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "SplitMix64", "WIFI_RATES", "WIMAX_CLASSES", "WIMAX_Z", "wifi_code", "wimax_code",
    "wimax_code_set", "info_bits", "std_normal", "sigma2_from_ebn0", "code_dims",
]

_MASK64 = (1 << 64) - 1

# Wi-Fi shaped codes (Tab. 1): 24 block columns; block rows per rate.
WIFI_RATES = {"1/2": 12, "2/3": 8, "3/4": 6, "5/6": 4}
# WiMAX shaped rate classes (Tab. 2, 802.16 naming): block rows per class.
WIMAX_CLASSES = {"1/2": 12, "2/3A": 8, "2/3B": 8, "3/4A": 6, "3/4B": 6, "5/6": 4}
# Expansion factors of the WiMAX shape: 24, 28, ..., 96 (Tab. 2).
WIMAX_Z = tuple(range(24, 97, 4))

# Probability that an information-part circulant is present, per block-row
# count (rate). The paper prints no full matrix; these densities give edge
# counts of the same order as the standard codes.
_DENSITY = {12: 0.45, 8: 0.60, 6: 0.70, 4: 0.85}
# The paper quotes a maximum check degree of 20 for the rate-5/6 Wi-Fi code
# (Sec. 4); the generator keeps every row at or below this.
_MAX_ROW_DEGREE = 20


class SplitMix64:
    """splitmix64 (Steele, Lea, Flood 2014): a 64-bit counter with a
    bijective output mix; used here only to draw base-matrix structure."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def below(self, n: int) -> int:
        """Uniform integer in [0, n) by rejection (no modulo bias)."""
        if n <= 0:
            raise ValueError("n must be positive")
        limit = (1 << 64) - ((1 << 64) % n)
        while True:
            x = self.next_u64()
            if x < limit:
                return x % n

    def unit(self) -> float:
        """Uniform float in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def _parity_part(Mb: int, Nb: int, a: int, b: int) -> np.ndarray:
    """Columns K_b .. N_b-1: h_b (a at rows 0 and M_b-1, b at row y) and the
    staircase H_b2' (zeros at (r, r) and (r+1, r))."""
    part = np.full((Mb, Mb), -1, dtype=np.int64)
    y = (Mb - 1) // 2
    part[0, 0] = a
    part[Mb - 1, 0] = a
    part[y, 0] = b
    for r in range(Mb - 1):
        part[r, 1 + r] = 0
        part[r + 1, 1 + r] = 0
    return part


def _info_structure(rng: SplitMix64, Mb: int, Kb: int, density: float) -> np.ndarray:
    """Boolean Mb x Kb presence mask with every column of weight >= 2 and every
    row degree (information part plus the parity part) <= 20."""
    # Parity-part row degrees: h_b entries (rows 0, y, Mb-1) plus staircase.
    y = (Mb - 1) // 2
    par_deg = np.zeros(Mb, dtype=np.int64)
    par_deg[[0, y, Mb - 1]] += 1
    par_deg[0] += 1
    par_deg[1:Mb - 1] += 2
    par_deg[Mb - 1] += 1
    for _attempt in range(10000):
        mask = np.zeros((Mb, Kb), dtype=bool)
        for i in range(Mb):
            for j in range(Kb):
                mask[i, j] = rng.unit() < density
        for j in range(Kb):
            while mask[:, j].sum() < 2:
                mask[rng.below(Mb), j] = True
        if np.all(mask.sum(axis=1) + par_deg <= _MAX_ROW_DEGREE):
            return mask
    raise RuntimeError("could not draw a base-matrix structure within the degree cap")


def wifi_code(rate: str, Z: int, seed: int = 1) -> np.ndarray:
    """Wi-Fi-shaped synthetic base matrix (24 block columns) at expansion Z.

    h_b is (1 at row 0, 0 at row y = floor((M_b-1)/2), 1 at row M_b-1);
    information shifts are uniform on [0, Z-1]. Returns int16 [M_b][24].
    """
    Mb = WIFI_RATES[rate]
    Nb = 24
    Kb = Nb - Mb
    if Z < 2:
        raise ValueError("Z must be at least 2")
    rng = SplitMix64(seed * 0x100000001B3 + Mb * 7919 + Z)
    mask = _info_structure(rng, Mb, Kb, _DENSITY[Mb])
    hbm = np.full((Mb, Nb), -1, dtype=np.int64)
    for i in range(Mb):
        for j in range(Kb):
            if mask[i, j]:
                hbm[i, j] = rng.below(Z)
    hbm[:, Kb:] = _parity_part(Mb, Nb, 1, 0)
    return hbm.astype(np.int16)


def _scale_shift(s96: int, Z: int, cls: str) -> int:
    # 802.16 shrinks its Z=96 model matrix to a smaller Z by floor(s*Z/96),
    # except for the 2/3A class which reduces modulo Z.
    if s96 < 0:
        return -1
    if s96 == 0:
        return 0
    if cls == "2/3A":
        return s96 % Z
    return (s96 * Z) // 96


def wimax_code(cls: str, Z: int, seed: int = 1) -> np.ndarray:
    """WiMAX-shaped synthetic base matrix for rate class `cls` at expansion Z.

    One Z=96 model matrix per class (shifts in [0, 95]) is drawn from `seed`,
    then its shifts are scaled to Z. h_b is (0 at row 0, b at row y, 0 at row
    M_b-1) with b drawn in [1, 95] before scaling. Returns int16 [M_b][24].
    """
    if cls not in WIMAX_CLASSES:
        raise ValueError(f"unknown WiMAX rate class {cls!r}")
    if Z < 2 or Z > 96:
        raise ValueError("Z must be in [2, 96]")
    Mb = WIMAX_CLASSES[cls]
    Nb = 24
    Kb = Nb - Mb
    cls_id = list(WIMAX_CLASSES).index(cls)
    rng = SplitMix64(seed * 0x9E3779B1 + 1000003 * (cls_id + 1))
    mask = _info_structure(rng, Mb, Kb, _DENSITY[Mb])
    model = np.full((Mb, Nb), -1, dtype=np.int64)
    for i in range(Mb):
        for j in range(Kb):
            if mask[i, j]:
                model[i, j] = rng.below(96)
    b96 = 1 + rng.below(95)
    model[:, Kb:] = _parity_part(Mb, Nb, 0, b96)
    hbm = np.vectorize(lambda s: _scale_shift(int(s), Z, cls))(model)
    return hbm.astype(np.int16)


def wimax_code_set(seed: int = 1):
    """All 114 WiMAX-shaped codes: 6 rate classes x 19 expansion factors.
    Returns a list of (class, Z, hbm)."""
    return [(cls, Z, wimax_code(cls, Z, seed)) for cls in WIMAX_CLASSES for Z in WIMAX_Z]


def code_dims(hbm: np.ndarray, Z: int):
    """(N, K, M) of the expanded code (Sec. 1: N = N_b Z, K = K_b Z)."""
    Mb, Nb = hbm.shape
    return Nb * Z, (Nb - Mb) * Z, Mb * Z


def info_bits(F: int, K: int, seed: int) -> np.ndarray:
    """F x K uniform information bits, one per byte (0/1)."""
    g = np.random.Generator(np.random.PCG64(seed))
    return g.integers(0, 2, size=(F, K), dtype=np.uint8)


def std_normal(F: int, N: int, seed: int, dtype=np.float32) -> np.ndarray:
    """F x N standard-normal samples (the channel noise before scaling)."""
    g = np.random.Generator(np.random.PCG64(seed))
    return g.standard_normal(size=(F, N)).astype(dtype)


def sigma2_from_ebn0(ebn0_db, rate: float):
    """Noise variance for BPSK at Eb/N0 (dB) and code rate R:
    sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)). A number gives a float, an array of
    Eb/N0 values (one per frame) an array of the same shape (float64)."""
    if np.ndim(ebn0_db) == 0:
        return 1.0 / (2.0 * rate * math.pow(10.0, float(ebn0_db) / 10.0))
    e = np.asarray(ebn0_db, dtype=np.float64)
    return 1.0 / (2.0 * rate * np.power(10.0, e / 10.0))


def heavy_column_code(Mb: int, heavy: int, Z: int, seed: int) -> np.ndarray:
    """A decodable QC base matrix of Mb x 24 blocks whose block column 0 has
    weight `heavy` and whose other columns are lighter (5 random blocks per
    row in columns 1..23, shifts uniform); it has no encoder structure. Used
    to test the column-weight limit of the packed fixed-point kernels."""
    rng = np.random.default_rng(seed)
    h = np.full((Mb, 24), -1, np.int16)
    for i in range(Mb):
        cols = rng.choice(np.arange(1, 24), size=5, replace=False)
        h[i, cols] = rng.integers(0, Z, 5)
    h[:heavy, 0] = rng.integers(0, Z, heavy)
    return h


def zero_word_llr(N: int, F: int, seed: int, sigma: float = 0.9) -> np.ndarray:
    """Channel LLRs (2y/sigma^2, FP32 [F][N]) of the all-zero word, a codeword
    of every linear code, sent as BPSK +1 over AWGN of deviation sigma."""
    z = std_normal(F, N, seed)
    return (np.float32(2.0 / sigma**2) * (np.float32(1.0) + np.float32(sigma) * z)).astype(np.float32)


def limit_code(Mb: int, Nb: int, Z: int, full_row_degree: int, other_degree: int, seed: int) -> np.ndarray:
    """An encodable base matrix at chosen sizes (the library's limits in the
    tests): the dual-diagonal parity part of the Wi-Fi shape (h_b = 1 at rows
    0 and M_b-1, 0 at row y), block row 0 of check degree `full_row_degree`
    and the others of degree `other_degree`, information columns drawn
    uniformly, shifts uniform in [0, Z-1]. Returns int16 [Mb][Nb]."""
    rng = np.random.default_rng(seed)
    Kb = Nb - Mb
    h = np.full((Mb, Nb), -1, dtype=np.int64)
    h[:, Kb:] = _parity_part(Mb, Nb, 1, 0)
    for i in range(Mb):
        parity = int((h[i, Kb:] >= 0).sum())
        want = (full_row_degree if i == 0 else other_degree) - parity
        cols = rng.choice(Kb, size=min(Kb, max(0, want)), replace=False)
        h[i, cols] = rng.integers(0, Z, len(cols))
    return h.astype(np.int16)
