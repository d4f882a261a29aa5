"""Independent reference computations used to pin the oracle.

Nothing here calls the oracle: these are textbook GF(2) linear algebra,
brute-force codebooks and max-marginals, written directly from definitions.
"""
from __future__ import annotations

import numpy as np


def dense_h(hbm, Z):
    """Expands a base matrix into the binary parity-check matrix H (Sec. 1,
    eq. 2): block (i, j) is zero for -1, otherwise the Z x Z identity whose
    row r has its one in column (r + s) mod Z."""
    hbm = np.asarray(hbm)
    Mb, Nb = hbm.shape
    H = np.zeros((Mb * Z, Nb * Z), dtype=np.uint8)
    for i in range(Mb):
        for j in range(Nb):
            s = int(hbm[i, j])
            if s < 0:
                continue
            for r in range(Z):
                H[i * Z + r, j * Z + (r + s) % Z] = 1
    return H


def gf2_solve(A, b):
    """Solves A x = b over GF(2) for square invertible A by Gauss-Jordan
    elimination. A: [n][n] uint8, b: [n][k] uint8. Raises if A is singular."""
    A = (np.asarray(A, dtype=np.uint8) & 1).copy()
    b = (np.asarray(b, dtype=np.uint8) & 1).copy()
    n = A.shape[0]
    if b.ndim == 1:
        b = b[:, None]
    M = np.concatenate([A, b], axis=1).astype(bool)
    for col in range(n):
        piv = np.nonzero(M[col:, col])[0]
        if piv.size == 0:
            raise np.linalg.LinAlgError("singular over GF(2)")
        p = col + piv[0]
        if p != col:
            M[[col, p]] = M[[p, col]]
        rows = np.nonzero(M[:, col])[0]
        rows = rows[rows != col]
        M[rows] ^= M[col]
    return M[:, n:].astype(np.uint8)


def gf2_encode(hbm, Z, info):
    """Systematic encoding by elimination: with H = [H1 | H2], solve
    H2 p = H1 s over GF(2). info: [F][K] -> codewords [F][N]."""
    H = dense_h(hbm, Z)
    Mb, Nb = np.asarray(hbm).shape
    K = (Nb - Mb) * Z
    H1, H2 = H[:, :K], H[:, K:]
    s = np.asarray(info, dtype=np.uint8) & 1
    rhs = (H1.astype(np.int64) @ s.T.astype(np.int64)) % 2
    p = gf2_solve(H2, rhs.astype(np.uint8))
    return np.concatenate([s, p.T], axis=1).astype(np.uint8)


def syndrome(H, x):
    """H x over GF(2) for each row of x ([F][N])."""
    return (np.asarray(x, dtype=np.int64) @ H.T.astype(np.int64)) % 2


def codebook(H):
    """All codewords of a tiny code, by brute force over 2^N words."""
    Mrows, N = H.shape
    if N > 22:
        raise ValueError("codebook brute force is limited to N <= 22")
    words = ((np.arange(1 << N, dtype=np.int64)[:, None] >> np.arange(N)) & 1).astype(np.uint8)
    ok = ~np.any(syndrome(H, words), axis=1)
    return words[ok]


def max_marginals(C, llr):
    """Exact max-product posteriors on a codebook C ([ncw][N]) for channel
    LLRs (positive = bit 0, eq. 17):
      L_n = max_{c: c_n=0} phi(c) - max_{c: c_n=1} phi(c),
      phi(c) = 1/2 sum_k llr_k (1 - 2 c_k)."""
    llr = np.asarray(llr, dtype=np.float64)
    phi = 0.5 * ((1.0 - 2.0 * C.astype(np.float64)) @ llr.T)   # [ncw][F]
    F, N = llr.shape
    out = np.empty((F, N))
    for n in range(N):
        m0 = phi[C[:, n] == 0].max(axis=0)
        m1 = phi[C[:, n] == 1].max(axis=0)
        out[:, n] = m0 - m1
    return out


def ml_decode(C, llr):
    """Maximum-likelihood codeword per frame: argmax_c phi(c)."""
    llr = np.asarray(llr, dtype=np.float64)
    phi = (1.0 - 2.0 * C.astype(np.float64)) @ llr.T
    return C[np.argmax(phi, axis=0)]
