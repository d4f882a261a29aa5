/*
 * oracle.c -- plain, slow CPU reference for the QC-LDPC direct encoder and the
 * layered single-scan min-sum decoder of Palenik & Szitkey, "High Throughput
 * Open-Source Implementation of Wi-Fi 6 and WiMAX LDPC Encoder and Decoder".
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header, table or helper with the GPU library; the two meet only at the
 * seeded inputs they both consume.
 *
 * Everything here follows the paper's definitions literally: the parity
 * check matrix is never compressed, every check message R is kept per edge,
 * and every check-node minimum is taken by brute force over the other edges.
 * Compile with -ffp-contract=off so that a*b+c is never fused.
 *
 * Conventions (readings of the paper, listed in the design notes):
 *  - H_bm(i,j) = -1 is a zero block, s >= 0 the identity cyclically shifted
 *    by s (Sec. 1, eq. 2). Check row r of block row i touches variable
 *    j*Z + (r + s) mod Z, i.e. (P_s u)[r] = u[(r + s) mod Z] and
 *    (P_s^-1 v)[c] = v[(c - s) mod Z].
 *  - sgn(q) = -1 iff q < 0, so -0.0 counts as positive (eq. 18).
 *  - x_hat = 0 iff the posterior is > 0, so a zero posterior decodes to 1
 *    (eq. 21).
 *  - Iterations are counted as completed full passes over all layers; the
 *    syndrome is tested after each one (Sec. 4, step 4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ESTRUCT (-2)
#define ORC_ENOMEM (-5)

/* ------------------------------------------------------------------------ */
/* Code model (Sec. 1, eq. 2)                                                */
/* ------------------------------------------------------------------------ */

/* Validates a base matrix: entries in [-1, Z-1]; for decoding every check
 * row must have at least two edges (the minimum over "all other" edges of
 * eq. 18 is otherwise empty). */
static int check_base(const int16_t *hbm, int Mb, int Nb, int Z, int need_deg2)
{
    if (!hbm || Mb < 1 || Nb <= Mb || Z < 1)
        return ORC_EINVAL;
    for (int i = 0; i < Mb; i++) {
        int deg = 0;
        for (int j = 0; j < Nb; j++) {
            int s = hbm[i * Nb + j];
            if (s < -1 || s >= Z)
                return ORC_EINVAL;
            deg += (s >= 0);
        }
        if (need_deg2 && deg < 2)
            return ORC_EINVAL;
    }
    return ORC_OK;
}

/* Variable (column of H) that check row r of block row i reaches through the
 * circulant with shift s in block column j. */
static long var_of(int j, int s, int r, int Z)
{
    return (long)j * Z + (r + s) % Z;
}

/* Number of edges of H (= ones in H) and the largest block-row degree. */
static long count_edges(const int16_t *hbm, int Mb, int Nb, int Z, int *max_deg)
{
    long e = 0;
    int md = 0;
    for (int i = 0; i < Mb; i++) {
        int d = 0;
        for (int j = 0; j < Nb; j++)
            d += hbm[i * Nb + j] >= 0;
        if (d > md)
            md = d;
        e += (long)d * Z;
    }
    if (max_deg)
        *max_deg = md;
    return e;
}

int orc_code_edges(const int16_t *hbm, int Mb, int Nb, int Z, int64_t *edges, int32_t *max_deg)
{
    int md = 0;
    if (check_base(hbm, Mb, Nb, Z, 0))
        return ORC_EINVAL;
    *edges = count_edges(hbm, Mb, Nb, Z, &md);
    *max_deg = md;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Direct encoder (Sec. 2, eqs. 8-15)                                        */
/* ------------------------------------------------------------------------ */

/* Checks the structure the direct encoder needs (Sec. 1, eqs. 3-7): h_b has
 * equal non-negative entries in its first and last rows and exactly one
 * more non-negative entry at some row y in between; H_b2' is the staircase
 * with zero shifts at (r, r) and (r+1, r). Returns y, or -1. */
static int find_y(const int16_t *hbm, int Mb, int Nb)
{
    int Kb = Nb - Mb;
    if (Mb < 3)
        return -1;
    int a0 = hbm[0 * Nb + Kb], a1 = hbm[(Mb - 1) * Nb + Kb];
    if (a0 < 0 || a0 != a1)
        return -1;
    int y = -1;
    for (int i = 1; i < Mb - 1; i++) {
        if (hbm[i * Nb + Kb] >= 0) {
            if (y >= 0)
                return -1;
            y = i;
        }
    }
    if (y < 0)
        return -1;
    for (int c = 0; c < Mb - 1; c++) {
        for (int i = 0; i < Mb; i++) {
            int s = hbm[i * Nb + Kb + 1 + c];
            int want = (i == c || i == c + 1) ? 0 : -1;
            if (s != want)
                return -1;
        }
    }
    return y;
}

int orc_encode(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *info, uint8_t *cw, int64_t F)
{
    if (check_base(hbm, Mb, Nb, Z, 0) || F < 0 || (F > 0 && (!info || !cw)))
        return ORC_EINVAL;
    int y = find_y(hbm, Mb, Nb);
    if (y < 0)
        return ORC_ESTRUCT;
    int Kb = Nb - Mb;
    long K = (long)Kb * Z, N = (long)Nb * Z;
    uint8_t *S = malloc((size_t)Mb * Z);  /* S_i, eq. 15 */
    uint8_t *T = malloc((size_t)Z);
    uint8_t *v = malloc((size_t)Mb * Z);  /* v_0 .. v_{Mb-1}, eqs. 10-11 */
    if (!S || !T || !v) {
        free(S); free(T); free(v);
        return ORC_ENOMEM;
    }
    for (int64_t f = 0; f < F; f++) {
        const uint8_t *s = info + f * K;   /* u_j = s[jZ .. jZ+Z-1], eqs. 8-9 */
        uint8_t *c = cw + f * N;
        /* eq. 15: S_i = sum_j P_{H(i,j)} u_j over GF(2), skipping -1 blocks */
        for (int i = 0; i < Mb; i++) {
            for (int r = 0; r < Z; r++) {
                uint8_t acc = 0;
                for (int j = 0; j < Kb; j++) {
                    int sh = hbm[i * Nb + j];
                    if (sh < 0)
                        continue;
                    acc ^= s[(long)j * Z + (r + sh) % Z] & 1;
                }
                S[i * Z + r] = acc;
            }
        }
        /* eq. 12: v_0 = P^-1_{h_b(y)} sum_i S_i */
        for (int r = 0; r < Z; r++) {
            uint8_t acc = 0;
            for (int i = 0; i < Mb; i++)
                acc ^= S[i * Z + r];
            T[r] = acc;
        }
        int hy = hbm[y * Nb + Kb];
        for (int r = 0; r < Z; r++)
            v[r] = T[((r - hy) % Z + Z) % Z];
        /* eq. 13: v_1 = P_{h_b(0)} v_0 + S_0 */
        int h0 = hbm[0 * Nb + Kb];
        for (int r = 0; r < Z; r++)
            v[1 * Z + r] = v[(r + h0) % Z] ^ S[0 * Z + r];
        /* eq. 14: v_{i+1} = v_i + P_{h_b(i)} v_0 + S_i for i = 1 .. Mb-2,
         * where a -1 entry of h_b contributes nothing */
        for (int i = 1; i <= Mb - 2; i++) {
            int hi = hbm[i * Nb + Kb];
            for (int r = 0; r < Z; r++) {
                uint8_t t = v[i * Z + r] ^ S[i * Z + r];
                if (hi >= 0)
                    t ^= v[(r + hi) % Z];
                v[(i + 1) * Z + r] = t;
            }
        }
        /* eq. 1: c = [s p], s = i */
        for (long k = 0; k < K; k++)
            c[k] = s[k] & 1;
        memcpy(c + K, v, (size_t)Mb * Z);
    }
    free(S); free(T); free(v);
    return ORC_OK;
}

/* Hard decisions of eq. 21 and the parity of every check of H x_hat. */
static int syndrome_zero(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *x)
{
    for (int i = 0; i < Mb; i++)
        for (int r = 0; r < Z; r++) {
            int p = 0;
            for (int j = 0; j < Nb; j++) {
                int s = hbm[i * Nb + j];
                if (s >= 0)
                    p ^= x[var_of(j, s, r, Z)];
            }
            if (p)
                return 0;
        }
    return 1;
}

int orc_syndrome_ok(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *bits, int64_t F, uint8_t *ok)
{
    if (check_base(hbm, Mb, Nb, Z, 0) || F < 0)
        return ORC_EINVAL;
    long N = (long)Nb * Z;
    for (int64_t f = 0; f < F; f++)
        ok[f] = (uint8_t)syndrome_zero(hbm, Mb, Nb, Z, bits + f * N);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Layered min-sum decoder in floating point (Sec. 4, eqs. 17-23)           */
/* ------------------------------------------------------------------------ */

/* One edge list per block row, in ascending block column: the order in
 * which a check row visits its variables. */
typedef struct {
    int Mb, Nb, Z;
    long N, E;
    int *deg;      /* [Mb] */
    int *col;      /* [Mb][Nb] block columns, ascending */
    int *shift;    /* [Mb][Nb] */
    long *ebase;   /* [Mb] first edge index of block row i */
} layers_t;

static int layers_init(layers_t *ly, const int16_t *hbm, int Mb, int Nb, int Z)
{
    ly->Mb = Mb; ly->Nb = Nb; ly->Z = Z;
    ly->N = (long)Nb * Z;
    ly->deg = calloc((size_t)Mb, sizeof(int));
    ly->col = calloc((size_t)Mb * Nb, sizeof(int));
    ly->shift = calloc((size_t)Mb * Nb, sizeof(int));
    ly->ebase = calloc((size_t)Mb, sizeof(long));
    if (!ly->deg || !ly->col || !ly->shift || !ly->ebase)
        return ORC_ENOMEM;
    long e = 0;
    for (int i = 0; i < Mb; i++) {
        int d = 0;
        for (int j = 0; j < Nb; j++) {
            int s = hbm[i * Nb + j];
            if (s >= 0) {
                ly->col[i * Nb + d] = j;
                ly->shift[i * Nb + d] = s;
                d++;
            }
        }
        ly->deg[i] = d;
        ly->ebase[i] = e;
        e += (long)d * Z;
    }
    ly->E = e;
    return ORC_OK;
}

static void layers_free(layers_t *ly)
{
    free(ly->deg); free(ly->col); free(ly->shift); free(ly->ebase);
}

/* Edge index of edge k (0-based within the row) of check row r, block row i. */
static long edge_of(const layers_t *ly, int i, int r, int k)
{
    return ly->ebase[i] + (long)r * ly->deg[i] + k;
}

#define REAL float
#define SFX(name) name##_f32
#define RABS fabsf
#include "oracle_fp.inc"
#undef REAL
#undef SFX
#undef RABS

#define REAL double
#define SFX(name) name##_f64
#define RABS fabs
#include "oracle_fp.inc"
#undef REAL
#undef SFX
#undef RABS

/* ------------------------------------------------------------------------ */
/* Saturating fixed-point decoder: int8 LLRs and messages, int16 posteriors */
/* ------------------------------------------------------------------------ */

static int32_t sat16(int32_t x)
{
    /* symmetric saturation, so that negating a value never saturates */
    if (x > 32767)
        return 32767;
    if (x < -32767)
        return -32767;
    return x;
}

/*
 * Magnitude rule for the outgoing message, from the raw minimum m (0..127):
 *   wq == 0 : offset min-sum, max(m - offset, 0)
 *   wq >  0 : normalised min-sum with weight wq/16, min(127, (wq*m + 8) >> 4)
 * wq_table (nullable, [max_iter][Mb][Nb]) replaces the scalar wq per
 * iteration, block row and block column; its entries are always weights
 * (an entry of 0 gives magnitude 0) and the offset is then unused.
 */
int orc_decode_i8(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter,
                  int offset, int wq, const uint8_t *wq_table, int early_term,
                  uint8_t *bits, int16_t *post, int32_t *iters, uint8_t *ok)
{
    if (check_base(hbm, Mb, Nb, Z, 1) || F < 0 || max_iter < 1 || offset < 0 || offset > 127 ||
        wq < 0 || wq > 31)
        return ORC_EINVAL;
    layers_t ly;
    if (layers_init(&ly, hbm, Mb, Nb, Z)) {
        layers_free(&ly);
        return ORC_ENOMEM;
    }
    long N = ly.N;
    int16_t *L = malloc(sizeof(int16_t) * (size_t)N);
    int8_t *R = malloc((size_t)ly.E);
    int32_t *Q = malloc(sizeof(int32_t) * (size_t)Nb);
    int32_t *Rn = malloc(sizeof(int32_t) * (size_t)Nb);
    long *nv = malloc(sizeof(long) * (size_t)Nb);
    uint8_t *x = malloc((size_t)N);
    if (!L || !R || !Q || !Rn || !nv || !x) {
        free(L); free(R); free(Q); free(Rn); free(nv); free(x); layers_free(&ly);
        return ORC_ENOMEM;
    }
    for (int64_t f = 0; f < F; f++) {
        for (long n = 0; n < N; n++)
            L[n] = llr[f * N + n];
        memset(R, 0, (size_t)ly.E);
        int done = 0, k;
        for (k = 1; k <= max_iter && !done; k++) {
            for (int i = 0; i < Mb; i++) {
                int d = ly.deg[i];
                for (int r = 0; r < Z; r++) {
                    for (int e = 0; e < d; e++) {
                        nv[e] = var_of(ly.col[i * Nb + e], ly.shift[i * Nb + e], r, Z);
                        Q[e] = sat16((int32_t)L[nv[e]] - R[edge_of(&ly, i, r, e)]);
                    }
                    for (int e = 0; e < d; e++) {
                        int32_t m = INT32_MAX;
                        int neg = 0;
                        for (int e2 = 0; e2 < d; e2++) {
                            if (e2 == e)
                                continue;
                            /* message magnitudes live in int8: |Q| is clipped to 127 */
                            int32_t a = Q[e2] < 0 ? -Q[e2] : Q[e2];
                            if (a > 127)
                                a = 127;
                            if (a < m)
                                m = a;
                            if (Q[e2] < 0)
                                neg ^= 1;
                        }
                        int32_t mag;
                        /* a table entry is always a weight (0 is weight 0);
                         * only the scalar wq == 0 selects offset min-sum */
                        int wk = wq_table ? wq_table[((long)(k - 1) * Mb + i) * Nb + ly.col[i * Nb + e]] : wq;
                        if (wq_table || wk > 0) {
                            mag = (wk * m + 8) >> 4;
                            if (mag > 127)
                                mag = 127;
                        } else {
                            mag = m - offset;
                            if (mag < 0)
                                mag = 0;
                        }
                        Rn[e] = neg ? -mag : mag;
                    }
                    for (int e = 0; e < d; e++) {
                        R[edge_of(&ly, i, r, e)] = (int8_t)Rn[e];
                        L[nv[e]] = (int16_t)sat16(Q[e] + Rn[e]);
                    }
                }
            }
            for (long n = 0; n < N; n++)
                x[n] = L[n] > 0 ? 0 : 1;
            if (early_term && syndrome_zero(hbm, Mb, Nb, Z, x))
                done = 1;
        }
        int it = k - 1;
        uint8_t good = done ? 1 : (uint8_t)syndrome_zero(hbm, Mb, Nb, Z, x);
        if (bits)
            memcpy(bits + f * N, x, (size_t)N);
        if (post)
            memcpy(post + f * N, L, sizeof(int16_t) * (size_t)N);
        if (iters)
            iters[f] = it;
        if (ok)
            ok[f] = good;
    }
    free(L); free(R); free(Q); free(Rn); free(nv); free(x); layers_free(&ly);
    return ORC_OK;
}

/*
 * Flooding schedule on the saturating fixed-point path: the check phase is
 * that of orc_decode_i8 (int8 messages, |Q| clipped to 127, offset or wq/16
 * magnitude rule), all rows reading the posteriors of the previous
 * iteration; the variable phase is Z[n] = sat16(... sat16(Z0[n] + R_a) + R_b
 * ...), the new messages at n added in ascending block-row order (eq. 20).
 */
int orc_decode_flood_i8(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter,
                        int offset, int wq, int early_term, uint8_t *bits, int16_t *post, int32_t *iters,
                        uint8_t *ok)
{
    if (check_base(hbm, Mb, Nb, Z, 1) || F < 0 || max_iter < 1 || offset < 0 || offset > 127 ||
        wq < 0 || wq > 31)
        return ORC_EINVAL;
    layers_t ly;
    if (layers_init(&ly, hbm, Mb, Nb, Z)) {
        layers_free(&ly);
        return ORC_ENOMEM;
    }
    long N = ly.N;
    int16_t *L = malloc(sizeof(int16_t) * (size_t)N);
    int8_t *R = malloc((size_t)ly.E);
    int32_t *Q = malloc(sizeof(int32_t) * (size_t)Nb);
    long *nv = malloc(sizeof(long) * (size_t)Nb);
    uint8_t *x = malloc((size_t)N);
    if (!L || !R || !Q || !nv || !x) {
        free(L); free(R); free(Q); free(nv); free(x); layers_free(&ly);
        return ORC_ENOMEM;
    }
    for (int64_t f = 0; f < F; f++) {
        const int8_t *Z0 = llr + f * N;
        for (long n = 0; n < N; n++)
            L[n] = Z0[n];
        memset(R, 0, (size_t)ly.E);
        int done = 0, k;
        for (k = 1; k <= max_iter && !done; k++) {
            for (int i = 0; i < Mb; i++) {
                int d = ly.deg[i];
                for (int r = 0; r < Z; r++) {
                    for (int e = 0; e < d; e++) {
                        nv[e] = var_of(ly.col[i * Nb + e], ly.shift[i * Nb + e], r, Z);
                        Q[e] = sat16((int32_t)L[nv[e]] - R[edge_of(&ly, i, r, e)]);
                    }
                    for (int e = 0; e < d; e++) {
                        int32_t m = INT32_MAX;
                        int neg = 0;
                        for (int e2 = 0; e2 < d; e2++) {
                            if (e2 == e)
                                continue;
                            int32_t a = Q[e2] < 0 ? -Q[e2] : Q[e2];
                            if (a > 127)
                                a = 127;
                            if (a < m)
                                m = a;
                            if (Q[e2] < 0)
                                neg ^= 1;
                        }
                        int32_t mag;
                        if (wq > 0) {
                            mag = (wq * m + 8) >> 4;
                            if (mag > 127)
                                mag = 127;
                        } else {
                            mag = m - offset;
                            if (mag < 0)
                                mag = 0;
                        }
                        R[edge_of(&ly, i, r, e)] = (int8_t)(neg ? -mag : mag);
                    }
                }
            }
            for (long n = 0; n < N; n++)
                L[n] = Z0[n];
            for (int i = 0; i < Mb; i++)
                for (int r = 0; r < Z; r++)
                    for (int e = 0; e < ly.deg[i]; e++) {
                        long n = var_of(ly.col[i * Nb + e], ly.shift[i * Nb + e], r, Z);
                        L[n] = (int16_t)sat16((int32_t)L[n] + R[edge_of(&ly, i, r, e)]);
                    }
            for (long n = 0; n < N; n++)
                x[n] = L[n] > 0 ? 0 : 1;
            if (early_term && syndrome_zero(hbm, Mb, Nb, Z, x))
                done = 1;
        }
        uint8_t good = done ? 1 : (uint8_t)syndrome_zero(hbm, Mb, Nb, Z, x);
        if (bits)
            memcpy(bits + f * N, x, (size_t)N);
        if (post)
            memcpy(post + f * N, L, sizeof(int16_t) * (size_t)N);
        if (iters)
            iters[f] = k - 1;
        if (ok)
            ok[f] = good;
    }
    free(L); free(R); free(Q); free(nv); free(x); layers_free(&ly);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The paper's own fixed point (Sec. 5): Q_B-bit LLRs in int16              */
/* ------------------------------------------------------------------------ */

/* two's-complement wrap to int16, as storing an int into int16_t does */
static int32_t wrap16(int32_t x)
{
    return (int32_t)(int16_t)(uint16_t)(uint32_t)x;
}

static int32_t q16_fix(int32_t x, int wrap)
{
    return wrap ? wrap16(x) : sat16(x);
}

/*
 * Layered min-sum on int16 values (Sec. 5: Q_B-bit LLRs held in int16 with
 * headroom, C's wrap-around arithmetic; wrap = 0 gives the saturating twin
 * with symmetric saturation at +-32767). Per check row, with F the wrap or
 * the saturation:
 *   Q_e = F(L[n_e] - R_e);  a_e = |Q_e| (exact, up to 32768)
 *   m_e = min_{e' != e} a_e';  R_e = F(s_e * ((wq * m_e + 8) >> 4))
 *   L[n_e] = F(Q_e + R_e)
 * wq/16 is the normalisation (16: plain min-sum). Messages are 16-bit, with
 * no clipping below 16 bits. Hard decision and syndrome as the other decoders.
 */
int orc_decode_q16(const int16_t *hbm, int Mb, int Nb, int Z, const int16_t *llr, int64_t F, int max_iter, int wq,
                   int wrap, int early_term, uint8_t *bits, int16_t *post, int32_t *iters, uint8_t *ok)
{
    if (check_base(hbm, Mb, Nb, Z, 1) || F < 0 || max_iter < 1 || wq < 1 || wq > 31 || (F > 0 && !llr))
        return ORC_EINVAL;
    layers_t ly;
    if (layers_init(&ly, hbm, Mb, Nb, Z)) {
        layers_free(&ly);
        return ORC_ENOMEM;
    }
    long N = ly.N;
    int16_t *L = malloc(sizeof(int16_t) * (size_t)N);
    int16_t *R = malloc(sizeof(int16_t) * (size_t)ly.E);
    int32_t *Q = malloc(sizeof(int32_t) * (size_t)Nb);
    int32_t *Rn = malloc(sizeof(int32_t) * (size_t)Nb);
    long *nv = malloc(sizeof(long) * (size_t)Nb);
    uint8_t *x = malloc((size_t)N);
    if (!L || !R || !Q || !Rn || !nv || !x) {
        free(L); free(R); free(Q); free(Rn); free(nv); free(x); layers_free(&ly);
        return ORC_ENOMEM;
    }
    for (int64_t f = 0; f < F; f++) {
        for (long n = 0; n < N; n++)
            L[n] = llr[f * N + n];
        memset(R, 0, sizeof(int16_t) * (size_t)ly.E);
        int done = 0, k;
        for (k = 1; k <= max_iter && !done; k++) {
            for (int i = 0; i < Mb; i++) {
                int d = ly.deg[i];
                for (int r = 0; r < Z; r++) {
                    for (int e = 0; e < d; e++) {
                        nv[e] = var_of(ly.col[i * Nb + e], ly.shift[i * Nb + e], r, Z);
                        Q[e] = q16_fix((int32_t)L[nv[e]] - R[edge_of(&ly, i, r, e)], wrap);
                    }
                    for (int e = 0; e < d; e++) {
                        int32_t m = INT32_MAX;
                        int neg = 0;
                        for (int e2 = 0; e2 < d; e2++) {
                            if (e2 == e)
                                continue;
                            int32_t a = Q[e2] < 0 ? -Q[e2] : Q[e2];
                            if (a < m)
                                m = a;
                            if (Q[e2] < 0)
                                neg ^= 1;
                        }
                        int32_t mag = (wq * m + 8) >> 4;
                        Rn[e] = q16_fix(neg ? -mag : mag, wrap);
                    }
                    for (int e = 0; e < d; e++) {
                        R[edge_of(&ly, i, r, e)] = (int16_t)Rn[e];
                        L[nv[e]] = (int16_t)q16_fix(Q[e] + Rn[e], wrap);
                    }
                }
            }
            for (long n = 0; n < N; n++)
                x[n] = L[n] > 0 ? 0 : 1;
            if (early_term && syndrome_zero(hbm, Mb, Nb, Z, x))
                done = 1;
        }
        uint8_t good = done ? 1 : (uint8_t)syndrome_zero(hbm, Mb, Nb, Z, x);
        if (bits)
            memcpy(bits + f * N, x, (size_t)N);
        if (post)
            memcpy(post + f * N, L, sizeof(int16_t) * (size_t)N);
        if (iters)
            iters[f] = k - 1;
        if (ok)
            ok[f] = good;
    }
    free(L); free(R); free(Q); free(Rn); free(nv); free(x); layers_free(&ly);
    return ORC_OK;
}

/* Q_B-bit quantiser: q = clamp(rint(scale * llr), -qmax, qmax), half to even. */
int orc_quantize_q16(const float *llr, int16_t *q, int64_t n, float scale, int qmax)
{
    if (n < 0 || qmax < 1 || qmax > 32767)
        return ORC_EINVAL;
    for (int64_t k = 0; k < n; k++) {
        float v = rintf(scale * llr[k]);
        if (v > (float)qmax)
            v = (float)qmax;
        if (v < (float)-qmax)
            v = (float)-qmax;
        q[k] = (int16_t)v;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Packed bits (Sec. 3, bitmap encoder): bit k of a frame is bit (k mod 8)  */
/* of byte k/8 (least significant bit first); a frame of n bits takes       */
/* ceil(n/8) bytes, unused high bits of its last byte are 0.                */
/* ------------------------------------------------------------------------ */

static void unpack_bits(const uint8_t *in, long n, uint8_t *out)
{
    for (long k = 0; k < n; k++)
        out[k] = (uint8_t)((in[k >> 3] >> (k & 7)) & 1u);
}

static void pack_bits(const uint8_t *in, long n, uint8_t *out)
{
    memset(out, 0, (size_t)((n + 7) / 8));
    for (long k = 0; k < n; k++)
        out[k >> 3] |= (uint8_t)((in[k] & 1u) << (k & 7));
}

/* Cyclic shift of F packed Z-bit blocks by s (0 <= s < Z), the operation
 * the direct encoder applies to every block (eqs. 12-15):
 * out[r] = in[(r + s) mod Z]. */
int orc_shift_packed(const uint8_t *in, uint8_t *out, int64_t F, int Z, int s)
{
    if (F < 0 || Z < 1 || s < 0 || s >= Z)
        return ORC_EINVAL;
    long nb = (Z + 7) / 8;
    uint8_t *a = malloc((size_t)Z), *b = malloc((size_t)Z);
    if (!a || !b) {
        free(a); free(b);
        return ORC_ENOMEM;
    }
    for (int64_t f = 0; f < F; f++) {
        unpack_bits(in + f * nb, Z, a);
        for (int r = 0; r < Z; r++)
            b[r] = a[(r + s) % Z];
        pack_bits(b, Z, out + f * nb);
    }
    free(a); free(b);
    return ORC_OK;
}

/* Packed direct encoder: the codeword of orc_encode for the unpacked
 * information bits, packed. info: [F][ceil(K/8)], cw: [F][ceil(N/8)]. */
int orc_encode_packed(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *info, uint8_t *cw, int64_t F)
{
    if (check_base(hbm, Mb, Nb, Z, 0) || F < 0)
        return ORC_EINVAL;
    long K = (long)(Nb - Mb) * Z, N = (long)Nb * Z;
    long kb = (K + 7) / 8, nbyt = (N + 7) / 8;
    uint8_t *u = malloc((size_t)K), *c = malloc((size_t)N);
    if (!u || !c) {
        free(u); free(c);
        return ORC_ENOMEM;
    }
    int rc = ORC_OK;
    for (int64_t f = 0; f < F && rc == ORC_OK; f++) {
        unpack_bits(info + f * kb, K, u);
        rc = orc_encode(hbm, Mb, Nb, Z, u, c, 1);
        if (rc == ORC_OK)
            pack_bits(c, N, cw + f * nbyt);
    }
    free(u); free(c);
    return rc;
}

/* int8 quantiser of channel LLRs: q = clamp(rint(scale * llr), -127, 127),
 * rint rounding half to even (the default rounding mode). */
int orc_quantize_i8(const float *llr, int8_t *q, int64_t n, float scale)
{
    if (n < 0 || (n > 0 && (!llr || !q)))
        return ORC_EINVAL;
    for (int64_t k = 0; k < n; k++) {
        float v = rintf(scale * llr[k]);
        if (v > 127.0f)
            v = 127.0f;
        if (v < -127.0f)
            v = -127.0f;
        q[k] = (int8_t)v;
    }
    return ORC_OK;
}

/* Learned weights in 1/16 steps for the fixed-point decoder (the int8
 * decoder's normalisation wq/16, Sec. 5 fixed point): wq = clamp(rint(16 w),
 * 0, 31), rint rounding half to even. 16 w is exact in float (a power-of-two
 * scaling). A NaN weight maps to 0, +inf to 31 and -inf to 0. */
int orc_quantize_weights(const float *w, uint8_t *wq, int64_t n)
{
    if (n < 0 || (n > 0 && (!w || !wq)))
        return ORC_EINVAL;
    for (int64_t k = 0; k < n; k++) {
        float v = rintf(16.0f * w[k]);
        if (!(v >= 0.0f))   /* negative or NaN */
            v = 0.0f;
        if (v > 31.0f)
            v = 31.0f;
        wq[k] = (uint8_t)v;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Learned normalised min-sum: loss and its exact gradient                  */
/* ------------------------------------------------------------------------ */

/* softplus(z) = log(1 + exp(z)), evaluated without overflow */
static double softplus(double z)
{
    return (z > 0 ? z : 0.0) + log1p(exp(-fabs(z)));
}

static double sigmoid(double z)
{
    if (z >= 0)
        return 1.0 / (1.0 + exp(-z));
    double t = exp(z);
    return t / (1.0 + t);
}

/*
 * Unrolled layered min-sum with per-(iteration, block row, block column)
 * weights w[T][Mb][Nb]: the message leaving edge e of a check row in
 * iteration t (1-based) is sgn_e * w[t-1][i][j_e] * m_e. Early termination
 * is off: exactly T iterations run.
 *
 * Loss: l = 1/(T F N) * sum_t sum_f sum_n softplus(-(1 - 2 c_fn) L_fn^(t)),
 * i.e. binary cross-entropy of sigmoid(L) (the probability of bit 0 under
 * eq. 17) against the transmitted bit, at every iteration.
 *
 * If grad_w is non-null it receives dl/dw, obtained by running the
 * iterations and layers in reverse (adjoint method). The forward pass is
 * evaluated in float when fwd_f32 is set (so that its signs and minima are
 * those of a float decoder) and in double otherwise; the gradient itself is
 * always accumulated in double.
 *
 * loss_per_iter[t] receives the iteration-t share of l (they sum to l).
 * post_last (nullable, [F][N]) receives the posteriors after iteration T.
 */
int orc_nms_train(const int16_t *hbm, int Mb, int Nb, int Z, const double *llr, const uint8_t *cw,
                  int64_t F, int T, const double *w, int fwd_f32,
                  double *loss_per_iter, double *grad_w, double *post_last)
{
    if (check_base(hbm, Mb, Nb, Z, 1) || F < 1 || T < 1 || !llr || !cw || !w || !loss_per_iter)
        return ORC_EINVAL;
    layers_t ly;
    if (layers_init(&ly, hbm, Mb, Nb, Z)) {
        layers_free(&ly);
        return ORC_ENOMEM;
    }
    long N = ly.N, E = ly.E;
    double *L = malloc(sizeof(double) * (size_t)N);
    double *R = malloc(sizeof(double) * (size_t)E);
    double *Qt = malloc(sizeof(double) * (size_t)E * T);    /* Q of every edge, every iteration */
    double *Lt = malloc(sizeof(double) * (size_t)N * T);    /* L after every iteration */
    double *gL = malloc(sizeof(double) * (size_t)N);
    double *gR = malloc(sizeof(double) * (size_t)E);
    double *Rn = malloc(sizeof(double) * (size_t)Nb);
    double *gm = malloc(sizeof(double) * (size_t)Nb);
    double *ga = malloc(sizeof(double) * (size_t)Nb);
    long *nv = malloc(sizeof(long) * (size_t)Nb);
    if (!L || !R || !Qt || !Lt || !gL || !gR || !Rn || !gm || !ga || !nv) {
        free(L); free(R); free(Qt); free(Lt); free(gL); free(gR); free(Rn); free(gm); free(ga); free(nv);
        layers_free(&ly);
        return ORC_ENOMEM;
    }
    const double scale = 1.0 / ((double)T * (double)F * (double)N);
    for (int t = 0; t < T; t++)
        loss_per_iter[t] = 0.0;
    if (grad_w)
        for (long k = 0; k < (long)T * Mb * Nb; k++)
            grad_w[k] = 0.0;

    for (int64_t f = 0; f < F; f++) {
        const uint8_t *c = cw + f * N;
        for (long n = 0; n < N; n++)
            L[n] = fwd_f32 ? (double)(float)llr[f * N + n] : llr[f * N + n];
        memset(R, 0, sizeof(double) * (size_t)E);
        /* forward */
        for (int t = 1; t <= T; t++) {
            for (int i = 0; i < Mb; i++) {
                int d = ly.deg[i];
                for (int r = 0; r < Z; r++) {
                    double *Q = Qt + (long)(t - 1) * E + edge_of(&ly, i, r, 0);
                    for (int e = 0; e < d; e++) {
                        nv[e] = var_of(ly.col[i * Nb + e], ly.shift[i * Nb + e], r, Z);
                        long ed = edge_of(&ly, i, r, e);
                        Q[e] = fwd_f32 ? (double)((float)L[nv[e]] - (float)R[ed]) : L[nv[e]] - R[ed];
                    }
                    for (int e = 0; e < d; e++) {
                        double m = INFINITY;
                        int neg = 0;
                        for (int e2 = 0; e2 < d; e2++) {
                            if (e2 == e)
                                continue;
                            if (fabs(Q[e2]) < m)
                                m = fabs(Q[e2]);
                            if (Q[e2] < 0)
                                neg ^= 1;
                        }
                        double wt = w[((long)(t - 1) * Mb + i) * Nb + ly.col[i * Nb + e]];
                        double mag = fwd_f32 ? (double)((float)wt * (float)m) : wt * m;
                        Rn[e] = neg ? -mag : mag;
                    }
                    for (int e = 0; e < d; e++) {
                        R[edge_of(&ly, i, r, e)] = Rn[e];
                        L[nv[e]] = fwd_f32 ? (double)((float)Q[e] + (float)Rn[e]) : Q[e] + Rn[e];
                    }
                }
            }
            memcpy(Lt + (long)(t - 1) * N, L, sizeof(double) * (size_t)N);
            double acc = 0.0;
            for (long n = 0; n < N; n++)
                acc += softplus(-(1.0 - 2.0 * c[n]) * L[n]);
            loss_per_iter[t - 1] += acc * scale;
        }
        if (post_last)
            memcpy(post_last + f * N, L, sizeof(double) * (size_t)N);
        if (!grad_w)
            continue;
        /* reverse: gL is the adjoint of the current L, gR[e] the adjoint of
         * the message R[e] as it was produced (and is consumed one iteration
         * later) */
        memset(gR, 0, sizeof(double) * (size_t)E);
        for (long n = 0; n < N; n++)
            gL[n] = 0.0;
        for (int t = T; t >= 1; t--) {
            /* the loss reads L after iteration t directly */
            const double *Lend = Lt + (long)(t - 1) * N;
            for (long n = 0; n < N; n++) {
                double x = 1.0 - 2.0 * c[n];
                gL[n] += -x * sigmoid(-x * Lend[n]) * scale;
            }
            for (int i = Mb - 1; i >= 0; i--) {
                int d = ly.deg[i];
                for (int r = 0; r < Z; r++) {
                    const double *Q = Qt + (long)(t - 1) * E + edge_of(&ly, i, r, 0);
                    /* first and second smallest |Q|, lowest index first on ties */
                    int a1 = -1, a2 = -1;
                    for (int e = 0; e < d; e++) {
                        if (a1 < 0 || fabs(Q[e]) < fabs(Q[a1])) {
                            a2 = a1;
                            a1 = e;
                        } else if (a2 < 0 || fabs(Q[e]) < fabs(Q[a2])) {
                            a2 = e;
                        }
                    }
                    for (int e = 0; e < d; e++) {
                        nv[e] = var_of(ly.col[i * Nb + e], ly.shift[i * Nb + e], r, Z);
                        ga[e] = 0.0;
                    }
                    for (int e = 0; e < d; e++) {
                        int neg = 0;
                        for (int e2 = 0; e2 < d; e2++)
                            if (e2 != e && Q[e2] < 0)
                                neg ^= 1;
                        double sg = neg ? -1.0 : 1.0;
                        double m = fabs(Q[e == a1 ? a2 : a1]);
                        long widx = ((long)(t - 1) * Mb + i) * Nb + ly.col[i * Nb + e];
                        long ed = edge_of(&ly, i, r, e);
                        /* the new message feeds L[n_e] (eq. 20) and the next
                         * iteration's Q through R (eq. 22) */
                        double G = gL[nv[e]] + gR[ed];
                        grad_w[widx] += G * sg * m;
                        gm[e] = G * sg * w[widx];
                    }
                    for (int e = 0; e < d; e++) {
                        if (e == a1)
                            ga[a2] += gm[e];
                        else
                            ga[a1] += gm[e];
                    }
                    for (int e = 0; e < d; e++) {
                        double sq = Q[e] < 0 ? -1.0 : 1.0;
                        double gQ = gL[nv[e]] + ga[e] * sq;
                        gL[nv[e]] = gQ;                     /* Q = L - R_old */
                        gR[edge_of(&ly, i, r, e)] = -gQ;
                    }
                }
            }
        }
    }
    free(L); free(R); free(Qt); free(Lt); free(gL); free(gR); free(Rn); free(gm); free(ga); free(nv);
    layers_free(&ly);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers for frame generation                        */
/* ------------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
 * multiplies two counter words by fixed odd constants, swaps the halves and
 * mixes in the key; the key is bumped by the Weyl increments between rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * Seeded frames for the BPSK/AWGN channel (eqs. 16-17).
 *  Information bit k of frame f: bit (k mod 32) of word (k/32 mod 4) of
 *    Philox(ctr = {k/128, f, 0, 0}, key = {seed_lo, seed_hi}).
 *  Noise sample n of frame f: the Box-Muller pair built from words
 *    (2p, 2p+1), p = (n mod 4)/2, of Philox(ctr = {n/4, f, 1, 0}, key), with
 *    u = (word >> 8 + 1/2) 2^-24, z = sqrt(-2 ln u_a) * (cos | sin)(2 pi u_b)
 *    (cos for even n, sin for odd n), evaluated in double.
 */
int orc_frame_bits(uint64_t seed, int64_t F, int64_t K, uint8_t *info)
{
    if (F < 0 || K < 0)
        return ORC_EINVAL;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t f = 0; f < F; f++)
        for (int64_t k = 0; k < K; k++) {
            uint32_t ctr[4] = {(uint32_t)(k / 128), (uint32_t)f, 0u, 0u}, o[4];
            orc_philox4x32_10(ctr, key, o);
            info[f * K + k] = (uint8_t)((o[(k / 32) % 4] >> (k % 32)) & 1u);
        }
    return ORC_OK;
}

int orc_frame_noise(uint64_t seed, int64_t F, int64_t N, double *z)
{
    if (F < 0 || N < 0)
        return ORC_EINVAL;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t f = 0; f < F; f++)
        for (int64_t n = 0; n < N; n++) {
            uint32_t ctr[4] = {(uint32_t)(n / 4), (uint32_t)f, 1u, 0u}, o[4];
            orc_philox4x32_10(ctr, key, o);
            int p = (int)(n % 4) / 2;
            double ua = ((double)(o[2 * p] >> 8) + 0.5) * (1.0 / 16777216.0);
            double ub = ((double)(o[2 * p + 1] >> 8) + 0.5) * (1.0 / 16777216.0);
            double rad = sqrt(-2.0 * log(ua));
            z[f * N + n] = (n % 2 == 0) ? rad * cos(two_pi * ub) : rad * sin(two_pi * ub);
        }
    return ORC_OK;
}

/*
 * BPSK over AWGN and the channel LLR (eqs. 16-17), in float:
 *   y = (1 - 2x) + sigma * z,   LLR = y * scale,  scale = 2 / sigma^2.
 */
int orc_channel(const uint8_t *cw, const float *z, int64_t n, float sigma, float scale, float *llr)
{
    if (n < 0)
        return ORC_EINVAL;
    for (int64_t k = 0; k < n; k++) {
        float y = (cw[k] & 1 ? -1.0f : 1.0f) + sigma * z[k];
        llr[k] = y * scale;
    }
    return ORC_OK;
}
