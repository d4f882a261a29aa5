// FP32 layered normalised min-sum decode kernel for gfx950 (Sec. 4,
// eqs. 18, 20, 22, 23). Compiled once per (LDPC_MB, LDPC_D) shape.
//
// Per check row and frame, one layer does:
//   Q_e = L[n_e] - R_old_e                      (eq. 22)
//   min1, min2, argmin and sign bits of Q       (single scan of eq. 23)
//   R_e = sgn_e * fl(w * (e == argmin ? min2 : min1))
//   L[n_e] = Q_e + R_e                          (eq. 20)
// with sgn_e the product of the other edges' signs. R_old is rebuilt from the
// row's compressed state; with learned weights the state keeps the raw minima
// and the old message is rebuilt with the weight of the iteration that
// produced it.
#include <math.h>

#include "decode_common.h"

namespace ldpc {
namespace {

template <int MB, int MAXD, int KF, bool LEARNED>
__global__ __launch_bounds__(kMaxThreads) void k_decode_f32(
    const Sched sc, const int G, const int FWp, const float *__restrict__ llr, const int64_t *__restrict__ fidx,
    const int64_t F, const int max_iter, const float alpha, const int et, const float *__restrict__ wt,
    uint8_t *__restrict__ bits, float *__restrict__ post, int32_t *__restrict__ iters, uint8_t *__restrict__ okv)
{
    extern __shared__ float Ls[];
    __shared__ int unsat[64];
    __shared__ GatherEdge tbl[MB][MAXD];
    const int Z = sc.Z, Mb = sc.Mb, Nb = sc.Nb;
    const int FW = G * KF;
    const int tid = threadIdx.x;
    const int g = tid / Z;
    const int r = tid - g * Z;
    const bool lane_on = g < G;
    const int slot0 = g * KF;
    const int64_t f0 = (int64_t)blockIdx.x * FW;

    build_gather_table<MB, MAXD>(sc, FWp, tbl);
    // Adding +0.0f turns a -0.0 input into +0.0, so that from here on the
    // sign bit of every value equals (value < 0), the paper's sgn with
    // sgn(-0) = +1 (-0 cannot reappear: x - x and x + (-x) round to +0).
    load_frames(Ls, llr, fidx, f0, F, FW, FWp, sc.N, [](float v) { return v + 0.0f; });
    if (tid < 64)
        unsat[tid] = 0;
    const int rbase = r * FWp + slot0;
    const int zfw = Z * FWp;

    float sm1[KF][MB], sm2[KF][MB];
    uint32_t ssg[KF][MB];   // sign bits (edge e at bit d-1-e; 1 = message negative) | argmin << 27
    bool act[KF];
    int itk[KF], okk[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) {
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            sm1[k][i] = 0.0f;
            sm2[k][i] = 0.0f;
            ssg[k][i] = 0u;
        }
        act[k] = lane_on && (f0 + slot0 + k < F);
        itk[k] = max_iter;
        okk[k] = 0;
    }
    __syncthreads();

    for (int t = 0; t < max_iter; ++t) {
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            if (i < Mb) {
                const int d = sc.deg[i];
                int ix[MAXD];
#pragma unroll
                for (int e = 0; e < MAXD; ++e)
                    if (e < d)
                        ix[e] = gather_addr(tbl[i][e], r, rbase, zfw);
                float Q[KF][MAXD];
#pragma unroll
                for (int k = 0; k < KF; ++k) {
                    if (act[k]) {
                        const uint32_t om1 = __float_as_uint(sm1[k][i]), om2 = __float_as_uint(sm2[k][i]);
                        const uint32_t osg = ssg[k][i];
                        const uint32_t oidx = osg >> 27;
#pragma unroll
                        for (int e = 0; e < MAXD; ++e) {
                            if (e < d) {
                                uint32_t mag = (oidx == (uint32_t)e) ? om2 : om1;
                                if (LEARNED)
                                    mag = __float_as_uint(
                                        (t > 0 ? wt[((t - 1) * Mb + i) * Nb + tbl[i][e].col] : 0.0f) *
                                        __uint_as_float(mag));
                                // message sign: bit d-1-e of the state moved to bit 31
                                const uint32_t ro = mag | ((osg << (32 - d + e)) & 0x80000000u);
                                Q[k][e] = Ls[ix[e] + k] - __uint_as_float(ro);
                            }
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < KF; ++k) {
                    if (act[k]) {
                        float m1 = INFINITY, m2 = INFINITY;
                        uint32_t idx = 0, neg = 0;
#pragma unroll
                        for (int e = 0; e < MAXD; ++e) {
                            if (e < d) {
                                const float a = fabsf(Q[k][e]);
                                idx = (a < m1) ? (uint32_t)e : idx;
                                m2 = __builtin_amdgcn_fmed3f(a, m1, m2);
                                m1 = fminf(m1, a);
                                // shift the sign bit of Q in from the right
                                neg = __builtin_amdgcn_alignbit(neg, __float_as_uint(Q[k][e]), 31);
                            }
                        }
                        // sign of the message to edge e: parity of all sign bits but e's own
                        const uint32_t par = (uint32_t)__popc(neg) & 1u;
                        const uint32_t parbit = par << 31;
                        const uint32_t sgm = neg ^ ((0u - par) & ((1u << d) - 1u));
                        float n1 = 0.0f, n2 = 0.0f;
                        if (!LEARNED) {
                            n1 = alpha * m1;
                            n2 = alpha * m2;
                        }
#pragma unroll
                        for (int e = 0; e < MAXD; ++e) {
                            if (e < d) {
                                uint32_t mag;
                                if (LEARNED)
                                    mag = __float_as_uint(wt[(t * Mb + i) * Nb + tbl[i][e].col] *
                                                          ((idx == (uint32_t)e) ? m2 : m1));
                                else
                                    mag = __float_as_uint((idx == (uint32_t)e) ? n2 : n1);
                                const uint32_t rn = mag | ((__float_as_uint(Q[k][e]) ^ parbit) & 0x80000000u);
                                Ls[ix[e] + k] = Q[k][e] + __uint_as_float(rn);
                            }
                        }
                        sm1[k][i] = LEARNED ? m1 : n1;
                        sm2[k][i] = LEARNED ? m2 : n2;
                        ssg[k][i] = sgm | (idx << 27);
                    }
                }
            }
            __syncthreads();
        }
        if (et || t == max_iter - 1) {
#pragma unroll
            for (int k = 0; k < KF; ++k)
                if (act[k] && rows_unsatisfied<MB, MAXD>(sc, tbl, Ls, r, rbase + k, zfw))
                    unsat[slot0 + k] = 1;
            __syncthreads();
            const int any = settle_frames<KF>(unsat, slot0, t, max_iter, et, act, itk, okk);
            __syncthreads();
            if (tid < FW)
                unsat[tid] = 0;
            if (et && !__syncthreads_or(any))
                break;
        }
    }
    __syncthreads();
    if (lane_on && r == 0) {
#pragma unroll
        for (int k = 0; k < KF; ++k) {
            const int64_t fg = f0 + slot0 + k;
            if (fg < F) {
                const int64_t row = fidx ? fidx[fg] : fg;
                iters[row] = itk[k];
                if (okv)
                    okv[row] = (uint8_t)okk[k];
            }
        }
    }
    store_frames(Ls, fidx, f0, F, FW, FWp, sc.N, bits, post);
}

}  // namespace

template <int MB, int MAXD>
int run_decode_f32(const Sched &sc, const DecodeLaunch &lc, const float *llr, const int64_t *fidx, int64_t F,
                   int max_iter, float alpha, int et, const float *w, uint8_t *bits, float *post, int32_t *iters,
                   uint8_t *ok, hipStream_t st)
{
    const dim3 grid((unsigned)((F + lc.FW - 1) / lc.FW)), block(lc.threads);
#define LDPC_LAUNCH(KF, LEARNED)                                                                                \
    hipLaunchKernelGGL((k_decode_f32<MB, MAXD, KF, LEARNED>), grid, block, lc.lds, st, sc, lc.G, lc.FWp, llr, \
                       fidx, F, max_iter, alpha, et, w, bits, post, iters, ok)
    if (lc.KF == 2) {
        if (w)
            LDPC_LAUNCH(2, true);
        else
            LDPC_LAUNCH(2, false);
    } else {
        if (w)
            LDPC_LAUNCH(1, true);
        else
            LDPC_LAUNCH(1, false);
    }
#undef LDPC_LAUNCH
    return check_launch("decode_f32");
}

template int run_decode_f32<LDPC_MB, LDPC_D>(const Sched &, const DecodeLaunch &, const float *, const int64_t *,
                                             int64_t, int, float, int, const float *, uint8_t *, float *, int32_t *,
                                             uint8_t *, hipStream_t);

}  // namespace ldpc
