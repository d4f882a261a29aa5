// Saturating fixed-point layered min-sum decode kernel for gfx950: int8
// channel LLRs and check messages, int16 posteriors (the fixed-point decoder
// of Sec. 5, saturating where the paper's C code wraps around). Compiled
// once per (LDPC_MB, LDPC_D) shape.
//
// Per check row and frame, one layer does:
//   Q_e = sat16(L[n_e] - R_old_e)               (eq. 22)
//   a_e = min(|Q_e|, 127); min1, min2, argmin and sign bits of Q
//   magnitude: OMS max(m - offset, 0) (MODE 0), or min(127, (wq*m + 8) >> 4)
//              with a scalar (MODE 1) or per-(iteration, layer, column)
//              weight (MODE 2), m = min2 at the argmin and min1 elsewhere
//   R_e = sgn_e * magnitude,  L[n_e] = sat16(Q_e + R_e)   (eq. 20)
// Saturation is symmetric (+-32767), so negating a value never saturates.
#include "decode_common.h"

namespace ldpc {
namespace {

__device__ __forceinline__ int sat16(int x) { return min(max(x, -32767), 32767); }

__device__ __forceinline__ int norm_mag(int wq, int m) { return min(127, (wq * m + 8) >> 4); }

template <int MB, int MAXD, int KF, int MODE>
__global__ __launch_bounds__(kMaxThreads) void k_decode_i8(
    const Sched sc, const int G, const int FWp, const int8_t *__restrict__ llr, const int64_t *__restrict__ fidx,
    const int64_t F, const int max_iter, const int offset, const int wq, const uint8_t *__restrict__ wtab,
    const int et, uint8_t *__restrict__ bits, int16_t *__restrict__ post, int32_t *__restrict__ iters,
    uint8_t *__restrict__ okv)
{
    extern __shared__ int16_t L16[];
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
    load_frames(L16, llr, fidx, f0, F, FW, FWp, sc.N, [](int8_t v) { return (int16_t)v; });
    if (tid < 64)
        unsat[tid] = 0;
    const int rbase = r * FWp + slot0;
    const int zfw = Z * FWp;

    // Compressed row state: smg = m1 | m2 << 8 (output magnitudes in modes
    // 0/1, raw minima in mode 2); ssg = sign bits (1 = negative) | argmin << 27.
    uint32_t smg[KF][MB], ssg[KF][MB];
    bool act[KF];
    int itk[KF], okk[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) {
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            smg[k][i] = 0u;
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
                const int li = i;
                const int d = sc.deg[i];
                int ix[MAXD];
#pragma unroll
                for (int e = 0; e < MAXD; ++e)
                    if (e < d)
                        ix[e] = gather_addr(tbl[i][e], r, rbase, zfw);
                int Q[KF][MAXD];
#pragma unroll
                for (int k = 0; k < KF; ++k) {
                    if (act[k]) {
                        const int om1 = (int)(smg[k][i] & 0xffu), om2 = (int)((smg[k][i] >> 8) & 0xffu);
                        const uint32_t osg = ssg[k][i];
                        const int oidx = (int)(osg >> 27);
#pragma unroll
                        for (int e = 0; e < MAXD; ++e) {
                            if (e < d) {
                                int mag = (e == oidx) ? om2 : om1;
                                if (MODE == 2)
                                    mag = t > 0 ? norm_mag(wtab[((t - 1) * Mb + li) * Nb + tbl[i][e].col], mag)
                                                : 0;
                                const int ro = ((osg >> e) & 1u) ? -mag : mag;
                                Q[k][e] = sat16((int)L16[ix[e] + k] - ro);
                            }
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < KF; ++k) {
                    if (act[k]) {
                        int m1 = 1 << 20, m2 = 1 << 20, idx = 0;
                        uint32_t neg = 0;
#pragma unroll
                        for (int e = 0; e < MAXD; ++e) {
                            if (e < d) {
                                const int q = Q[k][e];
                                const int a = min(q < 0 ? -q : q, 127);
                                if (a < m1) {
                                    m2 = m1;
                                    m1 = a;
                                    idx = e;
                                } else if (a < m2) {
                                    m2 = a;
                                }
                                neg |= (uint32_t)(q < 0) << e;
                            }
                        }
                        const uint32_t par = (uint32_t)__popc(neg) & 1u;
                        const uint32_t sgm = neg ^ ((0u - par) & ((1u << d) - 1u));
                        int n1 = m1, n2 = m2;
                        if (MODE == 0) {
                            n1 = max(m1 - offset, 0);
                            n2 = max(m2 - offset, 0);
                        } else if (MODE == 1) {
                            n1 = norm_mag(wq, m1);
                            n2 = norm_mag(wq, m2);
                        }
#pragma unroll
                        for (int e = 0; e < MAXD; ++e) {
                            if (e < d) {
                                int mag;
                                if (MODE == 2)
                                    mag = norm_mag(wtab[(t * Mb + li) * Nb + tbl[i][e].col],
                                                   (e == idx) ? m2 : m1);
                                else
                                    mag = (e == idx) ? n2 : n1;
                                const int rn = ((sgm >> e) & 1u) ? -mag : mag;
                                L16[ix[e] + k] = (int16_t)sat16(Q[k][e] + rn);
                            }
                        }
                        smg[k][i] = (uint32_t)n1 | ((uint32_t)n2 << 8);
                        ssg[k][i] = sgm | ((uint32_t)idx << 27);
                    }
                }
            }
            __syncthreads();
        }
        if (et || t == max_iter - 1) {
#pragma unroll
            for (int k = 0; k < KF; ++k)
                if (act[k] && rows_unsatisfied<MB, MAXD>(sc, tbl, L16, r, rbase + k, zfw))
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
    store_frames(L16, fidx, f0, F, FW, FWp, sc.N, bits, post);
}

}  // namespace

template <int MB, int MAXD>
int run_decode_i8(const Sched &sc, const DecodeLaunch &lc, const int8_t *llr, const int64_t *fidx, int64_t F,
                  int max_iter, int offset, int wq, const uint8_t *wtab, int et, uint8_t *bits, int16_t *post,
                  int32_t *iters, uint8_t *ok, hipStream_t st)
{
    const dim3 grid((unsigned)((F + lc.FW - 1) / lc.FW)), block(lc.threads);
#define LDPC_LAUNCH(KF, MODE)                                                                                    \
    hipLaunchKernelGGL((k_decode_i8<MB, MAXD, KF, MODE>), grid, block, lc.lds, st, sc, lc.G, lc.FWp, llr, fidx, \
                       F, max_iter, offset, wq, wtab, et, bits, post, iters, ok)
    const int mode = wtab ? 2 : (wq > 0 ? 1 : 0);
    if (lc.KF == 2) {
        if (mode == 2)
            LDPC_LAUNCH(2, 2);
        else if (mode == 1)
            LDPC_LAUNCH(2, 1);
        else
            LDPC_LAUNCH(2, 0);
    } else {
        if (mode == 2)
            LDPC_LAUNCH(1, 2);
        else if (mode == 1)
            LDPC_LAUNCH(1, 1);
        else
            LDPC_LAUNCH(1, 0);
    }
#undef LDPC_LAUNCH
    return check_launch("decode_i8");
}

template int run_decode_i8<LDPC_MB, LDPC_D>(const Sched &, const DecodeLaunch &, const int8_t *, const int64_t *,
                                            int64_t, int, int, int, const uint8_t *, int, uint8_t *, int16_t *,
                                            int32_t *, uint8_t *, hipStream_t);

}  // namespace ldpc
