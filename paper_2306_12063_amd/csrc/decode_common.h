// Device helpers shared by the layered decode kernels (Sec. 4).
//
// Work mapping. A workgroup owns FW = G*KF frames. Its threads form G groups
// of Z threads; thread (g, r) owns check row r of every block row for the KF
// frames of group g. Rows of one block row never share a variable (each
// circulant is a permutation), so the Z threads of a group update a layer in
// parallel without conflicts; a workgroup barrier separates layers.
//
// Memory. Posteriors stay in LDS for all iterations, frame-minor: element
// (n, slot) at n*FWp + slot, so one gather address serves the KF frames of a
// thread through immediate offsets, and a wave reading consecutive rows hits
// consecutive LDS rows (the row stride is an odd number of dwords, which
// spreads them over the banks). Check messages are never stored per edge:
// each thread keeps, per frame and block row, the compressed state of its
// check row in VGPRs -- the two smallest magnitudes, the index of the
// smallest and one sign bit per edge (the single-scan form of Sec. 4).
//
// Early termination tests the exact syndrome H x = 0 of the hard decisions
// after the last layer of each iteration (eq. 21); a frame that satisfies it
// stops updating and reports the iteration count.
#pragma once

#include "ldpc_internal.h"

namespace ldpc {

// One edge of a block row, prepared for a launch's LDS layout: check row r
// reaches element base + r*FWp, minus Z*FWp once r >= thr (the cyclic wrap
// of (r + shift) mod Z). Built in LDS at kernel start; reading it from LDS
// each layer also keeps the compiler from hoisting every layer's addresses
// out of the iteration loop into registers.
struct GatherEdge {
    int base;   // (col*Z + shift) * FWp
    int thr;    // Z - shift
    int col;    // block column (weight-table index)
    int pad;
};

template <int MB, int MAXD>
__device__ __forceinline__ void build_gather_table(const Sched &sc, int FWp, GatherEdge (&tbl)[MB][MAXD])
{
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int e = 0; e < MAXD; ++e)
            if ((int)threadIdx.x == ((i * MAXD + e) & 255)) {
                GatherEdge ge{0, 1 << 30, 0, 0};
                if (i < sc.Mb && e < sc.deg[i]) {
                    const uint32_t ew = sc.edge[i][e];
                    const int col = (int)(ew >> 16), s = (int)(ew & 0xffffu);
                    ge.base = (col * sc.Z + s) * FWp;
                    ge.thr = sc.Z - s;
                    ge.col = col;
                }
                tbl[i][e] = ge;
            }
}

// LDS element (frame slot of rbase) that check row r reaches through edge ge;
// rbase = r*FWp + slot, zfw = Z*FWp.
__device__ __forceinline__ int gather_addr(const GatherEdge &ge, int r, int rbase, int zfw)
{
    return rbase + ge.base + ((r >= ge.thr) ? -zfw : 0);
}

__device__ __forceinline__ int edge_col(uint32_t ew) { return (int)(ew >> 16); }

// Loads the channel values of up to FW frames into the frame-minor layout.
template <typename TIn, typename TL, typename Conv>
__device__ __forceinline__ void load_frames(TL *Ls, const TIn *__restrict__ src, const int64_t *__restrict__ fidx,
                                            int64_t f0, int64_t F, int FW, int FWp, int N, Conv conv)
{
    for (int slot = 0; slot < FW; ++slot) {
        const int64_t fg = f0 + slot;
        if (fg >= F)
            break;
        const int64_t row = fidx ? fidx[fg] : fg;
        const TIn *p = src + row * (int64_t)N;
        for (int n = threadIdx.x; n < N; n += blockDim.x)
            Ls[n * FWp + slot] = conv(p[n]);
    }
}

// Writes hard decisions (eq. 21: a zero posterior decodes to 1) and,
// optionally, the posteriors of up to FW frames.
template <typename TL, typename TP>
__device__ __forceinline__ void store_frames(const TL *Ls, const int64_t *__restrict__ fidx, int64_t f0, int64_t F,
                                             int FW, int FWp, int N, uint8_t *__restrict__ bits,
                                             TP *__restrict__ post)
{
    for (int slot = 0; slot < FW; ++slot) {
        const int64_t fg = f0 + slot;
        if (fg >= F)
            break;
        const int64_t row = fidx ? fidx[fg] : fg;
        for (int n = threadIdx.x; n < N; n += blockDim.x) {
            const TL v = Ls[n * FWp + slot];
            bits[row * N + n] = (v > (TL)0) ? 0 : 1;
            if (post)
                post[row * N + n] = (TP)v;
        }
    }
}

// 1 if any check row owned by this thread is unsatisfied by the hard
// decisions of the frame slot addressed by rbase.
template <int MB, int MAXD, typename TL>
__device__ __forceinline__ int rows_unsatisfied(const Sched &sc, const GatherEdge (&tbl)[MB][MAXD], const TL *Ls,
                                                int r, int rbase, int zfw)
{
    int bad = 0;
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        if (i < sc.Mb) {
            const int d = sc.deg[i];
            int p = 0;
#pragma unroll
            for (int e = 0; e < MAXD; ++e)
                if (e < d)
                    p ^= (Ls[gather_addr(tbl[i][e], r, rbase, zfw)] > (TL)0) ? 0 : 1;
            bad |= p;
        }
    }
    return bad;
}

// Per-frame convergence bookkeeping after an iteration's syndrome test.
// Returns nonzero while any frame of this thread is still decoding.
template <int KF>
__device__ __forceinline__ int settle_frames(int *unsat, int slot0, int t, int max_iter, int et, bool (&act)[KF],
                                             int (&itk)[KF], int (&okk)[KF])
{
    int any = 0;
#pragma unroll
    for (int k = 0; k < KF; ++k) {
        if (act[k]) {
            const int sat = unsat[slot0 + k] == 0;
            if (t == max_iter - 1)
                okk[k] = sat;
            if (et && sat) {
                act[k] = false;
                itk[k] = t + 1;
                okk[k] = 1;
            }
        }
        any |= act[k];
    }
    return any;
}

// Kernel variants are compiled per (block rows, max degree) shape, each in
// its own object; decode_dispatch.cpp picks the smallest that fits.
template <int MB, int MAXD>
int run_decode_f32(const Sched &sc, const DecodeLaunch &lc, const float *llr, const int64_t *fidx, int64_t F,
                   int max_iter, float alpha, int et, const float *w, uint8_t *bits, float *post, int32_t *iters,
                   uint8_t *ok, hipStream_t st);

template <int MB, int MAXD>
int run_decode_i8(const Sched &sc, const DecodeLaunch &lc, const int8_t *llr, const int64_t *fidx, int64_t F,
                  int max_iter, int offset, int wq, const uint8_t *wtab, int et, uint8_t *bits, int16_t *post,
                  int32_t *iters, uint8_t *ok, hipStream_t st);

}  // namespace ldpc
