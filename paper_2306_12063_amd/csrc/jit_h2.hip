// Fixed-point layered min-sum with two frames per lane in packed FP16,
// specialised for one code at run time (prelude of jit_decode.hip, with
// LDPC_G frame PAIRS per workgroup and LDPC_KF 1).
//
// The fixed-point path works on integers of magnitude at most 127 * (1 +
// column weight) (int8 messages, |L| bounded by the channel value plus the
// messages of its column), so for codes whose column weight is at most 15
// every value is below 2048 and exact in FP16. One 32-bit register then
// holds the same quantity for two frames: posteriors in LDS (element (n, p)
// at PAD + n*FWP + p holds frames 2p, 2p+1), the message of every edge of
// the thread's rows, and all per-edge arithmetic, which is the update of
// jit_decode.hip on pairs:
//   Q = L - R (v_pk_add_f16);  |Q| = Q & 0x7fff7fff;  min1/min2 by
//   three-input IEEE minimum/maximum (v_pk_minimum3_f16 / _maximum3_f16),
//   two edges per step;  sign parity = XOR of the Q words (bits 15, 31);
//   u = clamp(min1 + 1 - |Q|, 0, 1), which is 1 where |Q| == min1 and 0
//   elsewhere because every value is an integer (one v_pk_add_f16 with
//   clamp);  magnitude = u * (n2s - n1s) + n1s (v_pk_fma_f16, exact), with
//   n1s, n2s the row's two magnitudes carrying the parity in their sign
//   bits;  R = (Q & 0x80008000) ^ magnitude;  L = Q + R (v_pk_add_f16).
// A frame that stops (early termination) has its outputs written at once;
// its half of the pair then keeps being updated but is no longer tested or
// written, so the per-edge work needs no mask. Per-row magnitude rules (offset, or wq/16 in
// FP32) are those of the int8 definition; results are bit-identical to it.

#ifndef LDPC_PACKED
#define LDPC_PACKED 0
#endif

typedef unsigned char u8;
typedef unsigned int u32;
typedef long long i64;
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef unsigned short u2 __attribute__((ext_vector_type(2)));

constexpr int Z = LDPC_Z, MB = LDPC_MB, NB = LDPC_NB, N = LDPC_N, MAXD = LDPC_MAXD;
constexpr int G = LDPC_G, FWP = LDPC_FWP;
constexpr int FW = 2 * G;
constexpr int ZFW = Z * FWP;
constexpr int PAD = ZFW;

constexpr int row_edges()
{
    int s = 0;
    for (int i = 0; i < MB; ++i)
        s += kDeg[i];
    return s;
}
constexpr int edge_off(int i)
{
    int s = 0;
    for (int k = 0; k < i; ++k)
        s += kDeg[k];
    return s;
}
constexpr int ED = row_edges();

template <int V>
struct Int {
    static constexpr int value = V;
};
template <int I, int Nn, class Fn>
__device__ __forceinline__ void static_for(Fn &&f)
{
    if constexpr (I < Nn) {
        f(Int<I>());
        static_for<I + 1, Nn>(f);
    }
}

__device__ __forceinline__ int gather_b(int i, int e, int r, int rbn_b, int rbw_b)
{
    return ((r >= Z - kShift[i][e]) ? rbw_b : rbn_b) + (kCol[i][e] * Z + kShift[i][e]) * FWP * 4;
}

__device__ __forceinline__ h2 H(u32 x) { return __builtin_bit_cast(h2, x); }
__device__ __forceinline__ u2 V(u32 x) { return __builtin_bit_cast(u2, x); }
__device__ __forceinline__ u32 W(h2 x) { return __builtin_bit_cast(u32, x); }
__device__ __forceinline__ u32 W(u2 x) { return __builtin_bit_cast(u32, x); }

__device__ __forceinline__ u32 ldb(const u32 *Ls, int b) { return *(const u32 *)((const char *)Ls + b); }
__device__ __forceinline__ void stb(u32 *Ls, int b, u32 v) { *(u32 *)((char *)Ls + b) = v; }

// hard decisions of a pair (bit 0: frame 2p, bit 16: frame 2p+1): 1 where
// the value is <= 0, i.e. where its bits as int16 are <= 0 (no -0 occurs)
// XOR of v[0..D): two operands per v_bitop3_b32 (truth table 0x96 =
// a ^ b ^ c) instead of one per v_xor_b32
template <int D>
__device__ __forceinline__ u32 xor_bits(const u32 *v)
{
    u32 p = v[0];
#pragma unroll
    for (int e = 1; e + 1 < D; e += 2)
        p = __builtin_amdgcn_bitop3_b32(p, v[e], v[e + 1], 0x96);
    if constexpr (D % 2 == 0)
        p ^= v[D - 1];
    return p;
}

// Hard decisions of both halves as bits 15 and 31: (x - 1) on each 16-bit
// lane has its top bit set exactly where the FP16 value is <= 0 (posteriors
// are never -0: the channel values are converted from integers, and in
// round-to-nearest a sum or difference of values that are not -0 is not
// -0), so a row's two parities are bits 15 and 31 of the XOR of these
// words, taken three operands per v_bitop3_b32.
__device__ __forceinline__ u32 hb_word2(u32 x)
{
    const u2 one = {1, 1};
    return W(V(x) - one);
}

__device__ __forceinline__ float norm_mag(float w, float m)
{
    return __builtin_fminf(127.0f, __builtin_floorf((w * m + 8.0f) * 0.0625f));
}

// Occupancy target chosen by the layout tuner (waves per SIMD; 0: the
// compiler's choice).
#if LDPC_WAVES_HINT
#define LDPC_OCCUPANCY __attribute__((amdgpu_waves_per_eu(LDPC_WAVES_HINT)))
#else
#define LDPC_OCCUPANCY
#endif

extern "C" __global__ __launch_bounds__(LDPC_THREADS) LDPC_OCCUPANCY void LDPC_KERNEL(
    const signed char *__restrict__ llr, const i64 *__restrict__ fidx, const i64 Fmax, const int max_iter,
    const float alpha, const int offset, const int wq, const int et, const u8 *__restrict__ wt,
    u8 *__restrict__ bits, short *__restrict__ post, int *__restrict__ iters, u8 *__restrict__ okv,
    const i64 *__restrict__ Fdev)
{
    const i64 F = Fdev ? (*Fdev < Fmax ? *Fdev : Fmax) : Fmax;
    if ((i64)blockIdx.x * FW >= F)
        return;
    __shared__ u32 Ls[PAD + N * FWP];
    __shared__ int unsat[FW];
    const int tid = threadIdx.x;
    // lanes interleave the workgroup's frame groups: a wave holds about
    // 64 / G consecutive rows of each, so no two of its lanes read rows of
    // one block column 64 apart (the same LDS bank)
    const int g = tid % G;
    const int r = tid / G;
    const bool lane_on = tid < G * Z;
    const i64 f0 = (i64)blockIdx.x * FW;
    _Float16 *Lh = (_Float16 *)Ls;
    // Channel values into LDS (frame slot s in half s & 1 of pair s >> 1; a
    // slot past F holds zeros). The FW frames are one flat range of FW*N
    // values; each thread puts up to 16 loads in flight before it waits for
    // the first, so a workgroup pays one or two round trips to HBM before its
    // first layer, not one per frame and pass.
#if LDPC_MODE == 2
    // weight table: the weights of iterations t (buffer t & 1) and t + 1 in
    // LDS; row i's weights at i*WROW + e as a 16-bit pair (the same weight
    // for both frames), 16-byte aligned rows read as broadcast loads of four.
    // The next iteration's weights are loaded into registers at its
    // predecessor's first layer (fetch) and stored to LDS at its last layer
    // (put), so the round trip to HBM overlaps the layers; the loads are
    // unconditional (an entry without an edge reads element 0, not stored).
    constexpr int WROW = (MAXD + 3) / 4 * 4;
    __shared__ __attribute__((aligned(16))) u32 Wst[2][MB * WROW];
    constexpr int NWT = (MB * WROW + LDPC_THREADS - 1) / LDPC_THREADS;
    u32 wreg[NWT];
    bool wok[NWT];
    auto fetch_weights = [&](int t) {
#pragma unroll
        for (int j = 0; j < NWT; ++j) {
            const int k = tid + j * LDPC_THREADS;
            const bool in = k < MB * WROW;
            const int i = in ? k / WROW : 0, e = in ? k - i * WROW : 0;
            wok[j] = in && e < kDeg[i];
            wreg[j] = wt[wok[j] ? (i64)t * (MB * NB) + i * NB + kCol[i][e] : 0];
        }
    };
    auto put_weights = [&](int t) {
#pragma unroll
        for (int j = 0; j < NWT; ++j)
            if (wok[j])
                Wst[t & 1][tid + j * LDPC_THREADS] = wreg[j] | (wreg[j] << 16);
    };
    fetch_weights(0);   // its round trip overlaps the channel values'
#endif
    __shared__ i64 frow[FW];   // row of each frame slot's buffers, -1 past F
    __shared__ int conv[FW];
    if (tid < FW) {
        const i64 fg = f0 + tid;
        frow[tid] = fg < F ? (fidx ? fidx[fg] : fg) : (i64)-1;
        unsat[tid] = 0;
        conv[tid] = 0;
    }
    __syncthreads();
    {
        constexpr int TOT = FW * N;
        constexpr int PER = (TOT + LDPC_THREADS - 1) / LDPC_THREADS;
        constexpr int CH = PER < 16 ? PER : 16;
        for (int j0 = 0; j0 < PER; j0 += CH) {
            signed char v[CH];
            int dst[CH];
            // loads are unconditional (a value past the range or of a slot
            // past F is read from frame slot 0, which exists) so that none
            // waits for another; the store below zeroes the latter
            bool real[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int k = (j0 + j) * LDPC_THREADS + tid;
                const int kk = k < TOT ? k : 0;
                const int slot = kk / N, n = kk - slot * N;
                const i64 row = frow[slot];
                v[j] = llr[(row >= 0 ? row : frow[0]) * (i64)N + n];
                real[j] = row >= 0;
                dst[j] = k < TOT ? 2 * (PAD + n * FWP + (slot >> 1)) + (slot & 1) : -1;
            }
#pragma unroll
            for (int j = 0; j < CH; ++j)
                if (dst[j] >= 0)
                    Lh[dst[j]] = real[j] ? (_Float16)(float)v[j] : (_Float16)0.0f;
        }
    }
    const bool act0 = lane_on && f0 + 2 * g < F, act1 = lane_on && f0 + 2 * g + 1 < F;
    bool act[2] = {act0, act1};
    int itk[2] = {max_iter, max_iter}, okk[2] = {0, 0};
    u32 R[ED];
#pragma unroll
    for (int e = 0; e < ED; ++e)
        R[e] = 0u;
    const u32 beta = W((h2){(_Float16)(float)offset, (_Float16)(float)offset});
    const float wqf = (float)wq;
#if LDPC_MODE == 2
    put_weights(0);
#endif
    __syncthreads();

    // outputs of frame slot `slot` (bits, posteriors) from LDS, by the whole
    // workgroup; wide: four bits per 32-bit store (after the iterations only:
    // inside them its registers would spill)
    auto write_frame = [&](int slot, bool wide) {
        const i64 row = frow[slot];
        if (row < 0)
            return;
        const int hsel = slot & 1, pair = slot >> 1;
#if LDPC_PACKED
        constexpr int NB8 = (N + 7) / 8;
        for (int b = tid; b < NB8; b += LDPC_THREADS) {
            u32 byte = 0;
#pragma unroll
            for (int tt = 0; tt < 8; ++tt)
                if (8 * b + tt < N)
                    byte |= ((float)Lh[2 * (PAD + (8 * b + tt) * FWP + pair) + hsel] > 0.0f ? 0u : 1u) << tt;
            bits[row * NB8 + b] = (u8)byte;
        }
        if (post)
            for (int n = tid; n < N; n += LDPC_THREADS)
                post[row * N + n] = (short)(float)Lh[2 * (PAD + n * FWP + pair) + hsel];
#else
        // wide, N a multiple of 4 and the caller's buffer 4-byte aligned: a
        // thread writes four bits as one 32-bit word
        if (wide && N % 4 == 0 && ((unsigned long long)bits & 3) == 0) {
            for (int b = tid; b < N / 4; b += LDPC_THREADS) {
                u32 w = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    w |= ((float)Lh[2 * (PAD + (4 * b + q) * FWP + pair) + hsel] > 0.0f ? 0u : 1u) << (8 * q);
                *(u32 *)(bits + row * N + 4 * b) = w;
            }
        } else {
            for (int n = tid; n < N; n += LDPC_THREADS)
                bits[row * N + n] = (float)Lh[2 * (PAD + n * FWP + pair) + hsel] > 0.0f ? 0 : 1;
        }
        if (post)
            for (int n = tid; n < N; n += LDPC_THREADS)
                post[row * N + n] = (short)(float)Lh[2 * (PAD + n * FWP + pair) + hsel];
#endif
    };

    for (int t = 0; t < max_iter; ++t) {
        const bool check = et || (t == max_iter - 1);
        const bool live = lane_on && (f0 + 2 * g < F);   // the pair holds at least one frame
        u32 lastbad = 0;
        static_for<0, MB>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int d = kDeg[i];
            constexpr int eo = edge_off(i);
#if LDPC_MODE == 2
            // the next iteration's weights: loads issued here, stored to
            // their buffer (last read in iteration t - 1) at the last layer
            if constexpr (i == 0)
                if (t + 1 < max_iter)
                    fetch_weights(t + 1);
#endif
            int rr = r;
            if constexpr (i >= LDPC_HOIST)
                asm volatile("" : "+v"(rr));
            const int rbw = (rr * FWP + g) * 4, rbn = rbw + PAD * 4;
            if (live) {
                int ix[MAXD];
                u32 Q[MAXD];
#pragma unroll
                for (int e = 0; e < d; ++e) {
                    ix[e] = gather_b(i, e, rr, rbn, rbw);
                    Q[e] = W(H(ldb(Ls, ix[e])) - H(R[eo + e]));
                }
                // magnitudes; min1/min2 by IEEE minimum/maximum (no NaN,
                // no -0: non-negative values), two edges at a time
                h2 A[MAXD];
#pragma unroll
                for (int e = 0; e < d; ++e)
                    A[e] = H(Q[e] & 0x7fff7fffu);
                h2 m1 = __builtin_elementwise_minimum(A[0], A[1]);
                h2 m2 = __builtin_elementwise_maximum(A[0], A[1]);
#pragma unroll
                for (int e = 2; e + 1 < d; e += 2) {
                    const h2 lo = __builtin_elementwise_minimum(A[e], A[e + 1]);
                    const h2 hi = __builtin_elementwise_maximum(A[e], A[e + 1]);
                    m2 = __builtin_elementwise_minimum(__builtin_elementwise_minimum(m2, hi),
                                                       __builtin_elementwise_maximum(m1, lo));
                    m1 = __builtin_elementwise_minimum(m1, lo);
                }
                if constexpr (d % 2 == 1) {
                    m2 = __builtin_elementwise_minimum(m2, __builtin_elementwise_maximum(m1, A[d - 1]));
                    m1 = __builtin_elementwise_minimum(m1, A[d - 1]);
                }
                const u32 par = xor_bits<d>(Q) & 0x80008000u;
                const h2 cap = {(_Float16)127.0f, (_Float16)127.0f};
                const h2 c1 = __builtin_elementwise_minimum(m1, cap), c2 = __builtin_elementwise_minimum(m2, cap);
#if LDPC_MODE == 2
                // a weight per edge: magnitude min(127, (wq * m + 8) >> 4) on
                // 16-bit integer lanes, m = min2 at the row's minimum and min1
                // elsewhere; the clipped minima as integers (c + 1024 has the
                // integer c in its low ten bits)
                const h2 k1024 = {(_Float16)1024.0f, (_Float16)1024.0f};
                const u32 C1 = W(c1 + k1024) & 0x03ff03ffu, C2 = W(c2 + k1024) & 0x03ff03ffu;
                const u2 dC = V(C1) - V(C2), eight = {8, 8}, c127 = {127, 127};
                u32 one_w = 0x00010001u;
                asm volatile("" : "+v"(one_w));   // keeps min(d, 1) * dC as one multiply-add, not two selects
                const u2 one_u = V(one_w);
                // -1024, or +1024 in a half whose parity is odd: adding it to
                // the (signed) 1024 + magnitude leaves the signed magnitude
                const u32 ybias = 0xe400e400u ^ par;
                const uint4 *wrow = (const uint4 *)&Wst[t & 1][i * WROW];
                u32 bad = 0, hw = 0;
#pragma unroll
                for (int e = 0; e < d; ++e) {
                    const uint4 w4 = wrow[e / 4];
                    const u32 we = (e % 4 == 0) ? w4.x : (e % 4 == 1) ? w4.y : (e % 4 == 2) ? w4.z : w4.w;
                    const u2 c = __builtin_elementwise_min(V(W(A[e])) - V(W(m1)), one_u);   // 0 at the minimum
                    const u2 ms = c * dC + V(C2);
                    const u2 mg = __builtin_elementwise_min((V(we) * ms + eight) >> 4, c127);
                    const u32 mag = W(H(W(mg) | 0x64006400u | par) + H(ybias));
                    const u32 rv = (Q[e] & 0x80008000u) ^ mag;
                    R[eo + e] = rv;
#else
                h2 n1, n2;
#if LDPC_MODE == 0
                {
                    const h2 z = {(_Float16)0.0f, (_Float16)0.0f};
                    n1 = __builtin_elementwise_maximum(c1 - H(beta), z);
                    n2 = __builtin_elementwise_maximum(c2 - H(beta), z);
                }
#else
                n1 = (h2){(_Float16)norm_mag(wqf, (float)c1.x), (_Float16)norm_mag(wqf, (float)c1.y)};
                n2 = (h2){(_Float16)norm_mag(wqf, (float)c2.x), (_Float16)norm_mag(wqf, (float)c2.y)};
#endif
                // the parity in the magnitudes' sign bits; n2s - n1s is exact
                // (integers below 128 of one sign)
                const h2 n1s = H(W(n1) | par), dl = H(W(n2) | par) - n1s;
                const h2 one_h = {(_Float16)1.0f, (_Float16)1.0f}, zero_h = {(_Float16)0.0f, (_Float16)0.0f};
                const h2 m1p1 = m1 + one_h;
                u32 bad = 0, hw = 0;
#pragma unroll
                for (int e = 0; e < d; ++e) {
                    const h2 u = __builtin_elementwise_min(__builtin_elementwise_max(m1p1 - A[e], zero_h), one_h);
                    const u32 rv = (Q[e] & 0x80008000u) ^ W(__builtin_elementwise_fma(u, dl, n1s));
                    R[eo + e] = rv;
#endif
                    const u32 lv = W(H(Q[e]) + H(rv));
                    stb(Ls, ix[e], lv);
                    if (i == MB - 1) {   // row parities of the hard decisions, two edges at a time
                        if (e & 1)
                            bad = __builtin_amdgcn_bitop3_b32(bad, hw, hb_word2(lv), 0x96);
                        else
                            hw = hb_word2(lv);
                    }
                }
                if (i == MB - 1)
                    lastbad = (d & 1 ? bad ^ hw : bad) & 0x80008000u;
            }
#if LDPC_MODE == 2
            if constexpr (i == MB - 1)
                if (t + 1 < max_iter)
                    put_weights(t + 1);
#endif
            __syncthreads();
        });
        if (check) {
            // a failing row of the last block row decides a frame at once;
            // the check pass runs for the frames whose last block row is
            // satisfied (marking a frame while another thread still reads
            // its mark is harmless: it is unsatisfied either way)
            if (act[0] && (lastbad & 0x8000u))
                unsat[2 * g] = 1;
            if (act[1] && (lastbad & 0x80000000u))
                unsat[2 * g + 1] = 1;
            __syncthreads();
            const bool need0 = act[0] && unsat[2 * g] == 0, need1 = act[1] && unsat[2 * g + 1] == 0;
            u32 bad = 0;
            if (need0 || need1) {
                static_for<0, MB - 1>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    int rr = r;
                    if constexpr (i >= LDPC_HOIST)
                        asm volatile("" : "+v"(rr));
                    const int rbw = (rr * FWP + g) * 4, rbn = rbw + PAD * 4;
                    u32 w[kDeg[i]];
#pragma unroll
                    for (int e = 0; e < kDeg[i]; ++e)
                        w[e] = hb_word2(ldb(Ls, gather_b(i, e, rr, rbn, rbw)));
                    bad |= xor_bits<kDeg[i]>(w) & 0x80008000u;
                });
                if (need0 && (bad & 0x8000u))
                    unsat[2 * g] = 1;
                if (need1 && (bad & 0x80000000u))
                    unsat[2 * g + 1] = 1;
            }
            __syncthreads();
            int any = 0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (act[k]) {
                    const int sat = unsat[2 * g + k] == 0;
                    if (t == max_iter - 1)
                        okk[k] = sat;
                    if (et && sat) {
                        act[k] = false;
                        itk[k] = t + 1;
                        okk[k] = 1;
                        if (r == 0)
                            conv[2 * g + k] = 1;
                    }
                }
                any |= act[k];
            }
            __syncthreads();
            if (tid < FW)
                unsat[tid] = 0;
            // frames that stopped in this iteration: outputs now (their
            // halves are not written back later)
            for (int slot = 0; slot < FW; ++slot)
                if (conv[slot] == 1)
                    write_frame(slot, false);
            __syncthreads();
            if (tid < FW && conv[tid] == 1)
                conv[tid] = 2;
            if (et && !__syncthreads_or(any))
                break;
        }
    }
    __syncthreads();
    if (lane_on && r == 0) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const i64 fg = f0 + 2 * g + k;
            if (fg < F) {
                const i64 row = fidx ? fidx[fg] : fg;
                iters[row] = itk[k];
                if (okv)
                    okv[row] = (u8)okk[k];
            }
        }
    }
    for (int slot = 0; slot < FW; ++slot)
        if (conv[slot] == 0)
            write_frame(slot, true);
}
