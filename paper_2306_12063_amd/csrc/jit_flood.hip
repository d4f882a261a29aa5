// Flooding (two-phase) min-sum decode kernel, specialised for one code at
// run time (hipRTC) with the prelude of jit_decode.hip. Each iteration
// (eqs. 18-23 without the layered interleaving of Sec. 4):
//   check phase: every check row of every block row reads the posteriors
//     Z of the previous iteration: Q_e = Z[n_e] - R_e (eq. 22), and takes the
//     new message R_e from the min1/min2/sign-parity scan (eq. 23);
//   variable phase: Z[n] = Z0[n] + sum of the new messages at n (eq. 20),
//     added block row by block row in ascending order (the first block row
//     that has column j starts from the channel value Z0);
//   then the exact syndrome test of the hard decisions (eq. 21).
// Work mapping, message registers, addressing, fixed-point-as-FP32 and
// sign conventions are those of jit_decode.hip. LDS holds two arrays of the
// same layout: the posteriors Z at PAD + n*FWP + slot, and the channel
// values Z0 at ZOFF + PAD + n*FWP + slot, so both are reached from one
// gather address. The check phase needs no barrier between block rows (Z
// is only read); one barrier separates it from the variable phase, whose
// block rows are separated by barriers (a variable is updated once per
// block row).

typedef unsigned char u8;
typedef unsigned int u32;
typedef long long i64;

constexpr int Z = LDPC_Z, MB = LDPC_MB, NB = LDPC_NB, N = LDPC_N, MAXD = LDPC_MAXD;
constexpr int G = LDPC_G, KF = LDPC_KF, FWP = LDPC_FWP;
constexpr int FW = G * KF;
constexpr int ZFW = Z * FWP;
constexpr int PAD = ZFW;
constexpr int ZOFF = PAD + N * FWP;   // elements from Z to Z0

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

// true if block row i is the first (lowest) block row with an edge in block
// column j
constexpr bool first_in_column(int i, int j)
{
    for (int k = 0; k < i; ++k)
        for (int e = 0; e < kDeg[k]; ++e)
            if (kCol[k][e] == j)
                return false;
    return true;
}

#if LDPC_PATH == 0
typedef float TP;
typedef float TIn;
#else
typedef short TP;
typedef signed char TIn;
#endif

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

// byte address of the posterior that check row r reaches through edge e of
// block row i (bases rbn = rb + PAD, rbw = rb, in bytes)
__device__ __forceinline__ int gather_b(int i, int e, int r, int rbn_b, int rbw_b)
{
    return ((r >= Z - kShift[i][e]) ? rbw_b : rbn_b) + (kCol[i][e] * Z + kShift[i][e]) * FWP * 4;
}

// XOR of the bit patterns of v[0..D): two operands per v_bitop3_b32 (truth
// table 0x96 = a ^ b ^ c) instead of one per v_xor_b32
__device__ __forceinline__ u32 bits_of(float v) { return __float_as_uint(v); }
__device__ __forceinline__ u32 bits_of(u32 v) { return v; }
template <int D, class T>
__device__ __forceinline__ u32 xor_bits(const T *v)
{
    u32 p = bits_of(v[0]);
#pragma unroll
    for (int e = 1; e + 1 < D; e += 2)
        p = __builtin_amdgcn_bitop3_b32(p, bits_of(v[e]), bits_of(v[e + 1]), 0x96);
    if constexpr (D % 2 == 0)
        p ^= bits_of(v[D - 1]);
    return p;
}

__device__ __forceinline__ int hard_bit(float v) { return v > 0.0f ? 0 : 1; }
// Hard decision as bit 31 of a word: bits(v) - 1 has bit 31 set exactly
// where v <= 0 (+0 -> 0xffffffff, negative values keep their sign bit,
// positive ones lose nothing). Posteriors are never -0: the load maps -0 to
// +0, and in round-to-nearest a sum or difference of values that are not -0
// is not -0. The parity of a row's hard decisions is then bit 31 of the XOR
// of these words, taken three operands per v_bitop3_b32.
__device__ __forceinline__ u32 hb_word(float v) { return __float_as_uint(v) - 1u; }


__device__ __forceinline__ float ldb(const float *Ls, int b) { return *(const float *)((const char *)Ls + b); }

__device__ __forceinline__ void stb(float *Ls, int b, float v) { *(float *)((char *)Ls + b) = v; }

#if LDPC_PATH == 1
__device__ __forceinline__ float norm_mag(float w, float m)
{
    return __builtin_fminf(127.0f, __builtin_floorf((w * m + 8.0f) * 0.0625f));
}
#endif

extern "C" __global__ __launch_bounds__(LDPC_THREADS) void LDPC_KERNEL(
    const TIn *__restrict__ llr, const i64 Fmax, const int max_iter, const float alpha, const int offset,
    const int wq, const int et, u8 *__restrict__ bits, TP *__restrict__ post, int *__restrict__ iters,
    u8 *__restrict__ okv)
{
    const i64 F = Fmax;
    if ((i64)blockIdx.x * FW >= F)
        return;
    __shared__ float Ls[2 * ZOFF];
    __shared__ int unsat[FW];
    const int tid = threadIdx.x;
    const int g = tid / Z;
    const int r = tid - g * Z;
    const bool lane_on = g < G;
    const int slot0 = g * KF;
    const int rb = r * FWP + slot0;
    const i64 f0 = (i64)blockIdx.x * FW;

    // channel values into both arrays (-0.0 -> +0.0 as in jit_decode.hip):
    // the workgroup's frames are one flat range, up to 16 loads per thread in
    // flight before the first is waited for (a value past F is read from the
    // workgroup's first frame, which exists, and dropped)
    {
        const i64 nval = (F - f0 < FW ? F - f0 : (i64)FW) * (i64)N;
        constexpr int PER = (FW * N + LDPC_THREADS - 1) / LDPC_THREADS;
        constexpr int CH = PER < 16 ? PER : 16;
        for (int j0 = 0; j0 < PER; j0 += CH) {
            TIn x[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int k = (j0 + j) * LDPC_THREADS + tid;
                x[j] = llr[f0 * N + (k < nval ? k : 0)];
            }
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int k = (j0 + j) * LDPC_THREADS + tid;
                if (k < nval) {
                    const int slot = k / N, n = k - slot * N;
#if LDPC_PATH == 0
                    const float v = x[j] + 0.0f;
#else
                    const float v = (float)x[j];
#endif
                    Ls[PAD + n * FWP + slot] = v;
                    Ls[ZOFF + PAD + n * FWP + slot] = v;
                }
            }
        }
    }
    if (tid < FW)
        unsat[tid] = 0;
#if LDPC_PATH == 1
    const float off = (float)offset;
    const float wqf = (float)wq;
#endif
    float R[KF][ED];
    bool act[KF];
    int itk[KF], okk[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) {
#pragma unroll
        for (int e = 0; e < ED; ++e)
            R[k][e] = 0.0f;
        act[k] = lane_on && (f0 + slot0 + k < F);
        itk[k] = max_iter;
        okk[k] = 0;
    }
    __syncthreads();

    for (int t = 0; t < max_iter; ++t) {
        const bool check = et || (t == max_iter - 1);
        // ---- check phase: all block rows from the posteriors of iteration t-1
        static_for<0, MB>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int d = kDeg[i];
            constexpr int eo = edge_off(i);
            int rr = r;
            if constexpr (i >= LDPC_HOIST)
                asm volatile("" : "+v"(rr));
            const int rbw = (rr * FWP + slot0) * 4, rbn = rbw + PAD * 4;
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                if (!act[k])
                    continue;
                float Q[MAXD];
#pragma unroll
                for (int e = 0; e < d; ++e)
                    Q[e] = ldb(Ls, gather_b(i, e, rr, rbn, rbw) + k * 4) - R[k][eo + e];
                float m1 = __builtin_inff(), m2 = __builtin_inff();
#pragma unroll
                for (int e = 0; e < d; ++e) {
                    const float a = __builtin_fabsf(Q[e]);
                    m2 = __builtin_amdgcn_fmed3f(a, m1, m2);
                    m1 = __builtin_amdgcn_fmed3f(a, m1, -3.402823466e38f);
                }
                const u32 par = xor_bits<d>(Q) & 0x80000000u;
#if LDPC_PATH == 0
                const float n1 = alpha * m1, n2 = alpha * m2;
#else
                const float c1 = __builtin_fminf(m1, 127.0f), c2 = __builtin_fminf(m2, 127.0f);
#if LDPC_MODE == 0
                const float n1 = __builtin_fmaxf(c1 - off, 0.0f), n2 = __builtin_fmaxf(c2 - off, 0.0f);
#else
                const float n1 = norm_mag(wqf, c1), n2 = norm_mag(wqf, c2);
#endif
#endif
                u32 n1p = __float_as_uint(n1) | par, n2p = __float_as_uint(n2) | par;
                asm volatile("" : "+v"(n1p), "+v"(n2p));
#pragma unroll
                for (int e = 0; e < d; ++e) {
                    const u32 mp = (__builtin_fabsf(Q[e]) == m1) ? n2p : n1p;
                    R[k][eo + e] = __uint_as_float((__float_as_uint(Q[e]) & 0x80000000u) ^ mp);
                }
            }
        });
        __syncthreads();
        // ---- variable phase: Z = Z0 + new messages, block row by block row
        int lastbad[KF];
#pragma unroll
        for (int k = 0; k < KF; ++k)
            lastbad[k] = 0;
        static_for<0, MB>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int d = kDeg[i];
            constexpr int eo = edge_off(i);
            int rr = r;
            if constexpr (i >= LDPC_HOIST)
                asm volatile("" : "+v"(rr));
            const int rbw = (rr * FWP + slot0) * 4, rbn = rbw + PAD * 4;
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                if (!act[k])
                    continue;
                u32 bad = 0, hw = 0;
#pragma unroll
                for (int e = 0; e < d; ++e) {
                    const int a = gather_b(i, e, rr, rbn, rbw) + k * 4;
                    const float base = first_in_column(i, kCol[i][e]) ? ldb(Ls, a + ZOFF * 4) : ldb(Ls, a);
                    const float v = base + R[k][eo + e];
                    stb(Ls, a, v);
                    if (i == MB - 1) {   // row parity of the hard decisions, two edges at a time
                        if (e & 1)
                            bad = __builtin_amdgcn_bitop3_b32(bad, hw, hb_word(v), 0x96);
                        else
                            hw = hb_word(v);
                    }
                }
                if (i == MB - 1)
                    lastbad[k] = (int)((d & 1 ? bad ^ hw : bad) >> 31);
            }
            __syncthreads();
        });
        if (check) {
            // a failing row of the last block row decides a frame at once;
            // the check pass runs for the frames whose last block row is
            // satisfied (marking a frame while another thread still reads
            // its mark is harmless: it is unsatisfied either way)
#pragma unroll
            for (int k = 0; k < KF; ++k)
                if (act[k] && lastbad[k])
                    unsat[slot0 + k] = 1;
            __syncthreads();
            bool need[KF];
            int bad[KF];
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                need[k] = act[k] && unsat[slot0 + k] == 0;
                bad[k] = 0;
            }
            static_for<0, MB - 1>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                int rr = r;
                if constexpr (i >= LDPC_HOIST)
                    asm volatile("" : "+v"(rr));
                const int rbw = (rr * FWP + slot0) * 4, rbn = rbw + PAD * 4;
#pragma unroll
                for (int k = 0; k < KF; ++k) {
                    if (!need[k])
                        continue;
                    u32 w[kDeg[i]];
#pragma unroll
                    for (int e = 0; e < kDeg[i]; ++e)
                        w[e] = hb_word(ldb(Ls, gather_b(i, e, rr, rbn, rbw) + k * 4));
                    bad[k] |= (int)(xor_bits<kDeg[i]>(w) >> 31);
                }
            });
#pragma unroll
            for (int k = 0; k < KF; ++k)
                if (need[k] && bad[k])
                    unsat[slot0 + k] = 1;
            __syncthreads();
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
            const i64 fg = f0 + slot0 + k;
            if (fg < F) {
                iters[fg] = itk[k];
                if (okv)
                    okv[fg] = (u8)okk[k];
            }
        }
    }
    for (int slot = 0; slot < FW; ++slot) {
        const i64 fg = f0 + slot;
        if (fg >= F)
            break;
        for (int n = tid; n < N; n += LDPC_THREADS) {
            const float v = Ls[PAD + n * FWP + slot];
            bits[fg * N + n] = (u8)hard_bit(v);
            if (post)
                post[fg * N + n] = (TP)v;
        }
    }
}
