// The paper's own fixed point (Sec. 5): layered single-scan min-sum on
// int16 values (Q_B-bit LLRs with headroom), specialised for one code at
// run time with the prelude of jit_decode.hip. LDPC_WRAP 1: every 16-bit
// result wraps around as storing into int16_t does; 0: symmetric saturation
// at +-32767. Per check row (eqs. 18, 20, 22, 23), with fix() the wrap or
// the saturation:
//   Q_e = fix(L[n_e] - R_e);  min1, min2 of |Q| and the sign parity in one
//   scan;  R_e = fix(sgn_e * ((wq * m_e + 8) >> 4)), m_e = min2 where
//   |Q_e| == min1 else min1;  L[n_e] = fix(Q_e + R_e).
// Work mapping, message registers and addressing as in jit_decode.hip, on
// int32 VALU arithmetic (posteriors in LDS as int32 holding 16-bit values).

typedef unsigned char u8;
typedef unsigned int u32;
typedef long long i64;

constexpr int Z = LDPC_Z, MB = LDPC_MB, NB = LDPC_NB, N = LDPC_N, MAXD = LDPC_MAXD;
constexpr int G = LDPC_G, KF = LDPC_KF, FWP = LDPC_FWP;
constexpr int FW = G * KF;
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

__device__ __forceinline__ int ldb(const int *Ls, int b) { return *(const int *)((const char *)Ls + b); }

__device__ __forceinline__ void stb(int *Ls, int b, int v) { *(int *)((char *)Ls + b) = v; }

__device__ __forceinline__ int fix16(int x)
{
#if LDPC_WRAP
    return __builtin_amdgcn_sbfe(x, 0, 16);   // sign-extend the low 16 bits
#else
    return x < -32767 ? -32767 : (x > 32767 ? 32767 : x);
#endif
}

__device__ __forceinline__ int hard_bit(int v) { return v > 0 ? 0 : 1; }

extern "C" __global__ __launch_bounds__(LDPC_THREADS) void LDPC_KERNEL(
    const short *__restrict__ llr, const i64 Fmax, const int max_iter, const int wq, const int et,
    u8 *__restrict__ bits, short *__restrict__ post, int *__restrict__ iters, u8 *__restrict__ okv)
{
    const i64 F = Fmax;
    if ((i64)blockIdx.x * FW >= F)
        return;
    __shared__ int Ls[PAD + N * FWP];
    __shared__ int unsat[FW];
    const int tid = threadIdx.x;
    const int g = tid / Z;
    const int r = tid - g * Z;
    const bool lane_on = g < G;
    const int slot0 = g * KF;
    const int rb = r * FWP + slot0;
    const i64 f0 = (i64)blockIdx.x * FW;
    // channel values: the workgroup's frames are one flat range, up to 16
    // loads per thread in flight before the first is waited for (a value
    // past F is read from the workgroup's first frame, which exists, and
    // dropped)
    {
        const i64 nval = (F - f0 < FW ? F - f0 : (i64)FW) * (i64)N;
        constexpr int PER = (FW * N + LDPC_THREADS - 1) / LDPC_THREADS;
        constexpr int CH = PER < 16 ? PER : 16;
        for (int j0 = 0; j0 < PER; j0 += CH) {
            short x[CH];
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
                    Ls[PAD + n * FWP + slot] = (int)x[j];
                }
            }
        }
    }
    if (tid < FW)
        unsat[tid] = 0;
    int R[KF][ED];
    bool act[KF];
    int itk[KF], okk[KF];
#pragma unroll
    for (int k = 0; k < KF; ++k) {
#pragma unroll
        for (int e = 0; e < ED; ++e)
            R[k][e] = 0;
        act[k] = lane_on && (f0 + slot0 + k < F);
        itk[k] = max_iter;
        okk[k] = 0;
    }
    __syncthreads();

    for (int t = 0; t < max_iter; ++t) {
        const bool check = et || (t == max_iter - 1);
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
            int ix[MAXD];
#pragma unroll
            for (int e = 0; e < d; ++e)
                ix[e] = gather_b(i, e, rr, rbn, rbw);
#pragma unroll
            for (int k = 0; k < KF; ++k) {
                if (!act[k])
                    continue;
                int Q[MAXD];
#pragma unroll
                for (int e = 0; e < d; ++e)
                    Q[e] = fix16(ldb(Ls, ix[e] + k * 4) - R[k][eo + e]);
                int m1 = 0x7fffffff, m2 = 0x7fffffff;
                u32 px = 0;
#pragma unroll
                for (int e = 0; e < d; ++e) {
                    const int a = Q[e] < 0 ? -Q[e] : Q[e];
                    m2 = a > m1 ? (a < m2 ? a : m2) : m1;   // second smallest (a v_med3_i32)
                    m1 = a < m1 ? a : m1;
                    px ^= (u32)Q[e];
                }
                const int n1 = (wq * m1 + 8) >> 4, n2 = (wq * m2 + 8) >> 4;
                int bad = 0;
#pragma unroll
                for (int e = 0; e < d; ++e) {
                    const int a = Q[e] < 0 ? -Q[e] : Q[e];
                    const int mag = a == m1 ? n2 : n1;
                    const int s = (int)(((u32)Q[e] ^ px) & 0x80000000u) >> 31;   // -1: message negative
                    const int rv = fix16((mag ^ s) - s);
                    R[k][eo + e] = rv;
                    const int lv = fix16(Q[e] + rv);
                    stb(Ls, ix[e] + k * 4, lv);
                    if (i == MB - 1)
                        bad ^= hard_bit(lv);
                }
                if (i == MB - 1)
                    lastbad[k] = bad;
            }
            __syncthreads();
        });
        if (check) {
            int bad[KF];
#pragma unroll
            for (int k = 0; k < KF; ++k)
                bad[k] = lastbad[k];
            static_for<0, MB - 1>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                int rr = r;
                if constexpr (i >= LDPC_HOIST)
                    asm volatile("" : "+v"(rr));
                const int rbw = (rr * FWP + slot0) * 4, rbn = rbw + PAD * 4;
#pragma unroll
                for (int k = 0; k < KF; ++k) {
                    if (!act[k])
                        continue;
                    int p = 0;
#pragma unroll
                    for (int e = 0; e < kDeg[i]; ++e)
                        p ^= hard_bit(ldb(Ls, gather_b(i, e, rr, rbn, rbw) + k * 4));
                    bad[k] |= p;
                }
            });
#pragma unroll
            for (int k = 0; k < KF; ++k)
                if (act[k] && bad[k])
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
            const int v = Ls[PAD + n * FWP + slot];
            bits[fg * N + n] = (u8)hard_bit(v);
            if (post)
                post[fg * N + n] = (short)v;
        }
    }
}
