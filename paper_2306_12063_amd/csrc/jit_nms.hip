// Learned normalised min-sum: training forward with per-iteration
// checkpoints and loss, and its hand-written adjoint, specialised for one
// code at run time (hipRTC, same prelude as jit_decode.hip; LDPC_KF is 1).
//
// Model. Weights w[T][MB][NB] scale the messages: in iteration t (0-based)
// the message leaving edge e of a check row of block row i is
//   R_e = sgn_e * fl(w[t][i][col_e] * m_e),
// m_e = min over the other edges of |Q|, sgn_e = product of their signs,
// Q_e = L[n_e] - R_old_e (eq. 22) with R_old_e the message of iteration t-1,
// and L[n_e] = Q_e + R_e (eq. 20), in the layered order of Sec. 4. The loss
// is l = 1/(T F N) sum_t sum_f sum_n softplus(-(1 - 2 c_fn) L_fn^(t)), the
// binary cross-entropy of sigmoid(L) (the probability of bit 0, eq. 17)
// after every iteration. Early termination is off.
//
// Weight gradients: each lane holds one term per weight and iteration; the
// terms are summed within each 16-lane row of the wave (DPP row shifts),
// each row stores its sum in its own LDS slot, the workgroup adds the slots
// in a fixed order and stores the sums, and a reduction kernel adds the
// workgroups' sums in a fixed order: the gradient is the same on every run.
//
// Checkpoint of iteration t (taken when it starts), per frame: L (N FP32)
// and the compressed row state (raw minima m1, m2 and sign/argmin word,
// one triple per check row). The adjoint restores it and recomputes the
// iteration; each row's state after its update, plus the index of the
// second smallest |Q| and the parity of the Q signs, is all the backward
// needs of Q (|Q| enters only through the two minima, Q's sign is the
// message's sign times the parity). Then it runs the layers in reverse:
//   G_e = gL[n_e] + gR_e                      (R_e feeds L and the next Q)
//   gw[t][i][col_e] += G_e * sgn_e * m_e
//   gm_e = G_e * sgn_e * w[t][i][col_e]
//   g|Q|_a1 += sum_{e != a1} gm_e,  g|Q|_a2 += gm_a1   (a1, a2: first and second
//                                                       smallest |Q|, lowest index first)
//   gQ_e = gL[n_e] + g|Q|_e * sgn(Q_e);  gL[n_e] = gQ_e;  gR_e = -gQ_e
// and before the layers of iteration t adds d l / d L^(t+1) to gL.

typedef unsigned char u8;
typedef unsigned int u32;
typedef long long i64;

constexpr int Z = LDPC_Z, MB = LDPC_MB, NB = LDPC_NB, N = LDPC_N, MAXD = LDPC_MAXD;
constexpr int G = LDPC_G, FWP = LDPC_FWP;
constexpr int M = MB * Z;
constexpr int ZFW = Z * FWP;

// edges of a check row over all block rows, and the offset of block row i
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

__device__ __forceinline__ int gather(int i, int e, int r, int rb)
{
    const int base = (kCol[i][e] * Z + kShift[i][e]) * FWP;
    return rb + base - ((r >= Z - kShift[i][e]) ? ZFW : 0);
}

// Sum of v over each row of 16 lanes, in lane 15 of the row: inclusive sums
// by DPP row shifts (lanes a shift does not reach add 0). Stopping at the
// rows saves the cross-row broadcast steps, whose masked form costs three
// instructions each: the rows' sums go to LDS instead.
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf,
                                                                     false));
}
__device__ __forceinline__ float row_sum(float v)
{
    v = dpp_add<0x111>(v);   // row_shr:1
    v = dpp_add<0x112>(v);   // row_shr:2
    v = dpp_add<0x114>(v);   // row_shr:4
    return dpp_add<0x118>(v);   // row_shr:8
}

// Softplus and sigmoid on the transcendental unit: v_exp_f32 and v_log_f32
// (base 2) and v_rcp_f32 are accurate to about one ulp, and the loss and its
// gradient are means over every bit of every frame, where these errors stay
// orders of magnitude below the loss and gradient tolerances. (The library
// expf and log1pf cost several times the decoder's own arithmetic per bit.)
__device__ __forceinline__ float exp_neg_abs(float z)   // e^-|z| in (0, 1]
{
    return __builtin_amdgcn_exp2f(-__builtin_fabsf(z) * 1.44269504088896341f);
}
__device__ __forceinline__ float softplus(float z)
{
    return __builtin_fmaxf(z, 0.0f) + __builtin_amdgcn_logf(1.0f + exp_neg_abs(z)) * 0.693147180559945309f;
}
__device__ __forceinline__ float sigmoid(float z)
{
    const float e = exp_neg_abs(z);
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    return z >= 0.0f ? r : e * r;
}

// Checkpoint layout for iteration t and frame f (all FP32 words):
//   L      at ((t*F + f) * CK)             N values
//   m1, m2 at ((t*F + f) * CK) + N, + N + M  M values each (row i*Z + r)
//   sg     at ((t*F + f) * CK) + N + 2M    M words
constexpr int CK = N + 3 * M;

// The backward keeps, per check row, the index a2 of the second smallest |Q|
// and the parity of Q's signs. With at most 21 edges per row they fit in the
// unused bits 21..26 of the sign/argmin word (a2 at 21, parity at 26), else in
// a word of their own.
constexpr bool PACK = MAXD <= 21;
constexpr int NWAVE = (LDPC_THREADS + 63) / 64;
constexpr int NSLOT = 4 * NWAVE;   // 16-lane rows of the workgroup

// One layer of the forward for the thread's check row. Writes new L values
// to LDS and the new compressed state; with KEEP (backward recompute) also
// a2, the index of the second smallest |Q| (lowest index first among equal
// values, as for the smallest), and the parity of Q's signs: packed into sgs
// (PACK) or as aux = a2 | parity << 5.
template <bool KEEP>
__device__ __forceinline__ void fwd_layer(int i, int t, int r, int rb, float *Ls, const float *__restrict__ w,
                                          float &m1s, float &m2s, u32 &sgs, u32 &aux)
{
    const int d = kDeg[i];
    int ix[MAXD];
    float Q[MAXD];
    // opaque: the addresses are recomputed per layer instead of all being
    // kept live across iterations (that would cost a register per edge)
    asm volatile("" : "+v"(r), "+v"(rb));
#pragma unroll
    for (int e = 0; e < MAXD; ++e)
        if (e < d)
            ix[e] = gather(i, e, r, rb);
    const u32 oidx = sgs >> 27;
#pragma unroll
    for (int e = 0; e < MAXD; ++e) {
        if (e >= d)
            continue;
        // old message: raw minimum times the weight of the iteration that made it
        const float m = (oidx == (u32)e) ? m2s : m1s;
        const float mag = t > 0 ? w[((t - 1) * MB + i) * NB + kCol[i][e]] * m : 0.0f;
        const u32 ro = __float_as_uint(mag) | ((sgs << (32 - d + e)) & 0x80000000u);
        Q[e] = Ls[ix[e]] - __uint_as_float(ro);
    }
    u32 idx = 0, idx2 = 0, neg = 0;
    float m1 = __builtin_inff(), m2 = __builtin_inff();
#pragma unroll
    for (int e = 0; e < MAXD; ++e) {
        if (e >= d)
            continue;
        const float a = __builtin_fabsf(Q[e]);
        if (KEEP)
            idx2 = (a < m1) ? idx : ((a < m2) ? (u32)e : idx2);
        idx = (a < m1) ? (u32)e : idx;
        m2 = __builtin_amdgcn_fmed3f(a, m1, m2);
        m1 = __builtin_fminf(m1, a);
        neg = __builtin_amdgcn_alignbit(neg, __float_as_uint(Q[e]), 31);
    }
    const u32 par = (u32)__popc(neg) & 1u;
    const u32 parbit = par << 31;
#pragma unroll
    for (int e = 0; e < MAXD; ++e) {
        if (e >= d)
            continue;
        const float mag = w[(t * MB + i) * NB + kCol[i][e]] * ((idx == (u32)e) ? m2 : m1);
        const u32 rn = __float_as_uint(mag) | ((__float_as_uint(Q[e]) ^ parbit) & 0x80000000u);
        Ls[ix[e]] = Q[e] + __uint_as_float(rn);
    }
    m1s = m1;
    m2s = m2;
    sgs = (neg ^ ((0u - par) & ((1u << d) - 1u))) | (idx << 27);
    if (KEEP && PACK)
        sgs |= (idx2 << 21) | (par << 26);
    if (KEEP && !PACK)
        aux = idx2 | (par << 5);
}

// The transmitted codeword's bits at variables j*Z + r (j < NB) of frame f,
// bit j of the result, read once per kernel instead of once per iteration
// (codes of up to 32 block columns; wider codes read them when used).
__device__ __forceinline__ u32 target_bits(const u8 *__restrict__ cw, i64 f, int r, bool on)
{
    u32 b = 0;
    if constexpr (NB <= 32) {
        if (on) {
            u8 c[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j)
                c[j] = cw[f * N + j * Z + r];
#pragma unroll
            for (int j = 0; j < NB; ++j)
                b |= (c[j] ? 1u : 0u) << j;
        }
    }
    return b;
}

// BPSK symbol of the transmitted bit at variable j*Z + r of frame f: -1 for
// bit 1, +1 for bit 0.
__device__ __forceinline__ float target_sign(const u8 *__restrict__ cw, u32 bits, i64 f, int j, int r)
{
    if constexpr (NB <= 32)
        return (bits >> j) & 1u ? -1.0f : 1.0f;
    else
        return cw[f * N + j * Z + r] ? -1.0f : 1.0f;
}

extern "C" __global__ __launch_bounds__(LDPC_THREADS) void ldpc_nms_fwd(
    const float *__restrict__ llr, const u8 *__restrict__ cw, const i64 F, const int T, const float *__restrict__ w,
    float *__restrict__ ckpt, float *__restrict__ loss_tf, float *__restrict__ post)
{
    __shared__ float Ls[N * FWP];
    __shared__ float part[G * Z];
    const int tid = threadIdx.x;
    const int g = tid / Z;
    const int r = tid - g * Z;
    const i64 f = (i64)blockIdx.x * G + g;
    const bool on = g < G && f < F;
    const int rb = r * FWP + g;
    // channel values: the workgroup's frames are one flat range of G*N
    // values, all of a thread's loads in flight before the first is waited
    // for (a value past F is read from frame 0 of the workgroup, which
    // exists, and dropped)
    {
        const i64 fb = (i64)blockIdx.x * G;
        const i64 nval = (F - fb < G ? F - fb : G) * (i64)N;
        constexpr int PER = (G * N + LDPC_THREADS - 1) / LDPC_THREADS;
        float v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = j * LDPC_THREADS + tid;
            v[j] = llr[fb * N + (k < nval ? k : 0)];
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = j * LDPC_THREADS + tid;
            if (k < nval) {
                const int s = k / N, n = k - s * N;
                Ls[n * FWP + s] = v[j] + 0.0f;
            }
        }
    }
    const u32 xbits = target_bits(cw, f, r, on);
    float sm1[MB], sm2[MB];
    u32 ssg[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        sm1[i] = 0.0f;
        sm2[i] = 0.0f;
        ssg[i] = 0u;
    }
    __syncthreads();
    for (int t = 0; t < T; ++t) {
        if (on) {
            float *ck = ckpt + ((i64)t * F + f) * CK;
#pragma unroll
            for (int j = 0; j < NB; ++j)
                ck[j * Z + r] = Ls[(j * Z + r) * FWP + g];
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                ck[N + i * Z + r] = sm1[i];
                ck[N + M + i * Z + r] = sm2[i];
                ck[N + 2 * M + i * Z + r] = __uint_as_float(ssg[i]);
            }
        }
        // layer 0 rewrites L values other threads are copying out above
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            u32 unused;
            if (on)
                fwd_layer<false>(i, t, r, rb, Ls, w, sm1[i], sm2[i], ssg[i], unused);
            __syncthreads();
        }
        // per-frame loss of this iteration: thread r sums variables j*Z + r
        float acc = 0.0f;
        if (on) {
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int n = j * Z + r;
                const float x = target_sign(cw, xbits, f, j, r);
                acc += softplus(-x * Ls[n * FWP + g]);
            }
        }
        if (g < G)
            part[g * Z + r] = acc;
        __syncthreads();
        if (on && r == 0) {
            float s = 0.0f;
            for (int k = 0; k < Z; ++k)
                s += part[g * Z + k];
            loss_tf[(i64)t * F + f] = s;
        }
        __syncthreads();
    }
    if (post && on) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
            post[f * N + j * Z + r] = Ls[(j * Z + r) * FWP + g];
    }
}

// loss[t] = (1 / (T F N)) sum_f loss_tf[t][f], one workgroup per iteration,
// summed in a fixed order.
extern "C" __global__ __launch_bounds__(256) void ldpc_nms_loss_reduce(const float *__restrict__ loss_tf, const i64 F,
                                                                      const int T, float *__restrict__ loss)
{
    __shared__ double red[256];
    const int t = blockIdx.x;
    double s = 0.0;
    for (i64 f = threadIdx.x; f < F; f += 256)
        s += (double)loss_tf[(i64)t * F + f];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k)
            red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss[t] = (float)(red[0] / ((double)T * (double)F * (double)N));
}

// Two waves per SIMD: the per-edge message gradients and the row state of
// one iteration exceed 256 registers by a few dozen for the larger codes;
// spilling those costs less than running one wave per SIMD.
extern "C" __global__ __launch_bounds__(LDPC_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void ldpc_nms_bwd(
    const u8 *__restrict__ cw, const i64 F, const int T, const float *__restrict__ w,
    const float *__restrict__ ckpt, const float *__restrict__ dloss, float *__restrict__ partial)
{
    __shared__ float Ls[N * FWP];
    __shared__ float gL[N * FWP];
    __shared__ float gw[NSLOT][MB * NB];   // per 16-lane row: its sums of the iteration's weight terms
    const int tid = threadIdx.x;
    const int slot = tid >> 4;
    const int g = tid / Z;
    const int r = tid - g * Z;
    const i64 f = (i64)blockIdx.x * G + g;
    const bool on = g < G && f < F;
    const int rb = r * FWP + g;
    const double inv = 1.0 / ((double)T * (double)F * (double)N);
    const u32 xbits = target_bits(cw, f, r, on);
    float gR[ED];   // d loss / d R_e of the iteration being reversed
#pragma unroll
    for (int k = 0; k < ED; ++k)
        gR[k] = 0.0f;
    for (int n = tid; n < N * FWP; n += LDPC_THREADS)
        gL[n] = 0.0f;
    for (int k = tid; k < NSLOT * MB * NB; k += LDPC_THREADS)
        gw[k / (MB * NB)][k % (MB * NB)] = 0.0f;   // weights without an edge stay 0
    __syncthreads();
    for (int t = T - 1; t >= 0; --t) {
        // restore the start of iteration t and recompute it; afterwards the
        // row state is iteration t's own
        float sm1[MB], sm2[MB];
        u32 ssg[MB], aux[PACK ? 1 : MB];
        if (on) {
            const float *ck = ckpt + ((i64)t * F + f) * CK;
#pragma unroll
            for (int j = 0; j < NB; ++j)
                Ls[(j * Z + r) * FWP + g] = ck[j * Z + r];
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                sm1[i] = ck[N + i * Z + r];
                sm2[i] = ck[N + M + i * Z + r];
                ssg[i] = __float_as_uint(ck[N + 2 * M + i * Z + r]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            if (on)
                fwd_layer<true>(i, t, r, rb, Ls, w, sm1[i], sm2[i], ssg[i], aux[PACK ? 0 : i]);
            __syncthreads();
        }
        // the loss reads L after iteration t directly
        const float sc = (float)((double)dloss[t] * inv);
        if (on) {
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int n = j * Z + r;
                const float x = target_sign(cw, xbits, f, j, r);
                gL[n * FWP + g] += -x * sigmoid(-x * Ls[n * FWP + g]) * sc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ii = 0; ii < MB; ++ii) {
            const int i = MB - 1 - ii;
            const int d = kDeg[i];
            float gwc[MAXD];   // this lane's terms of the row's weight gradients
#pragma unroll
            for (int e = 0; e < MAXD; ++e)
                gwc[e] = 0.0f;
            if (on) {
                float *gr = gR + edge_off(i);
                int ix[MAXD], rr = r, rbb = rb;
                asm volatile("" : "+v"(rr), "+v"(rbb));
#pragma unroll
                for (int e = 0; e < MAXD; ++e)
                    if (e < d)
                        ix[e] = gather(i, e, rr, rbb);
                // smallest and second smallest |Q| (v1 at a1, v2 at a2), the
                // message signs (bit d-1-e of sw) and the parity of Q's signs
                const float v1 = sm1[i], v2 = sm2[i];
                const u32 sw = ssg[i];
                const u32 ax = PACK ? sw >> 21 : aux[PACK ? 0 : i];
                const u32 a1 = sw >> 27, a2 = ax & 31u, par = (ax >> 5) & 1u;
                float gQ1 = 0.0f, gQ2 = 0.0f, gl[MAXD];
#pragma unroll
                for (int e = 0; e < MAXD; ++e) {
                    if (e >= d)
                        continue;
                    gl[e] = gL[ix[e]];
                    const float sg = ((sw >> (d - 1 - e)) & 1u) ? -1.0f : 1.0f;
                    const float m = ((u32)e == a1) ? v2 : v1;
                    const float Ge = gl[e] + gr[e];
                    const float wv = w[(t * MB + i) * NB + kCol[i][e]];
                    gwc[e] = Ge * sg * m;
                    const float gm = Ge * sg * wv;
                    if ((u32)e == a1)
                        gQ2 += gm;
                    else
                        gQ1 += gm;
                }
#pragma unroll
                for (int e = 0; e < MAXD; ++e) {
                    if (e >= d)
                        continue;
                    const float ga = ((u32)e == a1) ? gQ1 : (((u32)e == a2) ? gQ2 : 0.0f);
                    const float sq = (((sw >> (d - 1 - e)) ^ par) & 1u) ? -1.0f : 1.0f;
                    const float gq = gl[e] + ga * sq;
                    gL[ix[e]] = gq;
                    gr[e] = -gq;
                }
            }
            // every lane of the workgroup has a term for the same weights:
            // each 16-lane row sums them (DPP) and stores the sum in its own
            // slot, which nothing else writes (no atomics, a fixed order)
#pragma unroll
            for (int e = 0; e < MAXD; ++e) {
                if (e >= d)
                    continue;
                const float s = row_sum(gwc[e]);
                if ((tid & 15) == 15)
                    gw[slot][i * NB + kCol[i][e]] = s;
            }
            __syncthreads();
        }
        // this iteration's weight gradient of the workgroup's frames (its
        // rows' sums in row order), summed over workgroups by
        // ldpc_nms_grad_reduce
        for (int k = tid; k < MB * NB; k += LDPC_THREADS) {
            float s = gw[0][k];
#pragma unroll
            for (int v = 1; v < NSLOT; ++v)
                s += gw[v][k];
            partial[((i64)blockIdx.x * T + t) * (MB * NB) + k] = s;
        }
        __syncthreads();
    }
}

// grad_w[k] = sum over the adjoint's workgroups b of partial[b][k], k over
// the T*MB*NB weights. A workgroup of 1024 threads takes 64 consecutive
// weights (one per lane, coalesced); wave v adds the workgroups b = v,
// v + 16, ... in order, then the 16 wave sums are added in wave order: the
// same sum on every run.
extern "C" __global__ __launch_bounds__(1024) void ldpc_nms_grad_reduce(const float *__restrict__ partial,
                                                                       const i64 nwg, const int nw,
                                                                       float *__restrict__ grad_w)
{
    __shared__ double red[16][64];
    const int lane = threadIdx.x & 63, v = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (k < nw) {
        i64 b = v;
        for (; b + 48 < nwg; b += 64) {   // four loads in flight
            const float x0 = partial[b * nw + k], x1 = partial[(b + 16) * nw + k];
            const float x2 = partial[(b + 32) * nw + k], x3 = partial[(b + 48) * nw + k];
            s += (double)x0;
            s += (double)x1;
            s += (double)x2;
            s += (double)x3;
        }
        for (; b < nwg; b += 16)
            s += (double)partial[b * nw + k];
    }
    red[v][lane] = s;
    __syncthreads();
    if (v == 0 && k < nw) {
        double t = red[0][lane];
        for (int u = 1; u < 16; ++u)
            t += red[u][lane];
        grad_w[k] = (float)t;
    }
}
