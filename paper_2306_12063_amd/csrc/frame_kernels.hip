// Frame generation kernels for gfx950: seeded information bits, the direct
// QC encoder (Sec. 2, eqs. 12-15), BPSK over AWGN with the channel LLR
// (eqs. 16-17) and the int8 LLR quantiser.
#include <math.h>

#include "ldpc_internal.h"

namespace ldpc {
namespace {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplies, a swap and a key xor; the key advances by the Weyl constants.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

// Bit k of frame f = bit (k % 32) of word (k / 32 % 4) of
// Philox({k / 128, f, 0, 0}, seed). One thread per 128-bit block.
__global__ void k_random_bits(uint64_t seed, const uint64_t *__restrict__ seed_dev, int64_t F, int64_t K,
                              uint8_t *__restrict__ out)
{
    if (seed_dev)
        seed = *seed_dev;
    const int64_t blocks_per_frame = (K + 127) / 128;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= F * blocks_per_frame)
        return;
    const int64_t f = gid / blocks_per_frame, b = gid - f * blocks_per_frame;
    const uint4 o = philox4x32_10(make_uint4((uint32_t)b, (uint32_t)f, 0u, 0u),
                                  make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    const uint32_t w[4] = {o.x, o.y, o.z, o.w};
    uint8_t *dst = out + f * K;
    const int64_t k0 = b * 128;
    for (int j = 0; j < 128 && k0 + j < K; ++j)
        dst[k0 + j] = (uint8_t)((w[j >> 5] >> (j & 31)) & 1u);
}

// Noise sample n of frame f: Box-Muller on words (2p, 2p+1), p = (n%4)/2, of
// Philox({n / 4, f, 1, 0}, seed), with u = ((word >> 8) + 1/2) 2^-24;
// cos for even n, sin for odd n. LLR = ((1 - 2x) + sigma z) * scale, in FP32
// without fused multiply-add. One thread per 4 consecutive positions.
__global__ void k_awgn_llr(uint64_t seed, const uint64_t *__restrict__ seed_dev, int64_t F, int64_t N,
                           const uint8_t *__restrict__ cw, float sigma, float scale,
                           const float *__restrict__ sigma_f, const float *__restrict__ scale_f,
                           float *__restrict__ llr)
{
    if (seed_dev)
        seed = *seed_dev;
    const int64_t quads = (N + 3) / 4;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= F * quads)
        return;
    const int64_t f = gid / quads, q = gid - f * quads;
    const uint4 o = philox4x32_10(make_uint4((uint32_t)q, (uint32_t)f, 1u, 0u),
                                  make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    const float two_pi = 6.28318530717958647692f;
    const float inv24 = 1.0f / 16777216.0f;
    const float ua0 = ((float)(o.x >> 8) + 0.5f) * inv24, ub0 = ((float)(o.y >> 8) + 0.5f) * inv24;
    const float ua1 = ((float)(o.z >> 8) + 0.5f) * inv24, ub1 = ((float)(o.w >> 8) + 0.5f) * inv24;
    const float r0 = sqrtf(-2.0f * logf(ua0)), r1 = sqrtf(-2.0f * logf(ua1));
    const float z[4] = {r0 * cosf(two_pi * ub0), r0 * sinf(two_pi * ub0), r1 * cosf(two_pi * ub1),
                        r1 * sinf(two_pi * ub1)};
    const int64_t base = f * N + q * 4;
    if (sigma_f) {
        sigma = sigma_f[f];
        scale = scale_f[f];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (q * 4 + j < N) {
            const float x = (cw[base + j] & 1u) ? -1.0f : 1.0f;
            const float y = x + sigma * z[j];
            llr[base + j] = y * scale;
        }
    }
}

__global__ void k_quantize_i8(const float *__restrict__ in, int8_t *__restrict__ out, int64_t n, float scale)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    float v = rintf(scale * in[i]);
    v = fminf(fmaxf(v, -127.0f), 127.0f);
    out[i] = (int8_t)v;
}

// Learned weights in 1/16 steps for the fixed-point decoder:
// wq = clamp(rint(16 w), 0, 31), half to even (16 w is exact). v_max_f32
// returns the other operand for a NaN, so a NaN weight becomes 0.
__global__ void k_quantize_weights(const float *__restrict__ in, uint8_t *__restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    float v = rintf(16.0f * in[i]);
    v = fminf(fmaxf(v, 0.0f), 31.0f);
    out[i] = (uint8_t)v;
}

// Q_B-bit quantiser of the paper's fixed point: clamp(rint(scale x), +-qmax).
__global__ void k_quantize_q16(const float *__restrict__ in, int16_t *__restrict__ out, int64_t n, float scale,
                               float qmax)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    float v = rintf(scale * in[i]);
    v = fminf(fmaxf(v, -qmax), qmax);
    out[i] = (int16_t)v;
}

// Direct encoder. A workgroup encodes G frames; thread (g, r) owns row r of
// every Z-bit block of frame g.
//   S_i[r] = xor_j u_j[(r + H(i,j)) mod Z] over the information columns (eq. 15)
//   T = xor_i S_i,  v_0[c] = T[(c - h_b(y)) mod Z]                  (eq. 12)
//   v_1 = P_{h_b(0)} v_0 + S_0                                     (eq. 13)
//   v_{i+1} = v_i + P_{h_b(i)} v_0 + S_i,  i = 1 .. Mb-2          (eq. 14)
// The S_i bits of a thread live in one register; T and v_0 go through LDS
// because v_0 is read at shifted rows.
__global__ __launch_bounds__(kMaxThreads) void k_encode(const Sched sc, const int G, const uint8_t *__restrict__ info,
                                                         uint8_t *__restrict__ cw, int64_t F)
{
    extern __shared__ uint8_t lds[];
    const int Z = sc.Z, K = sc.K, N = sc.N, Mb = sc.Mb, Kb = sc.Nb - sc.Mb;
    uint8_t *ubuf = lds;                        // [G][K]
    uint8_t *tbuf = lds + (size_t)G * K;        // [G][Z]
    uint8_t *v0buf = tbuf + (size_t)G * Z;      // [G][Z]
    const int tid = threadIdx.x;
    const int64_t f0 = (int64_t)blockIdx.x * G;
    for (int g = 0; g < G; ++g) {
        const int64_t f = f0 + g;
        if (f >= F)
            break;
        for (int k = tid; k < K; k += blockDim.x) {
            const uint8_t b = info[f * K + k] & 1u;
            ubuf[g * K + k] = b;
            cw[f * N + k] = b;
        }
    }
    __syncthreads();
    const int g = tid / Z, r = tid - (tid / Z) * Z;
    const bool on = g < G && f0 + g < F;
    uint32_t S = 0;
    if (on) {
        const uint8_t *u = ubuf + g * K;
        for (int i = 0; i < Mb; ++i) {
            uint32_t acc = 0;
            const int d = sc.deg[i];
            for (int e = 0; e < d; ++e) {
                const uint32_t ew = sc.edge[i][e];
                const int col = (int)(ew >> 16);
                if (col >= Kb)
                    break;     // edges are in ascending column: the rest are parity columns
                int x = r + (int)(ew & 0xffffu);
                x = x >= Z ? x - Z : x;
                acc ^= u[col * Z + x];
            }
            S |= acc << i;
        }
        tbuf[g * Z + r] = (uint8_t)(__popc(S) & 1);
    }
    __syncthreads();
    if (on) {
        const int hy = sc.hb[sc.enc_y];
        int c = r - hy;
        c = c < 0 ? c + Z : c;
        v0buf[g * Z + r] = tbuf[g * Z + c];
    }
    __syncthreads();
    if (on) {
        const uint8_t *v0 = v0buf + g * Z;
        uint8_t *p = cw + (f0 + g) * N + K;
        const uint8_t v0r = v0[r];
        p[r] = v0r;
        int h0 = r + sc.hb[0];
        h0 = h0 >= Z ? h0 - Z : h0;
        uint8_t v = v0[h0] ^ (uint8_t)(S & 1u);
        p[Z + r] = v;
        for (int i = 1; i <= Mb - 2; ++i) {
            const int hi = sc.hb[i];
            uint8_t t = v ^ (uint8_t)((S >> i) & 1u);
            if (hi >= 0) {
                int x = r + hi;
                x = x >= Z ? x - Z : x;
                t ^= v0[x];
            }
            v = t;
            p[(i + 1) * Z + r] = v;
        }
    }
}

// Per-frame decoding statistics against the transmitted information bits
// (the first K code bits, eq. 1): counters[0] += information-bit errors,
// [1] += frames with any such error, [2] += iterations, [3] += frames whose
// syndrome check failed. Integer atomics, so the totals do not depend on
// the order of the additions. One workgroup per frame.
__global__ __launch_bounds__(256) void k_frame_stats(const uint8_t *__restrict__ bits, const uint8_t *__restrict__ info,
                                                     const int32_t *__restrict__ iters, const uint8_t *__restrict__ ok,
                                                     int64_t N, int64_t K, unsigned long long *__restrict__ counters)
{
    __shared__ unsigned int red[256];
    const int64_t f = blockIdx.x;
    unsigned int e = 0;
    for (int64_t k = threadIdx.x; k < K; k += 256)
        e += (bits[f * N + k] ^ info[f * K + k]) & 1u;
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&counters[0], (unsigned long long)red[0]);
        atomicAdd(&counters[1], red[0] ? 1ull : 0ull);
        if (iters)
            atomicAdd(&counters[2], (unsigned long long)iters[f]);
        if (ok)
            atomicAdd(&counters[3], ok[f] ? 0ull : 1ull);
    }
}

// Indices of the frames with ok == 0, in frame order: out[0] = count,
// out[1 .. count] = indices. One workgroup; each thread owns a contiguous
// chunk of frames and the chunk offsets come from a scan in LDS, so the
// list is the same on every run.
__global__ __launch_bounds__(1024) void k_compact_failed(const uint8_t *__restrict__ ok, int64_t F,
                                                        int64_t *__restrict__ out)
{
    __shared__ int64_t cnt[1024];
    const int64_t chunk = (F + 1023) / 1024;
    const int64_t lo = (int64_t)threadIdx.x * chunk, hi = lo + chunk < F ? lo + chunk : F;
    int64_t c = 0;
    for (int64_t f = lo; f < hi; ++f)
        c += ok[f] ? 0 : 1;
    cnt[threadIdx.x] = c;
    __syncthreads();
    // inclusive Hillis-Steele scan over the 1024 chunk counts
    for (int s = 1; s < 1024; s <<= 1) {
        const int64_t v = (int)threadIdx.x >= s ? cnt[threadIdx.x - s] : 0;
        __syncthreads();
        cnt[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t pos = cnt[threadIdx.x] - c;
    for (int64_t f = lo; f < hi; ++f)
        if (!ok[f])
            out[1 + pos++] = f;
    if (threadIdx.x == 1023)
        out[0] = cnt[1023];
}

inline int grid_for(int64_t work, int threads) { return (int)((work + threads - 1) / threads); }

}  // namespace

int launch_quantize_i8(const float *llr, int8_t *q, int64_t n, float scale, hipStream_t stream)
{
    hipLaunchKernelGGL(k_quantize_i8, dim3(grid_for(n, 256)), dim3(256), 0, stream, llr, q, n, scale);
    return check_launch(__func__);
}

int launch_quantize_weights(const float *w, uint8_t *wq, int64_t n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_quantize_weights, dim3(grid_for(n, 256)), dim3(256), 0, stream, w, wq, n);
    return check_launch(__func__);
}

int launch_quantize_q16(const float *llr, int16_t *q, int64_t n, float scale, int qmax, hipStream_t stream)
{
    hipLaunchKernelGGL(k_quantize_q16, dim3(grid_for(n, 256)), dim3(256), 0, stream, llr, q, n, scale, (float)qmax);
    return check_launch(__func__);
}

int launch_random_bits(uint64_t seed, const uint64_t *seed_dev, int64_t F, int64_t K, uint8_t *info,
                       hipStream_t stream)
{
    const int64_t work = F * ((K + 127) / 128);
    hipLaunchKernelGGL(k_random_bits, dim3(grid_for(work, 256)), dim3(256), 0, stream, seed, seed_dev, F, K, info);
    return check_launch(__func__);
}

int launch_awgn_llr(uint64_t seed, const uint64_t *seed_dev, int64_t F, int64_t N, const uint8_t *cw, float sigma,
                    float scale, const float *sigma_f, const float *scale_f, float *llr, hipStream_t stream)
{
    const int64_t work = F * ((N + 3) / 4);
    hipLaunchKernelGGL(k_awgn_llr, dim3(grid_for(work, 256)), dim3(256), 0, stream, seed, seed_dev, F, N, cw, sigma,
                       scale, sigma_f, scale_f, llr);
    return check_launch(__func__);
}

int launch_frame_stats(const uint8_t *bits, const uint8_t *info, const int32_t *iters, const uint8_t *ok, int64_t F,
                       int64_t N, int64_t K, int64_t *counters, hipStream_t stream)
{
    hipLaunchKernelGGL(k_frame_stats, dim3((unsigned)F), dim3(256), 0, stream, bits, info, iters, ok, N, K,
                       (unsigned long long *)counters);
    return check_launch(__func__);
}

// LDS read bandwidth probe: each thread of a 256-thread workgroup reads
// 16-byte words of a 64 KB LDS buffer, 8 per round at fixed offsets from a
// base that moves every round (so the loads cannot be hoisted), and folds
// them into a checksum with three-input bit operations (two per read, so
// the ALU stays below the LDS rate). Indices stay below 3840 of 4096.
__global__ __launch_bounds__(256) void k_lds_probe(float *out, int rounds)
{
    __shared__ uint4 buf[4096];
    const int t = threadIdx.x;
    for (int k = t; k < 4096; k += 256)
        buf[k] = make_uint4(k, k * 3u, k * 5u, k * 7u);
    __syncthreads();
    uint32_t a0 = 0, a1 = 0;
    int base = t;
    for (int k = 0; k < rounds; ++k) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint4 v = buf[base + u * 256];
            a0 = __builtin_amdgcn_bitop3_b32(a0, v.x, v.y, 0x96);
            a1 = __builtin_amdgcn_bitop3_b32(a1, v.z, v.w, 0x96);
        }
        base = (base + 64) & 2047;
    }
    out[blockIdx.x * 256 + t] = (float)(a0 ^ a1);
}

int launch_lds_probe(int blocks, int rounds, float *out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_lds_probe, dim3((unsigned)blocks), dim3(256), 0, stream, out, rounds);
    return check_launch(__func__);
}

int launch_compact_failed(const uint8_t *ok, int64_t F, int64_t *out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_compact_failed, dim3(1), dim3(1024), 0, stream, ok, F, out);
    return check_launch(__func__);
}

int launch_encode(const Sched &sc, const uint8_t *info, uint8_t *cw, int64_t F, hipStream_t stream)
{
    int G = kMaxThreads / sc.Z;
    if (G < 1)
        G = 1;
    const int threads = ((G * sc.Z + 63) / 64) * 64;
    const size_t lds = (size_t)G * sc.K + 2 * (size_t)G * sc.Z;
    hipLaunchKernelGGL(k_encode, dim3((unsigned)((F + G - 1) / G)), dim3(threads), lds, stream, sc, G, info, cw, F);
    return check_launch(__func__);
}

// ---------------------------------------------------------------------------
// Packed bits (bitmap encoder of Sec. 3). Bit k of a frame is bit k mod 8 of
// byte k/8; in LDS a frame's bits are 32-bit words, bit k at bit k mod 32 of
// word k/32. A thread produces one 32-bit word of a Z-bit block: its bits
// r = 32w .. 32w + nv - 1 come from source bits (r + s) mod Z, i.e. from at
// most two runs of the source block (one wrap), each read at an arbitrary
// bit position with a funnel shift. This generalises the word rotation of
// Algorithm A1 (which needs Z to be a multiple of the word size) to any Z.
// ---------------------------------------------------------------------------

// 32 bits of the word stream W starting at bit position p (W must hold one
// more word than the highest word read)
__device__ __forceinline__ uint32_t bits32(const uint32_t *W, int p)
{
    const int q = p >> 5;
    return __builtin_amdgcn_alignbit(W[q + 1], W[q], (uint32_t)(p & 31));
}

__device__ __forceinline__ uint32_t low_mask(int n) { return n >= 32 ? 0xffffffffu : ((1u << n) - 1u); }

// word w (nv valid bits) of the block at bit offset b0 of W, cyclically
// shifted by s: bit t = source bit (32w + t + s) mod Z
__device__ __forceinline__ uint32_t shifted_word(const uint32_t *W, int b0, int Z, int s, int w, int nv)
{
    int o = 32 * w + s;
    o = o >= Z ? o - Z : o;
    o = o >= Z ? o - Z : o;   // 32w < Z and s < Z
    const int L1 = nv < Z - o ? nv : Z - o;
    uint32_t x = bits32(W, b0 + o) & low_mask(L1);
    if (L1 < nv)
        x |= bits32(W, b0) << L1;
    return x & low_mask(nv);
}

// stage packed frames (nbytes each) into LDS words (nw words each, zeroed
// beyond the data) for frames f0 .. f0+G-1
__device__ __forceinline__ void stage_bytes(const uint8_t *__restrict__ src, int64_t nbytes, int nw, int G, int64_t f0,
                                            int64_t F, uint32_t *W)
{
    for (int k = threadIdx.x; k < G * nw; k += blockDim.x)
        W[k] = 0u;
    __syncthreads();
    uint8_t *Wb = (uint8_t *)W;
    for (int g = 0; g < G; ++g) {
        if (f0 + g >= F)
            break;
        const uint8_t *p = src + (f0 + g) * nbytes;
        for (int64_t b = threadIdx.x; b < nbytes; b += blockDim.x)
            Wb[(size_t)g * nw * 4 + b] = p[b];
    }
    __syncthreads();
}

__global__ __launch_bounds__(kMaxThreads) void k_shift_packed(const uint8_t *__restrict__ in, uint8_t *__restrict__ out,
                                                               int64_t F, int Z, int s, int G)
{
    extern __shared__ uint32_t lw[];
    const int ZW = (Z + 31) / 32, nw = ZW + 1;
    const int64_t nbytes = (Z + 7) / 8;
    const int64_t f0 = (int64_t)blockIdx.x * G;
    uint32_t *Wi = lw, *Wo = lw + (size_t)G * nw;
    stage_bytes(in, nbytes, nw, G, f0, F, Wi);
    const int g = threadIdx.x / ZW, w = threadIdx.x - g * ZW;
    if (g < G && f0 + g < F) {
        const int nv = Z - 32 * w < 32 ? Z - 32 * w : 32;
        Wo[g * nw + w] = shifted_word(Wi + g * nw, 0, Z, s, w, nv);
    }
    __syncthreads();
    const uint8_t *Ob = (const uint8_t *)Wo;
    for (int gg = 0; gg < G; ++gg) {
        if (f0 + gg >= F)
            break;
        for (int64_t b = threadIdx.x; b < nbytes; b += blockDim.x)
            out[(f0 + gg) * nbytes + b] = Ob[(size_t)gg * nw * 4 + b];
    }
}

// Packed direct encoder (eqs. 12-15 on 32-bit words). Thread (g, w) owns word
// w of every Z-bit block of frame g: S_i[w] (eq. 15) for all block rows in
// registers, T[w] and v_0[w] through LDS (v_0 is read at shifted positions),
// then v_1 .. v_{Mb-1} (eqs. 13-14) OR-ed into the packed codeword in LDS at
// bit offsets K + i Z + 32 w (blocks need not be word aligned).
__global__ __launch_bounds__(kMaxThreads) void k_encode_packed(const Sched sc, const int G,
                                                                const uint8_t *__restrict__ info,
                                                                uint8_t *__restrict__ cw, int64_t F)
{
    extern __shared__ uint32_t lw[];
    const int Z = sc.Z, K = sc.K, N = sc.N, Mb = sc.Mb, Kb = sc.Nb - sc.Mb;
    const int ZW = (Z + 31) / 32;
    const int kw = (K + 31) / 32 + 1, nwo = (N + 31) / 32 + 1, zw1 = ZW + 1;
    const int64_t kbytes = (K + 7) / 8, nbytes = (N + 7) / 8;
    uint32_t *U = lw;                                   // [G][kw]  information bits
    uint32_t *T = U + (size_t)G * kw;                   // [G][zw1]
    uint32_t *V0 = T + (size_t)G * zw1;                 // [G][zw1]
    uint32_t *C = V0 + (size_t)G * zw1;                 // [G][nwo] codeword
    const int64_t f0 = (int64_t)blockIdx.x * G;
    for (int k = threadIdx.x; k < G * (2 * zw1 + nwo); k += blockDim.x)
        T[k] = 0u;
    stage_bytes(info, kbytes, kw, G, f0, F, U);   // (its barriers also cover the zeroing)
    const int g = threadIdx.x / ZW, w = threadIdx.x - g * ZW;
    const bool on = g < G && f0 + g < F;
    const int nv = on ? (Z - 32 * w < 32 ? Z - 32 * w : 32) : 0;
    uint32_t S[kMaxMb];
    if (on) {
        const uint32_t *u = U + g * kw;
        uint32_t t = 0;
        for (int i = 0; i < Mb; ++i) {
            uint32_t acc = 0;
            for (int e = 0; e < sc.deg[i]; ++e) {
                const uint32_t ew = sc.edge[i][e];
                const int col = (int)(ew >> 16);
                if (col >= Kb)
                    break;   // ascending columns: the rest are parity columns
                acc ^= shifted_word(u, col * Z, Z, (int)(ew & 0xffffu), w, nv);
            }
            S[i] = acc;
            t ^= acc;
        }
        T[g * zw1 + w] = t;   // T = xor_i S_i
    }
    __syncthreads();
    if (on) {
        const int hy = sc.hb[sc.enc_y];
        V0[g * zw1 + w] = shifted_word(T + g * zw1, 0, Z, hy == 0 ? 0 : Z - hy, w, nv);   // eq. 12
    }
    __syncthreads();
    if (on) {
        const uint32_t *v0 = V0 + g * zw1;
        uint32_t *c = C + g * nwo;
        auto put = [&](int bit, uint32_t x) {
            const int q = bit >> 5, sh = bit & 31;
            atomicOr(&c[q], x << sh);
            if (sh && sh + nv > 32)
                atomicOr(&c[q + 1], x >> (32 - sh));
        };
        uint32_t v = v0[w];
        put(K + 32 * w, v);
        const int h0 = sc.hb[0];
        v = shifted_word(v0, 0, Z, h0, w, nv) ^ S[0];                          // eq. 13
        put(K + Z + 32 * w, v);
        for (int i = 1; i <= Mb - 2; ++i) {
            const int hi = sc.hb[i];
            v ^= S[i] ^ (hi >= 0 ? shifted_word(v0, 0, Z, hi, w, nv) : 0u);   // eq. 14
            put(K + (i + 1) * Z + 32 * w, v);
        }
        // systematic part: the information words (the last one masked to K bits)
        for (int q = w; q < (K + 31) / 32; q += ZW) {
            const int rem = K - 32 * q;
            atomicOr(&c[q], U[g * kw + q] & low_mask(rem));
        }
    }
    __syncthreads();
    const uint8_t *Cb = (const uint8_t *)C;
    for (int gg = 0; gg < G; ++gg) {
        if (f0 + gg >= F)
            break;
        for (int64_t b = threadIdx.x; b < nbytes; b += blockDim.x)
            cw[(f0 + gg) * nbytes + b] = Cb[(size_t)gg * nwo * 4 + b];
    }
}

int launch_shift_packed(const uint8_t *in, uint8_t *out, int64_t F, int Z, int s, hipStream_t stream)
{
    const int ZW = (Z + 31) / 32;
    int G = kMaxThreads / ZW;
    G = G < 1 ? 1 : G;
    const size_t lds = 2 * (size_t)G * (ZW + 1) * 4;
    hipLaunchKernelGGL(k_shift_packed, dim3((unsigned)((F + G - 1) / G)), dim3(kMaxThreads), lds, stream, in, out,
                       F, Z, s, G);
    return check_launch(__func__);
}

int launch_encode_packed(const Sched &sc, const uint8_t *info, uint8_t *cw, int64_t F, hipStream_t stream)
{
    const int ZW = (sc.Z + 31) / 32;
    const int per_frame = ((sc.K + 31) / 32 + 1) + 2 * (ZW + 1) + ((sc.N + 31) / 32 + 1);   // words
    int G = kMaxThreads / ZW;
    while (G > 1 && (size_t)G * per_frame * 4 > (size_t)kLdsBudget)
        --G;
    const size_t lds = (size_t)G * per_frame * 4;
    hipLaunchKernelGGL(k_encode_packed, dim3((unsigned)((F + G - 1) / G)), dim3(kMaxThreads), lds, stream, sc, G,
                       info, cw, F);
    return check_launch(__func__);
}

}  // namespace ldpc
