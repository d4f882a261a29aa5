// Host side of libldpc: the C ABI, argument validation, the QC base-matrix
// compiler (base matrix -> per-layer gather schedule) and launch planning.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "ldpc_internal.h"

namespace ldpc {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = '\0'; }

int check_launch(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(LDPC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return LDPC_OK;
}

// Row y of the direct encoder (Sec. 1, eqs. 3-7; Sec. 2 eq. 12): h_b (column
// K_b) must hold equal non-negative values in rows 0 and Mb-1 and exactly one
// more non-negative value in between (row y); H_b2' must be the staircase of
// zero shifts at (c, c) and (c+1, c). Returns y or -1.
static int encoder_row(const int16_t *hbm, int Mb, int Nb)
{
    const int Kb = Nb - Mb;
    if (Mb < 3)
        return -1;
    const int top = hbm[Kb], bottom = hbm[(Mb - 1) * Nb + Kb];
    if (top < 0 || top != bottom)
        return -1;
    int y = -1, count = 0;
    for (int i = 1; i + 1 < Mb; ++i)
        if (hbm[i * Nb + Kb] >= 0) {
            y = i;
            ++count;
        }
    if (count != 1)
        return -1;
    for (int c = 0; c + 1 < Mb; ++c)
        for (int i = 0; i < Mb; ++i) {
            const int v = hbm[i * Nb + Kb + 1 + c];
            if (v != ((i == c || i == c + 1) ? 0 : -1))
                return -1;
        }
    return y;
}

int compile_sched(const int16_t *hbm, int Mb, int Nb, int Z, bool need_deg2, Sched *out)
{
    if (!hbm)
        return fail(LDPC_EINVAL, "base matrix pointer is null");
    if (Mb < 1 || Nb <= Mb || Z < 1)
        return fail(LDPC_EINVAL, "bad code dimensions Mb=%d Nb=%d Z=%d (need Mb >= 1, Nb > Mb, Z >= 1)", Mb, Nb, Z);
    if (Mb > kMaxMb || Nb > kMaxNb || Z > kMaxZ)
        return fail(LDPC_ERANGE, "code Mb=%d Nb=%d Z=%d exceeds kernel limits (%d, %d, %d)", Mb, Nb, Z, kMaxMb, kMaxNb,
                    kMaxZ);
    Sched s;
    memset(&s, 0, sizeof(s));
    s.Z = Z;
    s.Mb = Mb;
    s.Nb = Nb;
    s.N = Nb * Z;
    s.K = (Nb - Mb) * Z;
    s.M = Mb * Z;
    for (int i = 0; i < Mb; ++i) {
        int d = 0;
        for (int j = 0; j < Nb; ++j) {
            const int v = hbm[i * Nb + j];
            if (v < -1 || v >= Z)
                return fail(LDPC_EINVAL, "H_bm(%d,%d) = %d outside [-1, Z-1] for Z=%d", i, j, v, Z);
            if (v < 0)
                continue;
            if (d >= kMaxDeg)
                return fail(LDPC_ERANGE, "block row %d has more than %d non-zero blocks", i, kMaxDeg);
            s.edge[i][d++] = ((uint32_t)j << 16) | (uint32_t)v;
        }
        if (need_deg2 && d < 2)
            return fail(LDPC_EINVAL, "block row %d has check degree %d (< 2)", i, d);
        s.deg[i] = d;
        s.dmax = std::max(s.dmax, d);
        s.E += d * Z;
        s.hb[i] = hbm[i * Nb + (Nb - Mb)];
    }
    s.enc_y = encoder_row(hbm, Mb, Nb);
    *out = s;
    return LDPC_OK;
}

DecodeLaunch make_launch(const Sched &sc, int elem_bytes, int G, int KF, int max_threads)
{
    DecodeLaunch lc{};
    const int FW = G * KF;
    if (G < 1 || KF < 1 || FW > 64 || G * sc.Z > max_threads)
        return lc;
    int FWp = FW;
    if (elem_bytes == 4)
        FWp = FW | 1;                       // odd dword stride: consecutive rows hit distinct banks
    else
        while (FWp % 4 != 2)
            ++FWp;                          // odd dword stride for 2-byte elements
    const size_t lds = (size_t)(sc.N + sc.Z) * FWp * elem_bytes;   // one column block of padding
    if (lds > (size_t)kLdsBudget)
        return lc;
    lc = DecodeLaunch{G, KF, FW, FWp, ((G * sc.Z + 63) / 64) * 64, lds, 0};
    return lc;
}

DecodeLaunch plan_decode(const Sched &sc, int elem_bytes, int kf_hint)
{
    DecodeLaunch best{};
    double best_util = -1.0;
    const int kf = kf_hint > 0 ? kf_hint : 2;
    for (int KF = kf; KF >= 1; --KF) {
        for (int G = 1; G * sc.Z <= kMaxThreads; ++G) {
            const DecodeLaunch lc = make_launch(sc, elem_bytes, G, KF, kMaxThreads);
            if (lc.G < 1)
                break;
            const double util = (double)(G * sc.Z) / lc.threads;
            if (util > best_util + 1e-9 || (util > best_util - 1e-9 && lc.FW > best.FW)) {
                best_util = util;
                best = lc;
            }
        }
        if (best_util > 0)
            break;
    }
    return best;
}

}  // namespace ldpc

using namespace ldpc;

namespace {

bool bad_ptrs(std::initializer_list<const void *> ps)
{
    for (const void *p : ps)
        if (!p)
            return true;
    return false;
}

int device_status(int rc, const char *what)
{
    // launchers already recorded the HIP error text; keep the entry point's name
    if (rc != LDPC_OK && ldpc_last_error()[0] == '\0')
        return fail(rc, "%s failed", what);
    return rc;
}

int decode_common_checks(const Sched &sc, int64_t F, int max_iter)
{
    (void)sc;
    if (F < 0)
        return fail(LDPC_EINVAL, "negative frame count %lld", (long long)F);
    if (max_iter < 1)
        return fail(LDPC_EINVAL, "max_iter must be >= 1 (got %d)", max_iter);
    return LDPC_OK;
}

}  // namespace

extern "C" {

const char *ldpc_last_error(void) { return g_err; }

void ldpc_cache_clear(void)
{
    jit_cache_clear();
    tune_cache_clear();
}

int ldpc_code_info(const int16_t *hbm, int Mb, int Nb, int Z, int64_t out[8])
{
    clear_error();
    if (!out || !hbm)
        return fail(LDPC_EINVAL, "null pointer");
    if (Mb < 1 || Nb <= Mb || Z < 1)
        return fail(LDPC_EINVAL, "bad code dimensions Mb=%d Nb=%d Z=%d", Mb, Nb, Z);
    int64_t E = 0, dmax = 0;
    for (int i = 0; i < Mb; ++i) {
        int64_t d = 0;
        for (int j = 0; j < Nb; ++j) {
            const int v = hbm[i * Nb + j];
            if (v < -1 || v >= Z)
                return fail(LDPC_EINVAL, "H_bm(%d,%d) = %d outside [-1, Z-1]", i, j, v);
            d += v >= 0;
        }
        E += d * Z;
        dmax = std::max(dmax, d);
    }
    out[0] = (int64_t)Nb * Z;
    out[1] = (int64_t)(Nb - Mb) * Z;
    out[2] = (int64_t)Mb * Z;
    out[3] = E;
    out[4] = dmax;
    out[5] = encoder_row(hbm, Mb, Nb);
    out[6] = Mb;
    out[7] = Nb;
    return LDPC_OK;
}

int ldpc_encode(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *info, uint8_t *cw, int64_t F,
                void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, false, &sc);
    if (rc)
        return rc;
    if (sc.enc_y < 0)
        return fail(LDPC_ESTRUCT, "base matrix lacks the dual-diagonal parity structure of the direct encoder");
    if (F < 0)
        return fail(LDPC_EINVAL, "negative frame count");
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({info, cw}))
        return fail(LDPC_EINVAL, "null device pointer");
    if (sc.Mb > 31)
        return fail(LDPC_ERANGE, "encoder supports at most 31 block rows");
    return device_status(launch_encode(sc, info, cw, F, (hipStream_t)stream), "ldpc_encode");
}

int ldpc_encode_packed(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *info, uint8_t *cw, int64_t F,
                       void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, false, &sc);
    if (rc)
        return rc;
    if (sc.enc_y < 0)
        return fail(LDPC_ESTRUCT, "base matrix lacks the dual-diagonal parity structure of the direct encoder");
    if (F < 0)
        return fail(LDPC_EINVAL, "negative frame count");
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({info, cw}))
        return fail(LDPC_EINVAL, "null device pointer");
    if ((size_t)((sc.K + 31) / 32 + 1 + 2 * ((sc.Z + 31) / 32 + 1) + (sc.N + 31) / 32 + 1) * 4 > (size_t)kLdsBudget)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the packed encoder's LDS budget", sc.N);
    return device_status(launch_encode_packed(sc, info, cw, F, (hipStream_t)stream), "ldpc_encode_packed");
}

int ldpc_shift_packed(const uint8_t *in, uint8_t *out, int64_t F, int Z, int s, void *stream)
{
    clear_error();
    if (F < 0 || Z < 1 || Z > LDPC_MAX_Z || s < 0 || s >= Z)
        return fail(LDPC_EINVAL, "need F >= 0, 1 <= Z <= %d and 0 <= s < Z", LDPC_MAX_Z);
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({in, out}))
        return fail(LDPC_EINVAL, "null device pointer");
    return device_status(launch_shift_packed(in, out, F, Z, s, (hipStream_t)stream), "ldpc_shift_packed");
}

int ldpc_decode_f32(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, int64_t F, int max_iter,
                    float alpha, int early_term, const float *w, uint8_t *bits, float *post, int32_t *iters,
                    uint8_t *ok, void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if ((rc = decode_common_checks(sc, F, max_iter)))
        return rc;
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({llr, bits, iters}))
        return fail(LDPC_EINVAL, "null device pointer (llr, bits and iters are required)");
    DecodeLaunch lc = plan_decode(sc, 4, 2);
    if (lc.G < 1)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the decoder's LDS budget", sc.N);
    if (jit_enabled()) {
        lc = decode_layout(sc, 0, w ? 1 : 0);
        return launch_jit_decode(sc, lc, 0, w ? 1 : 0, llr, nullptr, F, max_iter, alpha, 0, 0, early_term, w, bits,
                                 post, iters, ok, (hipStream_t)stream);
    }
    return device_status(launch_decode_f32(sc, lc, llr, nullptr, F, max_iter, alpha, early_term, w, bits, post,
                                           iters, ok, (hipStream_t)stream),
                         "ldpc_decode_f32");
}

int ldpc_decode_i8(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter,
                   int offset, int wq, const uint8_t *wq_table, int early_term, uint8_t *bits, int16_t *post,
                   int32_t *iters, uint8_t *ok, void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if ((rc = decode_common_checks(sc, F, max_iter)))
        return rc;
    if (offset < 0 || offset > 127)
        return fail(LDPC_EINVAL, "offset must be in [0, 127] (got %d)", offset);
    if (wq < 0 || wq > 31)
        return fail(LDPC_EINVAL, "wq must be in [0, 31] (got %d)", wq);
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({llr, bits, iters}))
        return fail(LDPC_EINVAL, "null device pointer (llr, bits and iters are required)");
    DecodeLaunch lc = plan_decode(sc, 2, 2);
    if (lc.G < 1)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the decoder's LDS budget", sc.N);
    if (jit_enabled()) {
        lc = decode_layout(sc, 1, wq_table ? 2 : (wq > 0 ? 1 : 0));
        return launch_jit_decode(sc, lc, 1, wq_table ? 2 : (wq > 0 ? 1 : 0), llr, nullptr, F, max_iter, 0.0f, offset,
                                 wq, early_term, wq_table, bits, post, iters, ok, (hipStream_t)stream);
    }
    return device_status(launch_decode_i8(sc, lc, llr, nullptr, F, max_iter, offset, wq, wq_table, early_term, bits,
                                          post, iters, ok, (hipStream_t)stream),
                         "ldpc_decode_i8");
}

int ldpc_decode_f32_packed(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, int64_t F, int max_iter,
                           float alpha, int early_term, const float *w, uint8_t *bits, float *post, int32_t *iters,
                           uint8_t *ok, void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if ((rc = decode_common_checks(sc, F, max_iter)))
        return rc;
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({llr, bits, iters}))
        return fail(LDPC_EINVAL, "null device pointer (llr, bits and iters are required)");
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "packed output needs run-time specialisation (LDPC_JIT=0 is set)");
    DecodeLaunch lc = jit_default_launch(sc, 0);
    if (lc.G < 1)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the decoder's LDS budget", sc.N);
    lc = decode_layout(sc, 0, w ? 1 : 0);
    return launch_jit_decode(sc, lc, 0, w ? 1 : 0, llr, nullptr, F, max_iter, alpha, 0, 0, early_term, w, bits, post,
                             iters, ok, (hipStream_t)stream, nullptr, true);
}

int ldpc_decode_i8_packed(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter,
                          int offset, int wq, const uint8_t *wq_table, int early_term, uint8_t *bits, int16_t *post,
                          int32_t *iters, uint8_t *ok, void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if ((rc = decode_common_checks(sc, F, max_iter)))
        return rc;
    if (offset < 0 || offset > 127)
        return fail(LDPC_EINVAL, "offset must be in [0, 127] (got %d)", offset);
    if (wq < 0 || wq > 31)
        return fail(LDPC_EINVAL, "wq must be in [0, 31] (got %d)", wq);
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({llr, bits, iters}))
        return fail(LDPC_EINVAL, "null device pointer (llr, bits and iters are required)");
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "packed output needs run-time specialisation (LDPC_JIT=0 is set)");
    DecodeLaunch lc = jit_default_launch(sc, 1);
    if (lc.G < 1)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the decoder's LDS budget", sc.N);
    lc = decode_layout(sc, 1, wq_table ? 2 : (wq > 0 ? 1 : 0));
    return launch_jit_decode(sc, lc, 1, wq_table ? 2 : (wq > 0 ? 1 : 0), llr, nullptr, F, max_iter, 0.0f, offset, wq,
                             early_term, wq_table, bits, post, iters, ok, (hipStream_t)stream, nullptr, true);
}

static int flood_common(const int16_t *hbm, int Mb, int Nb, int Z, const void *llr, int64_t F, int max_iter,
                        const void *bits, const int32_t *iters, Sched *sc, DecodeLaunch *lc)
{
    clear_error();
    int rc = compile_sched(hbm, Mb, Nb, Z, true, sc);
    if (rc)
        return rc;
    if ((rc = decode_common_checks(*sc, F, max_iter)))
        return rc;
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({llr, bits, iters}))
        return fail(LDPC_EINVAL, "null device pointer (llr, bits and iters are required)");
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "the flooding decoder needs run-time specialisation (LDPC_JIT=0 is set)");
    *lc = flood_launch(*sc);
    if (lc->G < 1)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the flooding decoder's LDS budget", sc->N);
    return LDPC_OK;
}

int ldpc_decode_flood_f32(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, int64_t F, int max_iter,
                          float alpha, int early_term, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok,
                          void *stream)
{
    Sched sc;
    DecodeLaunch lc{};
    int rc = flood_common(hbm, Mb, Nb, Z, llr, F, max_iter, bits, iters, &sc, &lc);
    if (rc || F == 0)
        return rc;
    return launch_jit_flood(sc, lc, 0, 0, llr, F, max_iter, alpha, 0, 0, early_term, bits, post, iters, ok,
                            (hipStream_t)stream);
}

int ldpc_decode_flood_i8(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter,
                         int offset, int wq, int early_term, uint8_t *bits, int16_t *post, int32_t *iters,
                         uint8_t *ok, void *stream)
{
    if (offset < 0 || offset > 127)
        return fail(LDPC_EINVAL, "offset must be in [0, 127] (got %d)", offset);
    if (wq < 0 || wq > 31)
        return fail(LDPC_EINVAL, "wq must be in [0, 31] (got %d)", wq);
    Sched sc;
    DecodeLaunch lc{};
    int rc = flood_common(hbm, Mb, Nb, Z, llr, F, max_iter, bits, iters, &sc, &lc);
    if (rc || F == 0)
        return rc;
    return launch_jit_flood(sc, lc, 1, wq > 0 ? 1 : 0, llr, F, max_iter, 0.0f, offset, wq, early_term, bits, post,
                            iters, ok, (hipStream_t)stream);
}

int ldpc_autotune_decode(const int16_t *hbm, int Mb, int Nb, int Z, int path, int max_iter, int64_t F,
                         int32_t out[7], float *ms, void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if (path < 0 || path > 3)
        return fail(LDPC_EINVAL, "path must be 0 (FP32), 1 (int8), 2 (FP32 weight table) or 3 (int8 weight table)");
    if (max_iter < 1 || F < 1)
        return fail(LDPC_EINVAL, "max_iter and F must be >= 1");
    if (!out || !ms)
        return fail(LDPC_EINVAL, "null output pointer");
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "the autotuner needs run-time specialised kernels (LDPC_JIT=0 is set)");
    DecodeLaunch best{};
    if ((rc = autotune_decode(sc, path, max_iter, F, (hipStream_t)stream, &best, ms)))
        return rc;
    out[0] = best.G;
    out[1] = best.KF;
    out[2] = best.FWp;
    out[3] = best.threads;
    out[4] = best.hoist;
    out[5] = best.h2;
    out[6] = best.waves;
    return LDPC_OK;
}

static void layout_row(const DecodeLaunch &lc, int32_t *o)
{
    o[0] = lc.G;
    o[1] = lc.KF;
    o[2] = lc.FWp;
    o[3] = lc.threads;
    o[4] = lc.hoist;
    o[5] = lc.h2;
    o[6] = lc.waves;
}

int ldpc_decode_layouts(const int16_t *hbm, int Mb, int Nb, int Z, int path, int32_t *out, int cap)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if (path < 0 || path > 3)
        return fail(LDPC_EINVAL, "path must be 0 (FP32), 1 (int8), 2 (FP32 weight table) or 3 (int8 weight table)");
    if (cap < 0 || (cap > 0 && !out))
        return fail(LDPC_EINVAL, "negative capacity or null output pointer");
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "decode layouts need run-time specialised kernels (LDPC_JIT=0 is set)");
    std::vector<DecodeLaunch> v;
    if ((rc = tuner_layouts(sc, path, &v, nullptr)))
        return rc;
    for (int k = 0; k < (int)v.size() && k < cap; ++k)
        layout_row(v[k], out + 7 * k);
    return (int)v.size();
}

int ldpc_set_decode_layout(const int16_t *hbm, int Mb, int Nb, int Z, int path, const int32_t layout[7])
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if (path < 0 || path > 3)
        return fail(LDPC_EINVAL, "path must be 0 (FP32), 1 (int8), 2 (FP32 weight table) or 3 (int8 weight table)");
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "decode layouts need run-time specialised kernels (LDPC_JIT=0 is set)");
    if (!layout) {
        clear_tuned_launch(sc, path);
        return LDPC_OK;
    }
    const int G = layout[0], KF = layout[1], hoist = layout[4], h2 = layout[5], waves = layout[6];
    if (h2 != 0 && h2 != 1)
        return fail(LDPC_EINVAL, "packed-FP16 flag must be 0 or 1");
    if (h2 && ((path & 1) != 1 || !h2_eligible(sc) || KF != 1))
        return fail(LDPC_EINVAL, "two frames per lane needs the fixed-point path (1 or 3), KF = 1 and column "
                    "weight <= 15");
    DecodeLaunch lc = h2 ? make_h2_launch(sc, G, kMaxThreads) : make_launch(sc, 4, G, KF, kMaxThreads);
    if (lc.G < 1 || KF < 1 || KF > 2)
        return fail(LDPC_ERANGE, "layout G=%d KF=%d does not fit this code (threads, LDS or frames per workgroup)", G,
                    KF);
    if (layout[2] != lc.FWp || layout[3] != lc.threads)
        return fail(LDPC_EINVAL, "FWp %d / threads %d do not match G=%d KF=%d (expected %d / %d)", layout[2],
                    layout[3], G, KF, lc.FWp, lc.threads);
    if (hoist < 0 || hoist > sc.Mb)
        return fail(LDPC_EINVAL, "hoisted block rows must be in [0, Mb]");
    if (waves != 0 && waves != 3 && waves != 4)
        return fail(LDPC_EINVAL, "waves must be 0, 3 or 4");
    lc.hoist = hoist;
    lc.waves = waves;
    lc.tuned = 1;
    set_tuned_launch(sc, path, lc);
    return LDPC_OK;
}

size_t ldpc_nms_ckpt_bytes(const int16_t *hbm, int Mb, int Nb, int Z, int64_t F, int T)
{
    clear_error();
    Sched sc;
    if (compile_sched(hbm, Mb, Nb, Z, true, &sc) || F < 0 || T < 1)
        return 0;
    return nms_ckpt_floats(sc, F, T) * sizeof(float);
}

int ldpc_nms_fwd(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, const uint8_t *cw, int64_t F, int T,
                 const float *w, void *ckpt, size_t ckpt_bytes, float *loss, float *post, void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if (F < 1 || T < 1)
        return fail(LDPC_EINVAL, "F and T must be >= 1");
    if (bad_ptrs({llr, cw, w, ckpt, loss}))
        return fail(LDPC_EINVAL, "null device pointer (llr, cw, w, ckpt and loss are required)");
    if (ckpt_bytes < nms_ckpt_floats(sc, F, T) * sizeof(float))
        return fail(LDPC_EINVAL, "checkpoint buffer too small: %zu < %zu bytes", ckpt_bytes,
                    nms_ckpt_floats(sc, F, T) * sizeof(float));
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "the training kernels need run-time specialisation (LDPC_JIT=0 is set)");
    return launch_nms_fwd(sc, llr, cw, F, T, w, (float *)ckpt, loss, post, (hipStream_t)stream);
}

int ldpc_nms_bwd(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *cw, int64_t F, int T, const float *w,
                 void *ckpt, size_t ckpt_bytes, const float *dloss, float *grad_w, void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if (F < 1 || T < 1)
        return fail(LDPC_EINVAL, "F and T must be >= 1");
    if (bad_ptrs({cw, w, ckpt, dloss, grad_w}))
        return fail(LDPC_EINVAL, "null device pointer (cw, w, ckpt, dloss and grad_w are required)");
    if (ckpt_bytes < nms_ckpt_floats(sc, F, T) * sizeof(float))
        return fail(LDPC_EINVAL, "checkpoint buffer too small");
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "the training kernels need run-time specialisation (LDPC_JIT=0 is set)");
    return launch_nms_bwd(sc, cw, F, T, w, (float *)ckpt, dloss, grad_w, (hipStream_t)stream);
}

int ldpc_random_bits(uint64_t seed, const uint64_t *seed_dev, int64_t F, int64_t K, uint8_t *info, void *stream)
{
    clear_error();
    if (F < 0 || K < 0)
        return fail(LDPC_EINVAL, "negative size");
    if (F == 0 || K == 0)
        return LDPC_OK;
    if (!info)
        return fail(LDPC_EINVAL, "null device pointer");
    return device_status(launch_random_bits(seed, seed_dev, F, K, info, (hipStream_t)stream), "ldpc_random_bits");
}

int ldpc_awgn_llr(uint64_t seed, const uint64_t *seed_dev, const uint8_t *cw, int64_t F, int64_t N, float sigma,
                  float scale, const float *sigma_f, const float *scale_f, float *llr, void *stream)
{
    clear_error();
    if (F < 0 || N < 0)
        return fail(LDPC_EINVAL, "negative size");
    if (F == 0 || N == 0)
        return LDPC_OK;
    if (bad_ptrs({cw, llr}))
        return fail(LDPC_EINVAL, "null device pointer");
    if (N >= (int64_t(1) << 34))
        return fail(LDPC_ERANGE, "frame length too large for the noise counter");
    if ((sigma_f == nullptr) != (scale_f == nullptr))
        return fail(LDPC_EINVAL, "per-frame sigma and scale must be given together");
    return device_status(launch_awgn_llr(seed, seed_dev, F, N, cw, sigma, scale, sigma_f, scale_f, llr,
                                         (hipStream_t)stream),
                         "ldpc_awgn_llr");
}

int ldpc_frame_stats(const uint8_t *bits, const uint8_t *info, const int32_t *iters, const uint8_t *ok, int64_t F,
                     int64_t N, int64_t K, int64_t *counters, void *stream)
{
    clear_error();
    if (F < 0 || K < 0 || N < K)
        return fail(LDPC_EINVAL, "bad sizes F=%lld N=%lld K=%lld", (long long)F, (long long)N, (long long)K);
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({bits, info, counters}))
        return fail(LDPC_EINVAL, "null device pointer (bits, info and counters are required)");
    return device_status(launch_frame_stats(bits, info, iters, ok, F, N, K, counters, (hipStream_t)stream),
                         "ldpc_frame_stats");
}

int ldpc_lds_probe(int blocks, int rounds, float *out, void *stream)
{
    clear_error();
    if (blocks < 1 || rounds < 1 || blocks > (1 << 20) || rounds > (1 << 20))
        return fail(LDPC_EINVAL, "blocks and rounds must be in [1, 2^20]");
    if (bad_ptrs({out}))
        return fail(LDPC_EINVAL, "null device pointer");
    return device_status(launch_lds_probe(blocks, rounds, out, (hipStream_t)stream), "ldpc_lds_probe");
}

namespace {

// Re-decodes, from their channel LLRs and with fresh state, the frames whose
// ok flag is 0, with plain normalised (or offset) min-sum and early
// termination; their bits, posteriors, iterations and ok are overwritten.
int fallback(const int16_t *hbm, int Mb, int Nb, int Z, int path, const void *llr, int64_t F, int max_iter,
             float alpha, int offset, int wq, uint8_t *bits, void *post, int32_t *iters, uint8_t *ok, int64_t *work,
             hipStream_t stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if ((rc = decode_common_checks(sc, F, max_iter)))
        return rc;
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({llr, bits, iters, ok, work}))
        return fail(LDPC_EINVAL, "null device pointer (llr, bits, iters, ok and work are required)");
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "the fallback decoder needs run-time specialisation (LDPC_JIT=0 is set)");
    DecodeLaunch lc = jit_default_launch(sc, path);
    if (lc.G < 1)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the decoder's LDS budget", sc.N);
    tuned_launch(sc, path, &lc);
    const int mode = path == 0 ? 0 : (wq > 0 ? 1 : 0);
    lc = usable_launch(sc, lc, path, mode);
    if ((rc = launch_compact_failed(ok, F, work, stream)))
        return device_status(rc, "fallback compaction");
    return launch_jit_decode(sc, lc, path, mode, llr, work + 1, F, max_iter, alpha, offset, wq, 1, nullptr, bits, post,
                             iters, ok, stream, work);
}

}  // namespace

int ldpc_fallback_f32(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, int64_t F, int max_iter,
                      float alpha, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok, int64_t *work,
                      void *stream)
{
    return fallback(hbm, Mb, Nb, Z, 0, llr, F, max_iter, alpha, 0, 0, bits, post, iters, ok, work,
                    (hipStream_t)stream);
}

int ldpc_fallback_i8(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter, int offset,
                     int wq, uint8_t *bits, int16_t *post, int32_t *iters, uint8_t *ok, int64_t *work, void *stream)
{
    if (offset < 0 || offset > 127 || wq < 0 || wq > 31)
        return fail(LDPC_EINVAL, "offset must be in [0, 127] and wq in [0, 31]");
    return fallback(hbm, Mb, Nb, Z, 1, llr, F, max_iter, 0.0f, offset, wq, bits, post, iters, ok, work,
                    (hipStream_t)stream);
}

int ldpc_quantize_q16(const float *llr, int16_t *q, int64_t n, float scale, int qmax, void *stream)
{
    clear_error();
    if (n < 0 || qmax < 1 || qmax > 32767)
        return fail(LDPC_EINVAL, "negative size or qmax outside [1, 32767]");
    if (n == 0)
        return LDPC_OK;
    if (bad_ptrs({llr, q}))
        return fail(LDPC_EINVAL, "null device pointer");
    return device_status(launch_quantize_q16(llr, q, n, scale, qmax, (hipStream_t)stream), "ldpc_quantize_q16");
}

int ldpc_decode_q16(const int16_t *hbm, int Mb, int Nb, int Z, const int16_t *llr, int64_t F, int max_iter, int wq,
                    int wrap, int early_term, uint8_t *bits, int16_t *post, int32_t *iters, uint8_t *ok, void *stream)
{
    clear_error();
    Sched sc;
    int rc = compile_sched(hbm, Mb, Nb, Z, true, &sc);
    if (rc)
        return rc;
    if ((rc = decode_common_checks(sc, F, max_iter)))
        return rc;
    if (wq < 1 || wq > 31)
        return fail(LDPC_EINVAL, "wq must be in [1, 31] (got %d)", wq);
    if (F == 0)
        return LDPC_OK;
    if (bad_ptrs({llr, bits, iters}))
        return fail(LDPC_EINVAL, "null device pointer (llr, bits and iters are required)");
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "the int16 decoder needs run-time specialisation (LDPC_JIT=0 is set)");
    DecodeLaunch lc = jit_default_launch(sc, 0);
    if (lc.G < 1)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the decoder's LDS budget", sc.N);
    return launch_jit_q16(sc, lc, wrap ? 1 : 0, llr, F, max_iter, wq, early_term, bits, post, iters, ok,
                          (hipStream_t)stream);
}

int ldpc_quantize_i8(const float *llr, int8_t *q, int64_t n, float scale, void *stream)
{
    clear_error();
    if (n < 0)
        return fail(LDPC_EINVAL, "negative size");
    if (n == 0)
        return LDPC_OK;
    if (bad_ptrs({llr, q}))
        return fail(LDPC_EINVAL, "null device pointer");
    return device_status(launch_quantize_i8(llr, q, n, scale, (hipStream_t)stream), "ldpc_quantize_i8");
}

int ldpc_quantize_weights(const float *w, uint8_t *wq, int64_t n, void *stream)
{
    clear_error();
    if (n < 0)
        return fail(LDPC_EINVAL, "negative size");
    if (n == 0)
        return LDPC_OK;
    if (bad_ptrs({w, wq}))
        return fail(LDPC_EINVAL, "null device pointer");
    return device_status(launch_quantize_weights(w, wq, n, (hipStream_t)stream), "ldpc_quantize_weights");
}

}  // extern "C"
