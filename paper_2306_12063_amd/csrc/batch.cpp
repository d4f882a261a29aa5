// Code sets and the batched (mixed-code) decode path.
//
// A code set holds several codes. Codes with the same block structure
// (block rows, block columns and non-zero block positions) form a class:
// the persistent kernel of jit_batch.hip is compiled once per code set with
// each class's degrees and columns as constants, and reads each code's Z,
// shifts and layout from the device tables built here. A batched decode is
// six stream-ordered kernels (clear, histogram by code, plan, work items,
// scatter of frame indices, persistent decode) with no host synchronisation,
// so a caller may capture it in a hipGraph.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <sstream>
#include <string>
#include <vector>

#include "ldpc_internal.h"

struct ldpc_codeset {
    int device = 0;
    int ncodes = 0;
    std::vector<ldpc::Sched> sc;
    std::vector<int> cls;              // class of each code
    std::vector<int> class_rep;        // a code of each class
    int cmb = 0, cd = 0;               // largest block-row count and degree
    bool h2 = false;                   // fixed point with two frames per lane in packed FP16
    // per arithmetic path (0 FP32, 1 fixed point): layout and device tables
    int threads[2] = {256, 256};       // workgroup size of the persistent kernel
    int gdiv[2] = {1, 1};              // frames per item = floor(threads / Z) / gdiv (at most 64)
    void *d_codes[2] = {nullptr, nullptr};
    void *d_etab[2] = {nullptr, nullptr};
    size_t lds_elems[2] = {0, 0};
    std::vector<int> G[2];             // frames per work item of each code
};

namespace ldpc {

constexpr int kNumBatchLayouts = 6;
extern const int kBatchLayouts[kNumBatchLayouts][2];

namespace {

struct CodeRec {
    int Z, N, cls, G, FWp, etab, pad0, pad1;
};

bool same_structure(const Sched &a, const Sched &b)
{
    if (a.Mb != b.Mb || a.Nb != b.Nb)
        return false;
    for (int i = 0; i < a.Mb; ++i) {
        if (a.deg[i] != b.deg[i])
            return false;
        for (int e = 0; e < a.deg[i]; ++e)
            if ((a.edge[i][e] >> 16) != (b.edge[i][e] >> 16))
                return false;
    }
    return true;
}

// odd dword stride: consecutive rows of a frame hit distinct LDS banks (the
// posteriors are FP32 in LDS on both paths)
int fwp_for(int G) { return G | 1; }

std::string batch_prelude(const ldpc_codeset &cs, int path, int mode)
{
    std::ostringstream o;
    const int nclass = (int)cs.class_rep.size();
    // edges per thread (one message register each) of the largest class
    int max_edges = 0;
    for (int c = 0; c < nclass; ++c) {
        const Sched &s = cs.sc[cs.class_rep[c]];
        int e = 0;
        for (int i = 0; i < s.Mb; ++i)
            e += s.deg[i];
        max_edges = std::max(max_edges, e);
    }
    // three waves per SIMD: measured on the 114-code WiMAX-shaped set
    // (up to 102 edges per class), where it holds with a few spilled
    // registers and makes the packed fixed-point batch 1.3x faster
    const int waves = max_edges <= 112 ? 3 : 0;
    o << "#define LDPC_WAVES_HINT " << waves << "\n";
    o << "#define LDPC_THREADS " << cs.threads[path] << "\n#define LDPC_LDS " << cs.lds_elems[path]
      << "\n#define LDPC_PATH " << path << "\n#define LDPC_MODE " << mode
      << "\n#define LDPC_H2 " << (path == 1 && cs.h2 ? 1 : 0) << "\n#define LDPC_NCLASS " << nclass
      << "\n#define LDPC_CMB " << cs.cmb << "\n#define LDPC_CD " << cs.cd << "\n";
    o << "__device__ constexpr int kMBc[" << nclass << "] = {";
    for (int c = 0; c < nclass; ++c)
        o << cs.sc[cs.class_rep[c]].Mb << (c + 1 < nclass ? "," : "};\n");
    o << "__device__ constexpr int kDegc[" << nclass << "][" << cs.cmb << "] = {";
    for (int c = 0; c < nclass; ++c) {
        const Sched &s = cs.sc[cs.class_rep[c]];
        o << "{";
        for (int i = 0; i < cs.cmb; ++i)
            o << (i < s.Mb ? s.deg[i] : 0) << (i + 1 < cs.cmb ? "," : "");
        o << "}" << (c + 1 < nclass ? "," : "};\n");
    }
    o << "#define LDPC_CLASS_CASES";
    for (int c = 0; c < nclass; ++c)
        o << " LDPC_CLASS_CASE(" << c << ")";
    o << "\n";
    return o.str();
}

}  // namespace

extern const char kJitBatchSource[];

// Layouts of the persistent kernel the batch autotuner times: {workgroup
// threads, divisor of the frames per work item}.
const int kBatchLayouts[kNumBatchLayouts][2] = {{256, 1}, {192, 1}, {384, 1}, {512, 1}, {256, 2}, {512, 2}};

// (Re)builds a path's device tables for a layout: workgroups of `threads`
// threads, floor(threads / Z) / gdiv lane groups per work item (at most 64),
// each holding one frame, or two on the packed-FP16 fixed-point path.
int build_tables(ldpc_codeset *cs, int path, int threads, int gdiv)
{
    const int n = cs->ncodes;
    const int per_group = (path == 1 && cs->h2) ? 2 : 1;
    std::vector<CodeRec> rec(n);
    std::vector<int> etab, G(n);
    size_t lds = 0;
    for (int c = 0; c < n; ++c) {
        const Sched &s = cs->sc[c];
        // a frame's Z rows need Z threads of the workgroup
        if (s.Z > threads)
            return fail(LDPC_ERANGE, "code %d: Z=%d exceeds a %d-thread workgroup", c, s.Z, threads);
        int groups = std::max(1, std::min(64, threads / s.Z) / gdiv);
        // fewer groups per item where the posteriors (one column block of
        // padding included) would not fit the LDS budget
        while (groups > 1 && (size_t)(s.N + s.Z) * fwp_for(groups) * 4 > (size_t)kLdsBudget)
            --groups;
        const int FWp = fwp_for(groups);
        if ((size_t)(s.N + s.Z) * FWp * 4 > (size_t)kLdsBudget)
            return fail(LDPC_ERANGE, "code %d (N=%d) does not fit the batched kernel's LDS budget", c, s.N);
        lds = std::max(lds, (size_t)(s.N + s.Z) * FWp);
        G[c] = groups * per_group;   // frames per work item
        rec[c] = CodeRec{s.Z, s.N, cs->cls[c], G[c], FWp, (int)(etab.size() / 2), 0, 0};
        for (int i = 0; i < cs->cmb; ++i)
            for (int e = 0; e < cs->cd; ++e) {
                int base = 0, thr = 1 << 30;
                if (i < s.Mb && e < s.deg[i]) {
                    const int col = (int)(s.edge[i][e] >> 16), sh = (int)(s.edge[i][e] & 0xffffu);
                    base = (col * s.Z + sh) * FWp * 4;
                    thr = s.Z - sh;
                }
                etab.push_back(base);
                etab.push_back(thr);
            }
    }
    void *dc = nullptr, *de = nullptr;
    if (hipMalloc(&dc, rec.size() * sizeof(CodeRec)) != hipSuccess ||
        hipMalloc(&de, etab.size() * sizeof(int)) != hipSuccess) {
        if (dc)
            (void)hipFree(dc);
        return fail(LDPC_ENOMEM, "code set: device allocation failed");
    }
    if (hipMemcpy(dc, rec.data(), rec.size() * sizeof(CodeRec), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(de, etab.data(), etab.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dc);
        (void)hipFree(de);
        return fail(LDPC_EDEVICE, "code set: copy to device failed");
    }
    if (cs->d_codes[path])
        (void)hipFree(cs->d_codes[path]);
    if (cs->d_etab[path])
        (void)hipFree(cs->d_etab[path]);
    cs->d_codes[path] = dc;
    cs->d_etab[path] = de;
    cs->lds_elems[path] = lds;
    cs->threads[path] = threads;
    cs->gdiv[path] = gdiv;
    cs->G[path] = G;
    return LDPC_OK;
}

int codeset_create(const int16_t *const *hbm, const int *Mb, const int *Nb, const int *Z, int n, ldpc_codeset **out)
{
    if (!hbm || !Mb || !Nb || !Z || !out || n < 1)
        return fail(LDPC_EINVAL, "null argument or empty code set");
    if (n > 1024)
        return fail(LDPC_ERANGE, "a code set holds at most 1024 codes");
    ldpc_codeset *cs = new ldpc_codeset();
    cs->ncodes = n;
    cs->sc.resize(n);
    for (int c = 0; c < n; ++c) {
        int rc = compile_sched(hbm[c], Mb[c], Nb[c], Z[c], true, &cs->sc[c]);
        if (rc) {
            delete cs;
            return rc;
        }
        int k = 0;
        for (; k < (int)cs->class_rep.size(); ++k)
            if (same_structure(cs->sc[cs->class_rep[k]], cs->sc[c]))
                break;
        if (k == (int)cs->class_rep.size())
            cs->class_rep.push_back(c);
        cs->cls.push_back(k);
        cs->cmb = std::max(cs->cmb, cs->sc[c].Mb);
        cs->cd = std::max(cs->cd, cs->sc[c].dmax);
        if (cs->sc[c].Z > kMaxThreads) {
            delete cs;
            return fail(LDPC_ERANGE, "code %d: Z=%d exceeds the batched kernel's workgroup", c, Z[c]);
        }
    }
    // two frames per lane in packed FP16 on the fixed-point path when every
    // code allows it (LDPC_BATCH_H2=0 in the environment at creation turns it off)
    {
        const char *hv = getenv("LDPC_BATCH_H2");
        cs->h2 = !(hv && hv[0] == '0');
        for (int c = 0; c < n && cs->h2; ++c)
            cs->h2 = h2_eligible(cs->sc[c]);
    }
    if (hipGetDevice(&cs->device) != hipSuccess) {
        delete cs;
        return fail(LDPC_EDEVICE, "hipGetDevice failed");
    }
    for (int path = 0; path < 2; ++path) {
        int rc = build_tables(cs, path, kMaxThreads, 1);
        if (rc) {
            ldpc_codeset_destroy(cs);
            return rc;
        }
    }
    *out = cs;
    return LDPC_OK;
}

// Work buffer (int64 words): head = items, queue, hist[ncodes],
// cursor[ncodes], ibase[ncodes] (padded to an even count); perm[F] (frame
// ids grouped by code); offp[F] (their offsets); then items[F + ncodes]
// (int4, 16-byte aligned).
static int64_t head_words(int ncodes)
{
    const int64_t h = 2 + 3 * (int64_t)ncodes;
    return h + (h & 1);
}

size_t batch_work_bytes(const ldpc_codeset *cs, int64_t F)
{
    return (size_t)(head_words(cs->ncodes) + 2 * F) * sizeof(int64_t) + (size_t)(F + cs->ncodes) * 4 * sizeof(int);
}

int launch_batch_decode(const ldpc_codeset *cs, int path, int mode, const int32_t *code_id, const int64_t *off,
                        const void *llr, int64_t n_llr, int64_t F, int max_iter, float alpha, int offset, int wq,
                        int et, uint8_t *bits, void *post, int32_t *iters, uint8_t *ok, void *work,
                        hipStream_t stream, bool loaded_only)
{
    const std::string pre = batch_prelude(*cs, path, mode);
    static const char *const names[6] = {"ldpc_batch_clear", "ldpc_batch_hist",    "ldpc_batch_plan",
                                         "ldpc_batch_items", "ldpc_batch_scatter", "ldpc_batch_decode"};
    hipFunction_t fn[6];
    int rc;
    for (int k = 0; k < 6; ++k) {
        rc = loaded_only ? jit_function_loaded("batch", pre, names[k], &fn[k])
                         : jit_function("batch", kJitBatchSource, pre, names[k], &fn[k]);
        if (rc)
            return rc;
    }
    hipFunction_t f_clear = fn[0], f_hist = fn[1], f_plan = fn[2], f_items = fn[3], f_scatter = fn[4],
                  f_dec = fn[5];
    const int64_t hw = head_words(cs->ncodes);
    int64_t *head = (int64_t *)work;
    int64_t *perm = head + hw;
    int64_t *offp = perm + F;
    int *items = (int *)(offp + F);
    int nc = cs->ncodes;
    int nwords = (int)hw;
    long long Fll = (long long)F;
    const void *codes = cs->d_codes[path], *etab = cs->d_etab[path];
    long long nll = (long long)n_llr;
    void *a_clear[] = {(void *)&head, (void *)&nwords};
    void *a_hist[] = {(void *)&code_id, (void *)&off, (void *)&codes, (void *)&nll, (void *)&Fll, (void *)&nc,
                      (void *)&head};
    void *a_plan[] = {(void *)&codes, (void *)&nc, (void *)&head};
    void *a_items[] = {(void *)&codes, (void *)&nc, (void *)&head, (void *)&items};
    void *a_scatter[] = {(void *)&code_id, (void *)&off,  (void *)&codes, (void *)&nll,   (void *)&Fll, (void *)&nc,
                         (void *)&head,    (void *)&perm, (void *)&offp,  (void *)&iters, (void *)&ok};
    // frames per workgroup of the histogram and the scatter (FPB in jit_batch.hip)
    const unsigned fblocks = (unsigned)((F + 4095) / 4096);
    if ((rc = jit_launch(f_clear, (unsigned)((nwords + 255) / 256), 256, stream, a_clear, "batch clear")) ||
        (rc = jit_launch(f_hist, fblocks, 256, stream, a_hist, "batch histogram")) ||
        (rc = jit_launch(f_plan, 1, 1024, stream, a_plan, "batch plan")) ||
        (rc = jit_launch(f_items, (unsigned)nc, 256, stream, a_items, "batch items")) ||
        (rc = jit_launch(f_scatter, fblocks, 256, stream, a_scatter, "batch scatter")))
        return rc;
    // persistent grid: as many workgroups as can be resident at once
    int per_cu = 0, cus = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f_dec, cs->threads[path], 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cs->device) != hipSuccess)
        return fail(LDPC_EDEVICE, "occupancy query failed");
    const unsigned grid = (unsigned)std::max(1, per_cu * cus);
    int64_t *nitems = head;
    unsigned long long *queue = (unsigned long long *)(head + 1);
    void *a_dec[] = {(void *)&items, (void *)&nitems, (void *)&queue, (void *)&perm, (void *)&offp, (void *)&codes,
                     (void *)&etab, (void *)&llr, (void *)&max_iter, (void *)&alpha, (void *)&offset, (void *)&wq,
                     (void *)&et, (void *)&bits, (void *)&post, (void *)&iters, (void *)&ok};
    return jit_launch(f_dec, grid, cs->threads[path], stream, a_dec, "batch decode");
}

// Times the batched decode of the caller's batch for each candidate layout
// and keeps the fastest (tables rebuilt for it).
int codeset_autotune(ldpc_codeset *cs, int path, const int32_t *code_id, const int64_t *off, const void *llr,
                     int64_t n_llr, int64_t F, int max_iter, uint8_t *bits, int32_t *iters, void *work,
                     hipStream_t stream, int32_t out[2], float *best_ms)
{
    const int(*cand)[2] = kBatchLayouts;
    constexpr int ncand = kNumBatchLayouts;
    int maxz = 0;
    for (int c = 0; c < cs->ncodes; ++c)
        maxz = std::max(maxz, cs->sc[c].Z);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return fail(LDPC_EDEVICE, "autotune: hipEventCreate failed");
    }
    int rc = LDPC_OK, best = -1;
    float best_t = 1e30f;
    const char *lv = getenv("LDPC_TUNE_LOG");
    const bool log = lv && lv[0] == '1';
    for (int k = 0; k < ncand && rc == LDPC_OK; ++k) {
        if (cand[k][0] < maxz)   // a frame's rows would not fit the workgroup
            continue;
        if ((rc = build_tables(cs, path, cand[k][0], cand[k][1])))
            break;
        auto run = [&]() {
            return launch_batch_decode(cs, path, 0, code_id, off, llr, n_llr, F, max_iter, 0.75f, 1, 0, 0, bits,
                                       nullptr, iters, nullptr, work, stream, false);
        };
        if ((rc = run()))   // compiles the variant and warms the caches
            break;
        hipEventRecord(e0, stream);
        for (int r = 0; r < 3 && rc == LDPC_OK; ++r)
            rc = run();
        hipEventRecord(e1, stream);
        if (rc)
            break;
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(LDPC_EDEVICE, "autotune: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        ms /= 3;
        if (log)
            fprintf(stderr, "ldpc batch autotune: path %d threads %d frames/item divisor %d  %.4f ms\n", path,
                    cand[k][0], cand[k][1], ms);
        if (ms < best_t) {
            best_t = ms;
            best = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best >= 0) {
        const int brc = build_tables(cs, path, cand[best][0], cand[best][1]);
        if (rc == LDPC_OK)
            rc = brc;
        out[0] = cand[best][0];
        out[1] = cand[best][1];
        *best_ms = best_t;
    }
    return rc;
}

}  // namespace ldpc

using namespace ldpc;

extern "C" {

int ldpc_codeset_create(const int16_t *const *hbm, const int *Mb, const int *Nb, const int *Z, int ncodes,
                        ldpc_codeset **out)
{
    clear_error();
    if (!jit_enabled())
        return fail(LDPC_ERANGE, "code sets need run-time specialisation (LDPC_JIT=0 is set)");
    return codeset_create(hbm, Mb, Nb, Z, ncodes, out);
}

void ldpc_codeset_destroy(ldpc_codeset *cs)
{
    if (!cs)
        return;
    for (int p = 0; p < 2; ++p) {
        if (cs->d_codes[p])
            (void)hipFree(cs->d_codes[p]);
        if (cs->d_etab[p])
            (void)hipFree(cs->d_etab[p]);
    }
    delete cs;
}

int ldpc_codeset_info(const ldpc_codeset *cs, int code, int64_t out[8])
{
    clear_error();
    if (!cs || !out || code < 0 || code >= cs->ncodes)
        return fail(LDPC_EINVAL, "bad code set, code index or output pointer");
    const Sched &s = cs->sc[code];
    out[0] = s.N;
    out[1] = s.K;
    out[2] = s.M;
    out[3] = s.E;
    out[4] = s.dmax;
    out[5] = cs->cls[code];
    out[6] = cs->G[0][code];
    out[7] = (int64_t)cs->class_rep.size();
    return LDPC_OK;
}

size_t ldpc_batch_work_bytes(const ldpc_codeset *cs, int64_t F)
{
    if (!cs || F < 0)
        return 0;
    return batch_work_bytes(cs, F);
}

static int batch_common(const ldpc_codeset *cs, const int32_t *code_id, const int64_t *off, const void *llr,
                        int64_t n_llr, int64_t F, int max_iter, const void *bits, const int32_t *iters, void *work,
                        size_t work_bytes)
{
    clear_error();
    if (!cs)
        return fail(LDPC_EINVAL, "null code set");
    if (F < 0 || max_iter < 1 || n_llr < 0)
        return fail(LDPC_EINVAL, "F and n_llr must be >= 0 and max_iter >= 1");
    if (F > ((int64_t)1 << 31) - 1)
        return fail(LDPC_ERANGE, "batch larger than 2^31 - 1 frames");
    if (F > 0 && (!code_id || !off || !llr || !bits || !iters || !work))
        return fail(LDPC_EINVAL, "null device pointer (code_id, off, llr, bits, iters and work are required)");
    if (F > 0 && work_bytes < batch_work_bytes(cs, F))
        return fail(LDPC_EINVAL, "work buffer too small: %zu < %zu bytes", work_bytes, batch_work_bytes(cs, F));
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != cs->device)
        return fail(LDPC_EINVAL, "the code set belongs to device %d", cs->device);
    return LDPC_OK;
}

int ldpc_decode_batch_f32(const ldpc_codeset *cs, const int32_t *code_id, const int64_t *off, const float *llr,
                          int64_t n_llr, int64_t F, int max_iter, float alpha, int early_term, uint8_t *bits,
                          float *post, int32_t *iters, uint8_t *ok, void *work, size_t work_bytes, void *stream)
{
    int rc = batch_common(cs, code_id, off, llr, n_llr, F, max_iter, bits, iters, work, work_bytes);
    if (rc || F == 0)
        return rc;
    return launch_batch_decode(cs, 0, 0, code_id, off, llr, n_llr, F, max_iter, alpha, 0, 0, early_term, bits, post,
                               iters, ok, work, (hipStream_t)stream, false);
}

int ldpc_decode_batch_f32_noalloc(const ldpc_codeset *cs, const int32_t *code_id, const int64_t *off,
                                  const float *llr, int64_t n_llr, int64_t F, int max_iter, float alpha,
                                  int early_term, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok,
                                  void *stream)
{
    clear_error();
    if (!cs)
        return fail(LDPC_EINVAL, "null code set");
    // the scratch is sized for kBatchScratchFrames frames of a 1024-code set
    if (F > kBatchScratchFrames || (F > 0 && batch_work_bytes(cs, F) > kBatchScratchBytes))
        return fail(LDPC_ERANGE, "%lld frames exceed the static scratch (at most %d frames)", (long long)F,
                    kBatchScratchFrames);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(LDPC_EDEVICE, "hipGetDevice failed");
    void *scratch = nullptr;
    int rc = batch_scratch(dev, &scratch);
    if (rc)
        return rc;
    rc = batch_common(cs, code_id, off, llr, n_llr, F, max_iter, bits, iters, scratch, kBatchScratchBytes);
    if (rc || F == 0)
        return rc;
    rc = launch_batch_decode(cs, 0, 0, code_id, off, llr, n_llr, F, max_iter, alpha, 0, 0, early_term, bits, post,
                             iters, ok, scratch, (hipStream_t)stream, true);
    if (rc == LDPC_ERANGE)
        return fail(LDPC_ERANGE, "the batch kernels of this code set are not loaded on device %d: make one "
                    "ldpc_decode_batch_f32 or ldpc_codeset_autotune call (FP32) with it first", dev);
    return rc;
}

int ldpc_decode_batch_i8(const ldpc_codeset *cs, const int32_t *code_id, const int64_t *off, const int8_t *llr,
                         int64_t n_llr, int64_t F, int max_iter, int offset, int wq, int early_term, uint8_t *bits,
                         int16_t *post, int32_t *iters, uint8_t *ok, void *work, size_t work_bytes, void *stream)
{
    int rc = batch_common(cs, code_id, off, llr, n_llr, F, max_iter, bits, iters, work, work_bytes);
    if (rc || F == 0)
        return rc;
    if (offset < 0 || offset > 127 || wq < 0 || wq > 31)
        return fail(LDPC_EINVAL, "offset must be in [0, 127] and wq in [0, 31]");
    return launch_batch_decode(cs, 1, wq > 0 ? 1 : 0, code_id, off, llr, n_llr, F, max_iter, 0.0f, offset, wq,
                               early_term, bits, post, iters, ok, work, (hipStream_t)stream, false);
}

int ldpc_codeset_set_layout(ldpc_codeset *cs, int path, int threads, int divisor)
{
    clear_error();
    if (!cs)
        return fail(LDPC_EINVAL, "null code set");
    if (path != 0 && path != 1)
        return fail(LDPC_EINVAL, "path must be 0 (FP32) or 1 (int8)");
    bool known = false;
    for (int k = 0; k < kNumBatchLayouts; ++k)
        known = known || (kBatchLayouts[k][0] == threads && kBatchLayouts[k][1] == divisor);
    if (!known)
        return fail(LDPC_EINVAL, "layout (%d threads, divisor %d) is not one of the batch autotuner's", threads,
                    divisor);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != cs->device)
        return fail(LDPC_EINVAL, "the code set belongs to device %d", cs->device);
    return build_tables(cs, path, threads, divisor);
}

int ldpc_codeset_autotune(ldpc_codeset *cs, int path, const int32_t *code_id, const int64_t *off, const void *llr,
                          int64_t n_llr, int64_t F, int max_iter, uint8_t *bits, int32_t *iters, void *work,
                          size_t work_bytes, int32_t out[2], float *ms, void *stream)
{
    clear_error();
    if (path != 0 && path != 1)
        return fail(LDPC_EINVAL, "path must be 0 (FP32) or 1 (int8)");
    int rc = batch_common(cs, code_id, off, llr, n_llr, F, max_iter, bits, iters, work, work_bytes);
    if (rc)
        return rc;
    if (F == 0 || !out || !ms)
        return fail(LDPC_EINVAL, "autotune needs a non-empty batch and output pointers");
    return codeset_autotune(cs, path, code_id, off, llr, n_llr, F, max_iter, bits, iters, work, (hipStream_t)stream,
                            out, ms);
}

}  // extern "C"
