// Decode-layout autotuner. For one code and arithmetic path it times the
// run-time specialised kernel over candidate layouts -- frame groups per
// workgroup (G), frames per thread (KF), whether gather addresses stay in
// registers across iterations, two frames per lane in packed FP16 (fixed
// point), and an occupancy target for the register allocator -- and keeps
// the fastest for later calls on that code. The layouts trade registers and
// LDS per frame against waves per SIMD, which is hard to predict, so they
// are measured.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "ldpc_internal.h"

namespace ldpc {

namespace {

std::mutex g_tmu;
std::unordered_map<std::string, DecodeLaunch> g_tuned;

std::string tune_key(const Sched &sc, int path)
{
    std::string k = std::to_string(path) + ":" + std::to_string(sc.Z) + ":" + std::to_string(sc.Mb) + ":" +
                    std::to_string(sc.Nb) + ":";
    for (int i = 0; i < sc.Mb; ++i)
        for (int e = 0; e < sc.deg[i]; ++e)
            k += std::to_string(sc.edge[i][e]) + ",";
    return k;
}

// A workgroup of one wave (codes with Z <= 64): no barrier waits on other
// waves, and a small batch spreads over more workgroups, so such layouts are
// candidates however many of their lanes idle.
bool single_wave(const Sched &sc, int G) { return G * sc.Z <= 64; }

// Candidate layouts: workgroups of at most 256 threads whose lanes are at
// least 85% busy (or of a single wave), one or two frames per thread, and the number of block rows
// whose gather addresses stay in registers (all, three quarters, half, a
// quarter, none).
// A thread keeps KF messages per edge of its rows in VGPRs, plus an address
// per hoisted edge; the registers decide how many waves share a SIMD, which
// is hard to predict, so the candidates are compiled and timed, and those
// that spill are dropped.
std::vector<DecodeLaunch> candidates(const Sched &sc, int elem_bytes, int path)
{
    std::vector<DecodeLaunch> out;
    const int per_row = sc.E / sc.Z;
    const int hoists[5] = {sc.Mb, (3 * sc.Mb + 3) / 4, sc.Mb / 2, sc.Mb / 4, 0};
    // fixed point (with or without a weight table): two frames per lane in
    // packed FP16 where the values fit
    if ((path & 1) == 1 && h2_eligible(sc)) {
        for (int G = 1; G * sc.Z <= kMaxThreads; ++G) {
            DecodeLaunch lc = make_h2_launch(sc, G, kMaxThreads);
            if (lc.G < 1 || (!single_wave(sc, G) && (double)(G * sc.Z) / lc.threads < 0.85))
                continue;
            int last = -1;
            for (int h : hoists) {
                if (h == last)
                    continue;
                last = h;
                lc.hoist = h;
                out.push_back(lc);
            }
        }
    }
    for (int KF = 1; KF <= 2 && KF * per_row <= 200; ++KF) {
        for (int G = 1; G * sc.Z <= kMaxThreads; ++G) {
            DecodeLaunch lc = make_launch(sc, elem_bytes, G, KF, kMaxThreads);
            if (lc.G < 1)
                continue;
            if (!single_wave(sc, G) && (double)(G * sc.Z) / lc.threads < 0.85)
                continue;
            int last = -1;
            for (int h : hoists) {
                if (h == last || (KF > 1 && h > 0))
                    continue;
                last = h;
                lc.hoist = h;
                out.push_back(lc);
            }
        }
    }
    return out;
}

}  // namespace

bool tuned_launch(const Sched &sc, int path, DecodeLaunch *out)
{
    std::lock_guard<std::mutex> lock(g_tmu);
    auto it = g_tuned.find(tune_key(sc, path));
    if (it == g_tuned.end())
        return false;
    *out = it->second;
    return true;
}

void set_tuned_launch(const Sched &sc, int path, const DecodeLaunch &lc)
{
    std::lock_guard<std::mutex> lock(g_tmu);
    g_tuned[tune_key(sc, path)] = lc;
}

void tune_cache_clear()
{
    std::lock_guard<std::mutex> lock(g_tmu);
    g_tuned.clear();
}

int tuner_layouts(const Sched &sc, int path, std::vector<DecodeLaunch> *out, std::vector<size_t> *scratch_out)
{
    // candidates, then for each one whose kernel holds more than 128 VGPRs
    // per lane the same layout compiled for one more wave per SIMD (a hint
    // to the register allocator). Spilled registers live in scratch memory
    // and add HBM traffic: an unhinted layout that spills is dropped, a
    // hinted one may spill at most 32 bytes per lane.
    const char *lv = getenv("LDPC_TUNE_LOG");
    const bool log = lv && lv[0] == '1';
    // tuning path: 0 FP32, 1 int8, 2 FP32 with a weight table, 3 int8 with a table
    const int kpath = path & 1, mode = tune_mode(path);
    std::vector<DecodeLaunch> work = candidates(sc, 4, path);   // FP32 posteriors in LDS on both paths
    out->clear();
    if (scratch_out)
        scratch_out->clear();
    for (size_t w = 0; w < work.size(); ++w) {
        const DecodeLaunch lc = work[w];
        size_t scratch = 0;
        int vgprs = 0;
        int rc = jit_decode_scratch(sc, lc, kpath, mode, &scratch, &vgprs);
        if (rc)
            return rc;
        const size_t allowed = lc.waves ? 32 : 0;
        if (scratch > allowed) {
            if (log)
                fprintf(stderr, "ldpc autotune: G %d KF %d hoist %d waves %d spills %zu bytes, skipped\n", lc.G,
                        lc.KF, lc.hoist, lc.waves, scratch);
            continue;
        }
        if (lc.waves == 0 && vgprs > 128) {
            DecodeLaunch v = lc;
            v.waves = vgprs > 168 ? 3 : 4;
            work.push_back(v);
        }
        out->push_back(lc);
        if (scratch_out)
            scratch_out->push_back(scratch);
    }
    return LDPC_OK;
}

int autotune_decode(const Sched &sc, int path, int max_iter, int64_t F, hipStream_t stream, DecodeLaunch *best,
                    float *best_ms)
{
    const int kpath = path & 1, mode = tune_mode(path);
    const size_t in_bytes = (size_t)F * sc.N * (kpath == 0 ? 4 : 1);
    // a zero weight table: the decode does the same work for any weights
    const size_t w_bytes = mode_has_table(path) ? (size_t)max_iter * sc.Mb * sc.Nb * (kpath == 0 ? 4 : 1) : 0;
    void *llr = nullptr, *bits = nullptr, *iters = nullptr, *wt = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = LDPC_OK;
    float best_t = 1e30f, spill_t = 1e30f;
    DecodeLaunch best_lc{}, spill_lc{};
    std::vector<DecodeLaunch> work;
    std::vector<size_t> spills;
    const char *lv = getenv("LDPC_TUNE_LOG");   // set to 1: print every candidate's time
    const bool log = lv && lv[0] == '1';
    if ((rc = tuner_layouts(sc, path, &work, &spills)))
        return rc;
    if (hipMalloc(&llr, in_bytes) != hipSuccess || hipMalloc(&bits, (size_t)F * sc.N) != hipSuccess ||
        hipMalloc(&iters, (size_t)F * sizeof(int32_t)) != hipSuccess ||
        (w_bytes && hipMalloc(&wt, w_bytes) != hipSuccess)) {
        rc = fail(LDPC_ENOMEM, "autotune: device allocation failed");
        goto done;
    }
    if (hipMemsetAsync(llr, 0, in_bytes, stream) != hipSuccess ||
        (w_bytes && hipMemsetAsync(wt, 0, w_bytes, stream) != hipSuccess) || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = fail(LDPC_EDEVICE, "autotune: HIP setup failed");
        goto done;
    }
    // a layout that spills replaces the fastest spill-free one only if it is
    // at least 5% faster
    for (size_t w = 0; w < work.size(); ++w) {
        const DecodeLaunch lc = work[w];
        const size_t scratch = spills[w];
        // the first launch warms the caches
        rc = launch_jit_decode(sc, lc, kpath, mode, llr, nullptr, F, max_iter, 0.75f, 1, 0, 0, wt, (uint8_t *)bits,
                               nullptr, (int32_t *)iters, nullptr, stream);
        if (rc)
            goto done;
        const int reps = 3;
        hipEventRecord(e0, stream);
        for (int k = 0; k < reps && rc == LDPC_OK; ++k)
            rc = launch_jit_decode(sc, lc, kpath, mode, llr, nullptr, F, max_iter, 0.75f, 1, 0, 0, wt,
                                   (uint8_t *)bits, nullptr, (int32_t *)iters, nullptr, stream);
        hipEventRecord(e1, stream);
        if (rc)
            goto done;
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(LDPC_EDEVICE, "autotune: %s", hipGetErrorString(hipGetLastError()));
            goto done;
        }
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (log)
            fprintf(stderr,
                    "ldpc autotune: path %d Z %d Mb %d  G %d KF %d threads %d hoisted rows %d h2 %d waves %d "
                    "scratch %zu  %.4f ms\n",
                    path, sc.Z, sc.Mb, lc.G, lc.KF, lc.threads, lc.hoist, lc.h2, lc.waves, scratch, ms);
        if (scratch == 0 && ms < best_t) {
            best_t = ms;
            best_lc = lc;
        } else if (scratch > 0 && ms < spill_t) {
            spill_t = ms;
            spill_lc = lc;
        }
    }
    if (spill_lc.G >= 1 && (best_lc.G < 1 || spill_t < 0.95f * best_t)) {
        best_t = spill_t;
        best_lc = spill_lc;
    }
    if (best_lc.G < 1) {
        rc = fail(LDPC_ERANGE, "autotune: no decode layout fits this code");
        goto done;
    }
    best_lc.tuned = 1;
    set_tuned_launch(sc, path, best_lc);
    *best = best_lc;
    *best_ms = best_t;
done:
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (llr)
        (void)hipFree(llr);
    if (bits)
        (void)hipFree(bits);
    if (iters)
        (void)hipFree(iters);
    if (wt)
        (void)hipFree(wt);
    return rc;
}

void clear_tuned_launch(const Sched &sc, int path)
{
    std::lock_guard<std::mutex> lock(g_tmu);
    g_tuned.erase(tune_key(sc, path));
}

}  // namespace ldpc
