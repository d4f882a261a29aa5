// Decode-layout autotuner. For one code and arithmetic path it times the
// run-time specialised kernel over candidate layouts -- frame groups per
// workgroup (G), frames per thread (KF) and whether gather addresses stay in
// registers across iterations -- and keeps the fastest for later calls on
// that code. The layouts trade registers and LDS per frame against waves
// per SIMD, which is hard to predict, so they are measured.
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

// Candidate layouts: for each frames-per-thread count, the workgroup shapes
// whose lanes are at least 85% busy, with and without address hoisting.
std::vector<DecodeLaunch> candidates(const Sched &sc, int elem_bytes)
{
    std::vector<DecodeLaunch> out;
    for (int KF = 1; KF <= 4; ++KF) {
        for (int G = 1; G * sc.Z <= kMaxJitThreads; ++G) {
            DecodeLaunch lc = make_launch(sc, elem_bytes, G, KF, kMaxJitThreads);
            if (lc.G < 1)
                continue;
            if ((double)(G * sc.Z) / lc.threads < 0.85)
                continue;
            for (int hoist = 0; hoist <= 1; ++hoist) {
                lc.hoist = hoist;
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

int autotune_decode(const Sched &sc, int path, int max_iter, int64_t F, hipStream_t stream, DecodeLaunch *best,
                    float *best_ms)
{
    const int eb = path == 0 ? 4 : 2;
    const size_t in_bytes = (size_t)F * sc.N * (path == 0 ? 4 : 1);
    void *llr = nullptr, *bits = nullptr, *iters = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = LDPC_OK;
    float best_t = 1e30f;
    DecodeLaunch best_lc{};
    if (hipMalloc(&llr, in_bytes) != hipSuccess || hipMalloc(&bits, (size_t)F * sc.N) != hipSuccess ||
        hipMalloc(&iters, (size_t)F * sizeof(int32_t)) != hipSuccess) {
        rc = fail(LDPC_ENOMEM, "autotune: device allocation failed");
        goto done;
    }
    if (hipMemsetAsync(llr, 0, in_bytes, stream) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = fail(LDPC_EDEVICE, "autotune: HIP setup failed");
        goto done;
    }
    for (const DecodeLaunch &lc : candidates(sc, eb)) {
        // the first launch compiles the variant and warms the caches
        rc = launch_jit_decode(sc, lc, path, 0, llr, nullptr, F, max_iter, 0.75f, 1, 0, 0, nullptr,
                               (uint8_t *)bits, nullptr, (int32_t *)iters, nullptr, stream);
        if (rc)
            goto done;
        const int reps = 3;
        hipEventRecord(e0, stream);
        for (int k = 0; k < reps && rc == LDPC_OK; ++k)
            rc = launch_jit_decode(sc, lc, path, 0, llr, nullptr, F, max_iter, 0.75f, 1, 0, 0, nullptr,
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
        if (ms < best_t) {
            best_t = ms;
            best_lc = lc;
        }
    }
    if (best_lc.G < 1) {
        rc = fail(LDPC_ERANGE, "autotune: no decode layout fits this code");
        goto done;
    }
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
    return rc;
}

}  // namespace ldpc
