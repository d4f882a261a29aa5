// Run-time specialisation of the decode kernel (hipRTC).
//
// The base matrix is turned into a prelude of compile-time constants
// (degrees, block columns, shifts, launch layout) that is prepended to the
// kernel source in jit_decode.hip, compiled for the current device's
// architecture and cached per (device, code, layout, arithmetic path). Each
// layer of the specialised kernel is straight-line code.
#include <hip/hiprtc.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>

#include "ldpc_internal.h"

namespace ldpc {

// Kernel sources, embedded at build time from jit_decode.hip and jit_nms.hip.
extern const char kJitDecodeSource[];
extern const char kJitNmsSource[];
extern const char kJitBatchSource[];
extern const char kJitFloodSource[];
extern const char kJitQ16Source[];
extern const char kJitH2Source[];

namespace {

struct JitKernel {
    hipModule_t mod = nullptr;
};

std::mutex g_mu;
std::unordered_map<std::string, JitKernel> g_cache;

std::string prelude(const Sched &sc, const DecodeLaunch &lc, int path, int mode)
{
    std::ostringstream o;
    o << "#define LDPC_Z " << sc.Z << "\n#define LDPC_MB " << sc.Mb << "\n#define LDPC_NB " << sc.Nb
      << "\n#define LDPC_N " << sc.N << "\n#define LDPC_MAXD " << sc.dmax << "\n#define LDPC_G " << lc.G
      << "\n#define LDPC_KF " << lc.KF << "\n#define LDPC_FWP " << lc.FWp << "\n#define LDPC_THREADS " << lc.threads
      << "\n#define LDPC_PATH " << path << "\n#define LDPC_MODE " << mode << "\n#define LDPC_HOIST " << lc.hoist
      << "\n#define LDPC_WAVES_HINT " << lc.waves << "\n";
    o << "__device__ constexpr int kDeg[" << sc.Mb << "] = {";
    for (int i = 0; i < sc.Mb; ++i)
        o << sc.deg[i] << (i + 1 < sc.Mb ? "," : "};\n");
    for (int pass = 0; pass < 2; ++pass) {
        o << "__device__ constexpr int " << (pass ? "kShift" : "kCol") << "[" << sc.Mb << "][" << sc.dmax << "] = {";
        for (int i = 0; i < sc.Mb; ++i) {
            o << "{";
            for (int e = 0; e < sc.dmax; ++e) {
                const int v = e < sc.deg[i] ? (pass ? (int)(sc.edge[i][e] & 0xffffu) : (int)(sc.edge[i][e] >> 16)) : 0;
                o << v << (e + 1 < sc.dmax ? "," : "");
            }
            o << "}" << (i + 1 < sc.Mb ? "," : "};\n");
        }
    }
    return o.str();
}

// Compiles specialised source for an architecture; needs no device.
int rtc_compile(const std::string &src, const std::string &arch, std::string *code)
{
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "ldpc_jit_decode.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return fail(LDPC_EDEVICE, "hiprtcCreateProgram failed");
    const std::string archopt = "--offload-arch=" + arch;
    const char *opts[] = {archopt.c_str(), "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n)
            hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(LDPC_EDEVICE, "hipRTC compile failed: %.400s", log.c_str());
    }
    size_t size = 0;
    hiprtcGetCodeSize(prog, &size);
    code->assign(size, '\0');
    hiprtcGetCode(prog, &(*code)[0]);
    hiprtcDestroyProgram(&prog);
    return LDPC_OK;
}

// Optional on-disk cache of compiled code objects, so that later processes
// skip hipRTC: directory from LDPC_JIT_CACHE (unset: no disk cache). The
// key hashes the architecture, the compiler version and the full source
// (prelude included), so a changed source never reuses an old object.
uint64_t fnv1a(const std::string &a, uint64_t h = 1469598103934665603ull)
{
    for (unsigned char c : a) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_path(const std::string &src, const std::string &arch)
{
    const char *dir = getenv("LDPC_JIT_CACHE");
    if (!dir || !dir[0])
        return std::string();
    int major = 0, minor = 0;
    hiprtcVersion(&major, &minor);
    const uint64_t h = fnv1a(src, fnv1a(arch + "|" + std::to_string(major) + "." + std::to_string(minor) + "|"));
    char name[64];
    snprintf(name, sizeof(name), "/ldpc_%016llx.co", (unsigned long long)h);
    return std::string(dir) + name;
}

bool cache_read(const std::string &path, std::string *code)
{
    FILE *f = path.empty() ? nullptr : fopen(path.c_str(), "rb");
    if (!f)
        return false;
    std::string buf;
    char tmp[65536];
    size_t n;
    while ((n = fread(tmp, 1, sizeof(tmp), f)) > 0)
        buf.append(tmp, n);
    fclose(f);
    if (buf.size() < 64)
        return false;
    *code = buf;
    return true;
}

void cache_write(const std::string &path, const std::string &code)
{
    if (path.empty())
        return;
    mkdir(getenv("LDPC_JIT_CACHE"), 0755);   // may exist already
    const std::string tmp = path + "." + std::to_string((long)getpid()) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f)
        return;
    const bool ok = fwrite(code.data(), 1, code.size(), f) == code.size();
    fclose(f);
    if (!ok || rename(tmp.c_str(), path.c_str()) != 0)
        remove(tmp.c_str());
}

int load(const std::string &code, JitKernel *out)
{
    hipModule_t mod;
    if (hipModuleLoadData(&mod, code.data()) != hipSuccess)
        return fail(LDPC_EDEVICE, "hipModuleLoadData failed: %s", hipGetErrorString(hipGetLastError()));
    out->mod = mod;
    return LDPC_OK;
}

// Module for (device, source, prelude), compiled on first use.
int get_module(const char *tag, const char *src, const std::string &pre, hipModule_t *mod)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(LDPC_EDEVICE, "hipGetDevice failed");
    const std::string key = std::to_string(dev) + "\n" + tag + "\n" + pre;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        *mod = it->second.mod;
        return LDPC_OK;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(LDPC_EDEVICE, "hipGetDeviceProperties failed");
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos)
        arch = arch.substr(0, colon);
    std::string code;
    const std::string full = pre + src;
    const std::string cpath = cache_path(full, arch);
    int rc;
    JitKernel k;
    const bool cached = cache_read(cpath, &code);
    // a cached object that does not load (a damaged file) is compiled again
    if (!cached || load(code, &k) != LDPC_OK) {
        clear_error();
        if ((rc = rtc_compile(full, arch, &code)))
            return rc;
        cache_write(cpath, code);
        if ((rc = load(code, &k)))
            return rc;
    }
    g_cache.emplace(key, k);
    *mod = k.mod;
    return LDPC_OK;
}

int get_function(const char *tag, const char *src, const std::string &pre, const char *name, hipFunction_t *fn)
{
    hipModule_t mod;
    int rc = get_module(tag, src, pre, &mod);
    if (rc)
        return rc;
    if (hipModuleGetFunction(fn, mod, name) != hipSuccess)
        return fail(LDPC_EDEVICE, "hipModuleGetFunction(%s) failed", name);
    return LDPC_OK;
}

int launch(hipFunction_t fn, unsigned blocks, unsigned threads, hipStream_t stream, void **args, const char *what)
{
    if (hipModuleLaunchKernel(fn, blocks, 1, 1, threads, 1, 1, 0, stream, args, nullptr) != hipSuccess)
        return fail(LDPC_EDEVICE, "%s launch failed: %s", what, hipGetErrorString(hipGetLastError()));
    return LDPC_OK;
}

}  // namespace

int jit_function(const char *tag, const char *src, const std::string &pre, const char *name, hipFunction_t *fn)
{
    return get_function(tag, src, pre, name, fn);
}

int jit_function_loaded(const char *tag, const std::string &pre, const char *name, hipFunction_t *fn)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(LDPC_EDEVICE, "hipGetDevice failed");
    const std::string key = std::to_string(dev) + "\n" + tag + "\n" + pre;
    hipModule_t mod;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        auto it = g_cache.find(key);
        if (it == g_cache.end())
            return fail(LDPC_ERANGE, "kernel %s is not loaded on device %d yet", name, dev);
        mod = it->second.mod;
    }
    if (hipModuleGetFunction(fn, mod, name) != hipSuccess)
        return fail(LDPC_EDEVICE, "hipModuleGetFunction(%s) failed", name);
    return LDPC_OK;
}

int jit_launch(hipFunction_t fn, unsigned blocks, unsigned threads, hipStream_t stream, void **args, const char *what)
{
    return launch(fn, blocks, threads, stream, args, what);
}

bool jit_enabled()
{
    const char *v = getenv("LDPC_JIT");
    return !(v && v[0] == '0');
}

void jit_cache_clear()
{
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &kv : g_cache)
        hipModuleUnload(kv.second.mod);
    g_cache.clear();
}

// Decode kernel of one code: named after its path and shape so that
// profiles tell the specialised kernels apart.
static std::string decode_kernel_name(const Sched &sc, int path, bool packed, bool h2)
{
    return std::string("ldpc_decode_") + (path == 0 ? "f32" : (h2 ? "i8h2" : "i8")) + "_z" + std::to_string(sc.Z) +
           "_mb" + std::to_string(sc.Mb) + "_nb" + std::to_string(sc.Nb) + (packed ? "_pk" : "");
}

static int get_decode_function(const Sched &sc, const DecodeLaunch &lc, int path, int mode, hipFunction_t *fn,
                               bool packed = false)
{
    const bool h2 = lc.h2 != 0;
    const std::string name = decode_kernel_name(sc, path, packed, h2);
    return get_function(h2 ? "decode_h2" : "decode", h2 ? kJitH2Source : kJitDecodeSource,
                        prelude(sc, lc, path, mode) + "#define LDPC_KERNEL " + name + "\n" +
                            (packed ? "#define LDPC_PACKED 1\n" : ""),
                        name.c_str(), fn);
}

DecodeLaunch flood_launch(const Sched &sc)
{
    // the flooding kernel keeps two FP32 arrays (posteriors, channel values)
    // in LDS; the widest workgroup of <= 256 threads with the most busy lanes
    DecodeLaunch best{};
    double best_util = -1.0;
    for (int G = 1; G * sc.Z <= kMaxThreads && G <= 64; ++G) {
        const int FWp = G | 1;
        const size_t lds = 2 * (size_t)(sc.N + sc.Z) * FWp * sizeof(float);
        if (lds > (size_t)kLdsBudget)
            break;
        const int threads = ((G * sc.Z + 63) / 64) * 64;
        const double util = (double)(G * sc.Z) / threads;
        if (util > best_util + 1e-9 || (util > best_util - 1e-9 && G > best.G)) {
            best_util = util;
            best = DecodeLaunch{G, 1, G, FWp, threads, lds, 0};
        }
    }
    const int per_row = sc.E / sc.Z;
    best.hoist = 2 * per_row <= 176 ? sc.Mb : 0;
    return best;
}

int launch_jit_flood(const Sched &sc, const DecodeLaunch &lc, int path, int mode, const void *llr, int64_t F,
                     int max_iter, float alpha, int offset, int wq, int et, uint8_t *bits, void *post, int32_t *iters,
                     uint8_t *ok, hipStream_t stream)
{
    const std::string name = std::string("ldpc_flood_") + (path == 0 ? "f32" : "i8") + "_z" + std::to_string(sc.Z) +
                             "_mb" + std::to_string(sc.Mb) + "_nb" + std::to_string(sc.Nb);
    hipFunction_t fn;
    int rc = get_function("flood", kJitFloodSource, prelude(sc, lc, path, mode) + "#define LDPC_KERNEL " + name + "\n",
                          name.c_str(), &fn);
    if (rc)
        return rc;
    long long Fll = (long long)F;
    void *args[] = {(void *)&llr, (void *)&Fll, (void *)&max_iter, (void *)&alpha, (void *)&offset, (void *)&wq,
                    (void *)&et, (void *)&bits, (void *)&post, (void *)&iters, (void *)&ok};
    return launch(fn, (unsigned)((F + lc.FW - 1) / lc.FW), lc.threads, stream, args, "flood decode");
}

int launch_jit_q16(const Sched &sc, const DecodeLaunch &lc, int wrap, const int16_t *llr, int64_t F, int max_iter,
                   int wq, int et, uint8_t *bits, int16_t *post, int32_t *iters, uint8_t *ok, hipStream_t stream)
{
    const std::string name = std::string("ldpc_q16_") + (wrap ? "wrap" : "sat") + "_z" + std::to_string(sc.Z) +
                             "_mb" + std::to_string(sc.Mb) + "_nb" + std::to_string(sc.Nb);
    hipFunction_t fn;
    int rc = get_function("q16", kJitQ16Source,
                          prelude(sc, lc, 1, 0) + "#define LDPC_WRAP " + std::to_string(wrap ? 1 : 0) +
                              "\n#define LDPC_KERNEL " + name + "\n",
                          name.c_str(), &fn);
    if (rc)
        return rc;
    long long Fll = (long long)F;
    void *args[] = {(void *)&llr, (void *)&Fll, (void *)&max_iter, (void *)&wq, (void *)&et, (void *)&bits,
                    (void *)&post, (void *)&iters, (void *)&ok};
    return launch(fn, (unsigned)((F + lc.FW - 1) / lc.FW), lc.threads, stream, args, "q16 decode");
}

// One frame per thread, FP32 posteriors in LDS (both paths).
static DecodeLaunch single_frame_launch(const Sched &sc)
{
    DecodeLaunch lc = plan_decode(sc, 4, 1);
    lc.hoist = 2 * (sc.E / sc.Z) <= 176 ? sc.Mb : 0;
    return lc;
}

int max_col_weight(const Sched &sc)
{
    int w[64] = {0}, best = 0;
    for (int i = 0; i < sc.Mb; ++i)
        for (int e = 0; e < sc.deg[i]; ++e) {
            const int j = (int)(sc.edge[i][e] >> 16);
            if (j < 64)
                best = std::max(best, ++w[j]);
        }
    return best;
}

DecodeLaunch make_h2_launch(const Sched &sc, int G, int max_threads)
{
    DecodeLaunch lc{};
    if (G < 1 || 2 * G > 64 || G * sc.Z > max_threads)
        return lc;
    const int FWp = G | 1;
    const size_t lds = (size_t)(sc.N + sc.Z) * FWp * 4;
    if (lds > (size_t)kLdsBudget)
        return lc;
    lc = DecodeLaunch{G, 1, 2 * G, FWp, ((G * sc.Z + 63) / 64) * 64, lds, 0};
    lc.h2 = 1;
    return lc;
}

static DecodeLaunch three_wave_layout(const Sched &sc, const DecodeLaunch &lc, int path, int mode);

DecodeLaunch usable_launch(const Sched &sc, const DecodeLaunch &lc, int path, int mode)
{
    DecodeLaunch out = lc;
    if (lc.h2 && (path != 1 || !h2_eligible(sc)))
        out = single_frame_launch(sc);
    // a layout the tuner did not time for this kernel: the default layout,
    // or a weighted mode (its kernel needs more registers than the plain one)
    const bool weighted = (path == 0 && mode == 1) || (path == 1 && mode == 2);
    if (weighted || !out.tuned)
        out = three_wave_layout(sc, out, path, mode);
    return out;
}

DecodeLaunch decode_layout(const Sched &sc, int path, int mode)
{
    DecodeLaunch lc = jit_default_launch(sc, path);
    const bool table = (path == 0 && mode == 1) || (path == 1 && mode == 2);
    if (table && tuned_launch(sc, path + 2, &lc))
        return lc;   // timed for the kernel with a weight table
    tuned_launch(sc, path, &lc);
    return usable_launch(sc, lc, path, mode);
}

DecodeLaunch jit_default_launch(const Sched &sc, int path)
{
    const int per_row = sc.E / sc.Z;          // messages (and gather addresses) per thread
    if (path == 1 && h2_eligible(sc)) {
        // fixed point: two frames per lane; the widest workgroup with the most busy lanes
        DecodeLaunch best{};
        double best_util = -1.0;
        for (int G = 1; G * sc.Z <= kMaxThreads; ++G) {
            const DecodeLaunch lc = make_h2_launch(sc, G, kMaxThreads);
            if (lc.G < 1)
                break;
            const double util = (double)(G * sc.Z) / lc.threads;
            if (util > best_util + 1e-9 || (util > best_util - 1e-9 && lc.FW > best.FW)) {
                best_util = util;
                best = lc;
            }
        }
        if (best.G >= 1) {
            best.hoist = 2 * per_row <= 176 ? sc.Mb : 0;
            return best;
        }
    }
    return single_frame_launch(sc);
}

int jit_decode_scratch(const Sched &sc, const DecodeLaunch &lc, int path, int mode, size_t *bytes, int *vgprs)
{
    hipFunction_t fn;
    int rc = get_decode_function(sc, lc, path, mode, &fn);
    if (rc)
        return rc;
    int v = 0;
    if (hipFuncGetAttribute(&v, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, fn) != hipSuccess)
        return fail(LDPC_EDEVICE, "hipFuncGetAttribute failed");
    *bytes = (size_t)v;
    if (vgprs) {
        if (hipFuncGetAttribute(&v, HIP_FUNC_ATTRIBUTE_NUM_REGS, fn) != hipSuccess)
            return fail(LDPC_EDEVICE, "hipFuncGetAttribute failed");
        *vgprs = v;
    }
    return LDPC_OK;
}

// Layouts the tuner has not timed for the kernel at hand -- the default
// layout, and any layout in a weighted mode, where the row's weights (read
// from LDS next to the messages) cost registers -- can need more than 168
// VGPRs and so lose a wave per SIMD, which this latency-bound loop pays for
// (measured: FP32 weight table of the WiMAX-shaped rate-1/2 code at Z=96,
// 20.8 against 33.0 Gbit/s). Above 168 the layout keeps its frames and
// takes the deepest address hoist of Mb/2, Mb/4 and 0 whose kernel, compiled
// for three waves per SIMD, does not spill; none at all hoisted is the last
// resort. Chosen once per code, layout and mode.
static DecodeLaunch three_wave_layout(const Sched &sc, const DecodeLaunch &lc, int path, int mode)
{
    static std::mutex mu;
    static std::unordered_map<std::string, DecodeLaunch> memo;
    const std::string key = prelude(sc, lc, path, mode);
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = memo.find(key);
        if (it != memo.end())
            return it->second;
    }
    DecodeLaunch best = lc;
    size_t bytes = 0;
    int vgprs = 0;
    if (lc.waves == 0 && jit_decode_scratch(sc, lc, path, mode, &bytes, &vgprs) == LDPC_OK && vgprs > 168) {
        const int cands[3] = {sc.Mb / 2, sc.Mb / 4, 0};
        for (int k = 0; k < 3; ++k) {
            if (cands[k] >= lc.hoist || (k > 0 && cands[k] == cands[k - 1]))
                continue;
            DecodeLaunch c = lc;
            c.hoist = cands[k];
            c.waves = 3;
            if (jit_decode_scratch(sc, c, path, mode, &bytes, &vgprs) != LDPC_OK)
                break;
            if (bytes == 0 || cands[k] == 0) {
                if (bytes != 0)
                    c.waves = 0;   // unhinted: no spill, fewer waves
                best = c;
                break;
            }
        }
    }
    std::lock_guard<std::mutex> lock(mu);
    memo[key] = best;
    return best;
}

int launch_jit_decode(const Sched &sc, const DecodeLaunch &lc, int path, int mode, const void *llr,
                      const int64_t *fidx, int64_t F, int max_iter, float alpha, int offset, int wq, int et,
                      const void *wt, uint8_t *bits, void *post, int32_t *iters, uint8_t *ok, hipStream_t stream,
                      const int64_t *Fdev, bool packed)
{
    if (lc.h2 && path != 1)
        return fail(LDPC_EINVAL, "internal: a two-frames-per-lane layout was chosen for path %d", path);
    hipFunction_t fn;
    int rc = get_decode_function(sc, lc, path, mode, &fn, packed);
    if (rc)
        return rc;
    long long Fll = (long long)F;
    void *args[] = {(void *)&llr, (void *)&fidx, (void *)&Fll, (void *)&max_iter, (void *)&alpha, (void *)&offset,
                    (void *)&wq, (void *)&et, (void *)&wt, (void *)&bits, (void *)&post, (void *)&iters, (void *)&ok,
                    (void *)&Fdev};
    return launch(fn, (unsigned)((F + lc.FW - 1) / lc.FW), lc.threads, stream, args, "decode");
}

// ---------------------------------------------------------------------------
// Learned normalised min-sum (jit_nms.hip)
// ---------------------------------------------------------------------------

DecodeLaunch plan_nms(const Sched &sc)
{
    // one frame per thread group; the adjoint keeps L and gL (FP32) for the
    // workgroup's frames in LDS, frame-minor with an odd row stride, and one
    // slot of weight-gradient sums per 16-lane row (gfx950 gives a workgroup
    // up to 160 KiB of LDS; 96 KiB keeps two adjoint workgroups per CU)
    DecodeLaunch best{};
    double best_util = -1.0;
    for (int G = 1; G * sc.Z <= kMaxThreads && G <= 64; ++G) {
        const int FWp = G | 1;
        const size_t frames_lds = 2 * (size_t)sc.N * FWp * sizeof(float);
        if (frames_lds > (size_t)kLdsBudget)
            break;
        const int threads = ((G * sc.Z + 63) / 64) * 64;
        const size_t lds = frames_lds + (size_t)(threads / 16) * sc.Mb * sc.Nb * sizeof(float);
        if (lds > 96 * 1024)
            break;
        const double util = (double)(G * sc.Z) / threads;
        if (util > best_util + 1e-9) {
            best_util = util;
            best = DecodeLaunch{G, 1, G, FWp, threads, lds, 1};
        }
    }
    return best;
}

// Checkpoint buffer: per iteration and frame L and the compressed row state,
// then the per-frame loss terms, then the adjoint's per-workgroup partial
// weight gradients.
static size_t nms_partial_offset(const Sched &sc, int64_t F, int T)
{
    return (size_t)T * (size_t)F * ((size_t)sc.N + 3 * (size_t)sc.M) + (size_t)T * (size_t)F;
}

size_t nms_ckpt_floats(const Sched &sc, int64_t F, int T)
{
    const DecodeLaunch lc = plan_nms(sc);
    const size_t nwg = lc.G < 1 ? 0 : (size_t)((F + lc.G - 1) / lc.G);
    return nms_partial_offset(sc, F, T) + nwg * (size_t)T * (size_t)sc.Mb * (size_t)sc.Nb;
}

int launch_nms_fwd(const Sched &sc, const float *llr, const uint8_t *cw, int64_t F, int T, const float *w,
                   float *ckpt, float *loss, float *post, hipStream_t stream)
{
    const DecodeLaunch lc = plan_nms(sc);
    if (lc.G < 1)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the training kernels' LDS budget", sc.N);
    const std::string pre = prelude(sc, lc, 0, 1);
    hipFunction_t fwd, red;
    int rc = get_function("nms", kJitNmsSource, pre, "ldpc_nms_fwd", &fwd);
    if (rc || (rc = get_function("nms", kJitNmsSource, pre, "ldpc_nms_loss_reduce", &red)))
        return rc;
    float *loss_tf = ckpt + (size_t)T * (size_t)F * ((size_t)sc.N + 3 * (size_t)sc.M);
    long long Fll = (long long)F;
    void *a1[] = {(void *)&llr, (void *)&cw, (void *)&Fll, (void *)&T, (void *)&w, (void *)&ckpt, (void *)&loss_tf,
                  (void *)&post};
    if ((rc = launch(fwd, (unsigned)((F + lc.G - 1) / lc.G), lc.threads, stream, a1, "nms forward")))
        return rc;
    void *a2[] = {(void *)&loss_tf, (void *)&Fll, (void *)&T, (void *)&loss};
    return launch(red, (unsigned)T, 256, stream, a2, "nms loss");
}

int launch_nms_bwd(const Sched &sc, const uint8_t *cw, int64_t F, int T, const float *w, float *ckpt,
                   const float *dloss, float *grad_w, hipStream_t stream)
{
    const DecodeLaunch lc = plan_nms(sc);
    if (lc.G < 1)
        return fail(LDPC_ERANGE, "code with N=%d does not fit the training kernels' LDS budget", sc.N);
    const std::string pre = prelude(sc, lc, 0, 1);
    hipFunction_t bwd, red;
    int rc = get_function("nms", kJitNmsSource, pre, "ldpc_nms_bwd", &bwd);
    if (rc || (rc = get_function("nms", kJitNmsSource, pre, "ldpc_nms_grad_reduce", &red)))
        return rc;
    long long Fll = (long long)F, nwg = (F + lc.G - 1) / lc.G;
    int nw = T * sc.Mb * sc.Nb;
    float *partial = ckpt + nms_partial_offset(sc, F, T);
    void *a[] = {(void *)&cw, (void *)&Fll, (void *)&T, (void *)&w, (void *)&ckpt, (void *)&dloss, (void *)&partial};
    if ((rc = launch(bwd, (unsigned)nwg, lc.threads, stream, a, "nms adjoint")))
        return rc;
    void *ar[] = {(void *)&partial, (void *)&nwg, (void *)&nw, (void *)&grad_w};
    return launch(red, (unsigned)((nw + 63) / 64), 1024, stream, ar, "nms gradient sum");
}

}  // namespace ldpc
