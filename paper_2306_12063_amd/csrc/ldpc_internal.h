// Internal declarations of libldpc (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ldpc.h"

namespace ldpc {

constexpr int kMaxMb = LDPC_MAX_MB;
constexpr int kMaxNb = LDPC_MAX_NB;
constexpr int kMaxDeg = LDPC_MAX_DEG;
constexpr int kMaxZ = LDPC_MAX_Z;
// Largest workgroup the decode kernels are compiled for.
constexpr int kMaxThreads = 256;
// Largest workgroup of a run-time specialised decode kernel.
constexpr int kMaxJitThreads = 512;
// Dynamic LDS a decode workgroup may take (two workgroups fit one CU).
constexpr int kLdsBudget = 56 * 1024;

// Compiled form of a base matrix: the gather schedule of the layered decoder
// and the encoder's parity-column data. It is small enough to travel as a
// kernel argument, so single-code launches need no device-side tables.
//
// For block row i, edges e = 0 .. deg[i]-1 are the non-zero blocks in
// ascending block column; edge[i][e] = (col << 16) | shift. Check row r of
// block row i reaches variable col*Z + (r + shift) mod Z through edge e.
struct Sched {
    int32_t Z, Mb, Nb, N, K, M, E, dmax;
    int32_t enc_y;             // row y of h_b for the direct encoder, or -1
    int32_t hb[kMaxMb];        // h_b = column K_b of H_bm (-1 = zero block)
    int32_t deg[kMaxMb];
    uint32_t edge[kMaxMb][kMaxDeg];
};

// Builds the schedule; returns LDPC_OK, LDPC_EINVAL or LDPC_ERANGE and sets
// the thread's error string on failure. need_deg2: every check row must have
// at least two edges (decoders); need_enc: the encoder structure must hold.
int compile_sched(const int16_t *hbm, int Mb, int Nb, int Z, bool need_deg2, Sched *out);

// Thread-local error string helpers. check_launch() turns a pending HIP
// launch error into LDPC_EDEVICE with the runtime's message.
int fail(int code, const char *fmt, ...);
void clear_error();
int check_launch(const char *what);

// Launch configuration of a decode kernel.
struct DecodeLaunch {
    int G;       // frame groups per workgroup (each group has Z threads)
    int KF;      // frames per thread
    int FW;      // frames per workgroup = G*KF
    int FWp;     // LDS row stride in elements (FW, padded against bank conflicts)
    int threads; // workgroup size
    size_t lds;  // LDS bytes of the posteriors
    int hoist = 0;  // specialised kernels: block rows whose gather addresses stay in registers
    int h2 = 0;     // fixed point with two frames per lane in packed FP16 (G = frame pairs, FW = 2G)
    int waves = 0;  // specialised kernels: occupancy target in waves per SIMD (0: the compiler's choice)
    int tuned = 0;  // chosen by the autotuner for this code's plain kernel
};

// Largest column weight (block rows with an edge in a block column).
int max_col_weight(const Sched &sc);
// Whether the packed-FP16 fixed-point kernel applies: its values, at most
// 127 * (1 + column weight), must be exact in FP16 (<= 2048).
inline bool h2_eligible(const Sched &sc) { return max_col_weight(sc) <= 15; }
// A layout with G frame pairs per workgroup for the packed-FP16 kernel
// (G < 1 if it does not fit).
DecodeLaunch make_h2_launch(const Sched &sc, int G, int max_threads);
// The layout to use for (path, mode): a packed-FP16 layout is replaced by
// the default one where it does not apply (FP32, weight tables).
DecodeLaunch usable_launch(const Sched &sc, const DecodeLaunch &lc, int path, int mode);
// The layout of a decode call on arithmetic path `path` in kernel `mode`: a
// layout the tuner timed for this kernel (with a weight table: tuning path
// path + 2), else the plain path's tuned or default layout made usable.
DecodeLaunch decode_layout(const Sched &sc, int path, int mode);

// Kernel launchers (decode_kernels.hip). Return LDPC_OK or LDPC_EDEVICE.
int launch_decode_f32(const Sched &sc, const DecodeLaunch &lc, const float *llr, const int64_t *fidx, int64_t F,
                      int max_iter, float alpha, int early_term, const float *w, uint8_t *bits, float *post,
                      int32_t *iters, uint8_t *ok, hipStream_t stream);
int launch_decode_i8(const Sched &sc, const DecodeLaunch &lc, const int8_t *llr, const int64_t *fidx, int64_t F,
                     int max_iter, int offset, int wq, const uint8_t *wq_table, int early_term, uint8_t *bits,
                     int16_t *post, int32_t *iters, uint8_t *ok, hipStream_t stream);
int launch_quantize_i8(const float *llr, int8_t *q, int64_t n, float scale, hipStream_t stream);
int launch_quantize_q16(const float *llr, int16_t *q, int64_t n, float scale, int qmax, hipStream_t stream);
int launch_quantize_weights(const float *w, uint8_t *wq, int64_t n, hipStream_t stream);
int launch_shift_packed(const uint8_t *in, uint8_t *out, int64_t F, int Z, int s, hipStream_t stream);
int launch_encode_packed(const Sched &sc, const uint8_t *info, uint8_t *cw, int64_t F, hipStream_t stream);
int launch_encode(const Sched &sc, const uint8_t *info, uint8_t *cw, int64_t F, hipStream_t stream);
int launch_random_bits(uint64_t seed, const uint64_t *seed_dev, int64_t F, int64_t K, uint8_t *info,
                       hipStream_t stream);
int launch_awgn_llr(uint64_t seed, const uint64_t *seed_dev, int64_t F, int64_t N, const uint8_t *cw, float sigma, float scale,
                    const float *sigma_f, const float *scale_f, float *llr, hipStream_t stream);
int launch_frame_stats(const uint8_t *bits, const uint8_t *info, const int32_t *iters, const uint8_t *ok, int64_t F,
                       int64_t N, int64_t K, int64_t *counters, hipStream_t stream);
int launch_compact_failed(const uint8_t *ok, int64_t F, int64_t *out, hipStream_t stream);
int launch_lds_probe(int blocks, int rounds, float *out, hipStream_t stream);

// Run-time specialised decode kernels (jit.cpp). path: 0 FP32, 1 int8;
// mode as in jit_decode.hip. LDPC_JIT=0 in the environment disables them.
bool jit_enabled();
void jit_cache_clear();
// Function `name` of the module built from prelude + source (cached per device).
int jit_function(const char *tag, const char *src, const std::string &pre, const char *name, hipFunction_t *fn);
// Static scratch of ldpc_decode_batch_f32_noalloc: the batched decode's
// work list for up to kBatchScratchFrames frames of a code set of up to 1024
// codes (2 + 3 * 1024 queue words, then 32 bytes per frame and 16 per code).
constexpr int kBatchScratchFrames = 1 << 18;
constexpr size_t kBatchScratchBytes =
    ((size_t)(3074 + 2 * (size_t)kBatchScratchFrames) * 8 + ((size_t)kBatchScratchFrames + 1024) * 16 + 255) &
    ~(size_t)255;
// Device address of the static scratch on device `dev` (which must be
// current): looked up once per device, then cached.
int batch_scratch(int dev, void **out);

// As jit_function, but only finds a kernel whose module this process has
// already loaded on the current device; never compiles or loads a module
// (LDPC_ERANGE if it is not loaded).
int jit_function_loaded(const char *tag, const std::string &pre, const char *name, hipFunction_t *fn);
int jit_launch(hipFunction_t fn, unsigned blocks, unsigned threads, hipStream_t stream, void **args, const char *what);
// Default run-time specialised decode layout: one frame per thread (each
// thread keeps one FP32 message per edge of its check rows), gather
// addresses kept in registers when they fit beside the messages.
DecodeLaunch jit_default_launch(const Sched &sc, int path);
// Bytes of per-lane scratch the specialised decode kernel for this layout
// needs (register spills) and its VGPRs per lane; compiles the variant if
// necessary.
int jit_decode_scratch(const Sched &sc, const DecodeLaunch &lc, int path, int mode, size_t *bytes,
                       int *vgprs = nullptr);
// Flooding schedule (jit_flood.hip): layout and launch.
DecodeLaunch flood_launch(const Sched &sc);
int launch_jit_flood(const Sched &sc, const DecodeLaunch &lc, int path, int mode, const void *llr, int64_t F,
                     int max_iter, float alpha, int offset, int wq, int et, uint8_t *bits, void *post, int32_t *iters,
                     uint8_t *ok, hipStream_t stream);
// The paper's int16 Q_B-bit fixed point (jit_q16.hip).
int launch_jit_q16(const Sched &sc, const DecodeLaunch &lc, int wrap, const int16_t *llr, int64_t F, int max_iter,
                   int wq, int et, uint8_t *bits, int16_t *post, int32_t *iters, uint8_t *ok, hipStream_t stream);
int launch_jit_decode(const Sched &sc, const DecodeLaunch &lc, int path, int mode, const void *llr,
                      const int64_t *fidx, int64_t F, int max_iter, float alpha, int offset, int wq, int et,
                      const void *wt, uint8_t *bits, void *post, int32_t *iters, uint8_t *ok, hipStream_t stream,
                      const int64_t *Fdev = nullptr, bool packed = false);

// Learned normalised min-sum training kernels (jit.cpp, jit_nms.hip).
size_t nms_ckpt_floats(const Sched &sc, int64_t F, int T);
int launch_nms_fwd(const Sched &sc, const float *llr, const uint8_t *cw, int64_t F, int T, const float *w,
                   float *ckpt, float *loss, float *post, hipStream_t stream);
int launch_nms_bwd(const Sched &sc, const uint8_t *cw, int64_t F, int T, const float *w, float *ckpt,
                   const float *dloss, float *grad_w, hipStream_t stream);

// Picks G/KF for a code and element size (4 for FP32, 2 for int16 posteriors).
DecodeLaunch plan_decode(const Sched &sc, int elem_bytes, int kf_hint);
// Layout for a given G and KF (G < 1 in the result if it does not fit).
DecodeLaunch make_launch(const Sched &sc, int elem_bytes, int G, int KF, int max_threads);

// Decode layout chosen by the autotuner for this code and path, if any.
// Tuning paths of the decode-layout autotuner: 0 FP32, 1 int8, 2 FP32 with a
// weight table, 3 int8 with a weight table. The arithmetic path is path & 1;
// the kernel mode is that of the plain decoder (alpha, offset) or of a
// weight table.
inline int tune_mode(int tpath) { return tpath == 2 ? 1 : (tpath == 3 ? 2 : 0); }
inline bool mode_has_table(int tpath) { return tpath >= 2; }
bool tuned_launch(const Sched &sc, int path, DecodeLaunch *out);
void set_tuned_launch(const Sched &sc, int path, const DecodeLaunch &lc);
void tune_cache_clear();
void clear_tuned_launch(const Sched &sc, int path);
// Every layout the autotuner times for this code and path, in timing order
// (compiles each candidate to read its registers and spills); scratch
// receives each layout's spilled bytes per lane.
int tuner_layouts(const Sched &sc, int path, std::vector<DecodeLaunch> *out, std::vector<size_t> *scratch);
// Times candidate layouts of the specialised kernel (jit) on F zero frames.
int autotune_decode(const Sched &sc, int path, int max_iter, int64_t F, hipStream_t stream, DecodeLaunch *best,
                    float *best_ms);

}  // namespace ldpc
