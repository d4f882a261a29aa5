/*
 * ldpc.h -- C ABI of libldpc: QC-LDPC direct encoding and layered
 * single-scan min-sum decoding on AMD Instinct MI355X (gfx950).
 *
 * The operations follow Palenik & Szitkey, "High Throughput Open-Source
 * Implementation of Wi-Fi 6 and WiMAX LDPC Encoder and Decoder":
 *   - the code is given by its base (model) matrix H_bm and expansion factor
 *     Z (Sec. 1, eq. 2);
 *   - encoding maps K = K_b Z information bits to the systematic codeword
 *     c = [s p] (eq. 1) by the direct encoder of Sec. 2 (eqs. 8-15);
 *   - decoding maps channel LLRs (eq. 17, positive = bit 0) to hard bits
 *     (eq. 21), posterior LLRs (eq. 20) and an iteration count, running the
 *     layered single-scan min-sum of Sec. 4 (eqs. 18, 20, 22, 23) and
 *     stopping when H x = 0 if early termination is enabled.
 *
 * Conventions shared by every entry point
 *  - Base matrix: `hbm` is a HOST pointer to int16 [Mb][Nb], row-major.
 *    -1 is a zero block; s in [0, Z-1] is the identity cyclically shifted by
 *    s, where check row r of block row i reaches variable j*Z + (r+s) mod Z.
 *    Nb > Mb; N = Nb*Z, K = (Nb-Mb)*Z, M = Mb*Z.
 *  - Data: every other pointer is a DEVICE pointer, frame-major and
 *    row-contiguous ([F][N] means frame f, position n at f*N + n). Bits are
 *    one per byte (0/1). The caller owns every buffer; the library keeps no
 *    reference after the call returns.
 *  - Execution: calls enqueue work on `stream` (a hipStream_t; NULL is the
 *    null stream) and return before it finishes. Outputs are valid once the
 *    stream is synchronised. F = 0 is a no-op that returns LDPC_OK.
 *  - Errors: every call returns an int status. Arguments are validated on
 *    the host before anything is enqueued; on error nothing is enqueued and
 *    ldpc_last_error() describes the problem. No exception crosses the ABI.
 *  - Threads: calls may be made from several host threads; the per-thread
 *    error string is thread-local.
 */
#ifndef LDPC_H
#define LDPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes */
#define LDPC_OK 0
#define LDPC_EINVAL (-1)   /* null pointer, negative size, shift outside [-1, Z-1],
                              Nb <= Mb, a check row of degree < 2, max_iter < 1 */
#define LDPC_ESTRUCT (-2)  /* base matrix lacks the structure the direct encoder needs */
#define LDPC_ERANGE (-3)   /* valid code, but beyond this library's kernel limits */
#define LDPC_EDEVICE (-4)  /* a HIP runtime call failed */
#define LDPC_ENOMEM (-5)   /* host or device allocation failed */

/* Kernel limits (LDPC_ERANGE beyond these). */
#define LDPC_MAX_MB 16     /* block rows */
#define LDPC_MAX_NB 32     /* block columns */
#define LDPC_MAX_DEG 26    /* non-zero blocks in one block row (check degree) */
#define LDPC_MAX_Z 256     /* expansion factor */

/*
 * Describes a code without touching the GPU (Sec. 1). Fills out[8] with:
 *   N, K, M, E (edges = ones of H), the largest check degree, the row y of
 *   h_b used by the direct encoder (or -1 when the code is not directly
 *   encodable, eqs. 3-7), Mb, Nb.
 * Returns LDPC_OK or LDPC_EINVAL.
 */
int ldpc_code_info(const int16_t *hbm, int Mb, int Nb, int Z, int64_t out[8]);

/*
 * Direct encoder (Sec. 2, eqs. 12-15).
 *   info : device u8 [F][K], bits 0/1 (only bit 0 of each byte is read)
 *   cw   : device u8 [F][N], receives [info | v_0 .. v_{Mb-1}]
 * Requires the dual-diagonal structure of eqs. 3-7: h_b (column K_b) has
 * equal non-negative entries in rows 0 and Mb-1 and exactly one more in a
 * row y in between; H_b2' is the zero-shift staircase. Otherwise
 * LDPC_ESTRUCT.
 */
int ldpc_encode(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *info, uint8_t *cw, int64_t F,
                void *stream);

/*
 * Layered normalised min-sum decoder in FP32 (Sec. 4, eqs. 18-23).
 *   llr      : device f32 [F][N], channel LLRs (eq. 17), positive = bit 0
 *   max_iter : >= 1 iterations (one iteration = one pass over all Mb layers)
 *   alpha    : normalisation of the check messages, R = sgn * (alpha * min)
 *   early_term : nonzero -> stop a frame after the first iteration whose
 *              hard decisions satisfy H x = 0
 *   w        : nullable device f32 [max_iter][Mb][Nb]; when given, message
 *              leaving block column j of block row i in iteration t (0-based)
 *              is sgn * (w[t][i][j] * min) and alpha is ignored
 *   bits     : device u8 [F][N]  hard decisions x = [L <= 0] (eq. 21)
 *   post     : nullable device f32 [F][N] posterior LLRs (eq. 20)
 *   iters    : device i32 [F]    completed iterations (1..max_iter)
 *   ok       : nullable device u8 [F]  1 iff H x = 0 for the returned bits
 * Arithmetic is IEEE FP32 with round-to-nearest and no fused multiply-add.
 */
int ldpc_decode_f32(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, int64_t F, int max_iter,
                    float alpha, int early_term, const float *w, uint8_t *bits, float *post, int32_t *iters,
                    uint8_t *ok, void *stream);

/*
 * Saturating fixed-point layered min-sum: int8 channel LLRs, int8 check
 * messages, int16 posteriors (the fixed-point decoder of Sec. 5, with
 * saturation instead of wrap-around).
 *   llr     : device i8 [F][N]  (see ldpc_quantize_i8)
 *   offset  : offset min-sum beta in LSB, 0..127, used when wq == 0 and
 *             wq_table == NULL: magnitude = max(min - offset, 0)
 *   wq      : 0, or normalisation weight in 1/16 steps (1..31):
 *             magnitude = min(127, (wq*min + 8) >> 4)
 *   wq_table: nullable device u8 [max_iter][Mb][Nb] of 1/16-step weights
 *             (0..31) that replaces wq per iteration, block row and column
 *   post    : nullable device i16 [F][N]
 * |Q| is clipped to 127 before the minimum; sums saturate at +-32767.
 * Other arguments as for ldpc_decode_f32.
 */
int ldpc_decode_i8(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter,
                   int offset, int wq, const uint8_t *wq_table, int early_term, uint8_t *bits, int16_t *post,
                   int32_t *iters, uint8_t *ok, void *stream);

/*
 * As ldpc_decode_f32 / ldpc_decode_i8, with the hard bits written packed:
 * bits is device u8 [F][ceil(N/8)], bit n of frame f being bit (n mod 8) of
 * byte n/8 (the packed layout of ldpc_encode_packed). Needs run-time
 * specialisation (LDPC_ERANGE if LDPC_JIT=0).
 */
int ldpc_decode_f32_packed(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, int64_t F, int max_iter,
                           float alpha, int early_term, const float *w, uint8_t *bits, float *post, int32_t *iters,
                           uint8_t *ok, void *stream);
int ldpc_decode_i8_packed(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter,
                          int offset, int wq, const uint8_t *wq_table, int early_term, uint8_t *bits, int16_t *post,
                          int32_t *iters, uint8_t *ok, void *stream);

/*
 * Flooding (two-phase) min-sum, for comparison with the layered schedule
 * (Sec. 4, eqs. 18-23 without layering). Each iteration first computes every
 * check row's new messages from the posteriors of the previous iteration
 * (eqs. 22-23), then sets every posterior to the channel value plus the new
 * messages at that position, added in ascending block-row order (eq. 20),
 * then tests H x = 0 (eq. 21). Arguments, layouts, arithmetic (FP32 with
 * alpha; int8 with offset or wq/16, saturating) and outputs as
 * ldpc_decode_f32 / ldpc_decode_i8 without weight tables. Needs run-time
 * specialisation (LDPC_ERANGE if LDPC_JIT=0).
 */
int ldpc_decode_flood_f32(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, int64_t F, int max_iter,
                          float alpha, int early_term, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok,
                          void *stream);
int ldpc_decode_flood_i8(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter,
                         int offset, int wq, int early_term, uint8_t *bits, int16_t *post, int32_t *iters,
                         uint8_t *ok, void *stream);

/*
 * Packed bits (the bitmap encoder of Sec. 3). A frame of n bits takes
 * ceil(n/8) bytes; bit k is bit (k mod 8) of byte k/8 (least significant
 * bit first); unused high bits of the last byte are written as 0 and
 * ignored on input.
 *
 * ldpc_encode_packed: the direct encoder (eqs. 8-15) on packed bits, any Z:
 *   info : device u8 [F][ceil(K/8)],  cw : device u8 [F][ceil(N/8)].
 *   Same structure requirements and errors as ldpc_encode.
 * ldpc_shift_packed: the cyclic shift the encoder applies to Z-bit blocks,
 *   out[r] = in[(r + s) mod Z] for each of F blocks of ceil(Z/8) bytes
 *   (Algorithm A1 generalised to any Z), 0 <= s < Z.
 */
int ldpc_encode_packed(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *info, uint8_t *cw, int64_t F,
                       void *stream);
int ldpc_shift_packed(const uint8_t *in, uint8_t *out, int64_t F, int Z, int s, void *stream);

/*
 * Decode-layout autotuner. Times the code-specialised decode kernel of
 * `path` (0 FP32, 1 int8, 2 FP32 with a weight table w, 3 int8 with a
 * weight table wq_table; a zero table is used for the timing, since the work
 * does not depend on the weights) over candidate layouts -- frame groups per
 * workgroup (those whose lanes are at least 85% busy, and for Z <= 64 the
 * single-wave ones, which suit small batches), frames per thread, and how
 * many block rows keep their gather addresses in registers across
 * iterations -- on F zero-valued frames at max_iter fixed
 * iterations, and keeps the fastest for later ldpc_decode_f32/_i8 calls on
 * this code in this process (until ldpc_cache_clear). out[7] receives
 * {G, KF, FWp, threads, hoisted block rows, packed FP16, waves} of the
 * winner and *ms its time per launch. On paths 1 and 3, for codes
 * whose values fit FP16 exactly (column weight <= 15), layouts that decode
 * two frames per lane in packed FP16 are candidates too (then G counts frame
 * pairs). A layout whose kernel needs more than 128 VGPRs per lane is also
 * timed compiled for one more wave per SIMD (waves = 3 above 168 VGPRs,
 * else 4); such a variant may spill at most 32 bytes of registers per lane
 * (scratch memory, extra HBM traffic) and is kept only if it is at least 5%
 * faster than the fastest layout that does not spill. A decode with a
 * weight table uses the layout tuned on path 2 or 3 when there is one. Layouts
 * the tuner has not timed for the kernel at hand -- the default layout of an
 * untuned code, and a plain path's layout used with a weight table -- keep their
 * frames but, where the kernel needs more than 168 VGPRs, hoist fewer block
 * rows' gather addresses (Mb/2, Mb/4 or 0: the deepest that fits three
 * waves per SIMD without spilling); the first such call on a code compiles
 * up to four kernel variants to find it.
 * Synchronises `stream`; allocates and frees temporary device buffers.
 * LDPC_ERANGE if run-time specialisation is disabled (LDPC_JIT=0).
 */
int ldpc_autotune_decode(const int16_t *hbm, int Mb, int Nb, int Z, int path, int max_iter, int64_t F,
                         int32_t out[7], float *ms, void *stream);

/*
 * Decode layouts, for reproducible runs and for checking every layout the
 * autotuner may choose (the layouts change the launch shape and register
 * use, never the arithmetic of Sec. 4).
 * ldpc_decode_layouts: the layouts ldpc_autotune_decode times for this code
 *   and path (0..3 as for the tuner), in its order, each as the 7 integers of its out[7]; writes at
 *   most `cap` rows to out (int32 [cap][7], host) and returns the total count
 *   (>= 0) or a negative status. Compiles every candidate kernel (hipRTC) to
 *   read its registers and spills; no device memory is touched.
 * ldpc_set_decode_layout: makes `layout` (the 7 integers, as returned above
 *   or by ldpc_autotune_decode) this process's layout for later
 *   ldpc_decode_f32/_i8 calls on this code and path, as if the tuner had
 *   chosen it; NULL restores the default layout. LDPC_EINVAL if FWp or
 *   threads do not follow from G and KF, hoist is outside [0, Mb], waves is
 *   not 0, 3 or 4, or packed FP16 is asked for on a path other than 1, with
 *   KF 2 or for a code of column weight above 15; LDPC_ERANGE if the layout does
 *   not fit (threads, LDS).
 * Both need run-time specialisation (LDPC_ERANGE if LDPC_JIT=0).
 */
int ldpc_decode_layouts(const int16_t *hbm, int Mb, int Nb, int Z, int path, int32_t *out, int cap);
int ldpc_set_decode_layout(const int16_t *hbm, int Mb, int Nb, int Z, int path, const int32_t layout[7]);

/*
 * Learned normalised min-sum (training). Weights w[T][Mb][Nb] (device f32)
 * replace the fixed normalisation: in iteration t (0-based) the message
 * leaving block column j of block row i is sgn * fl(w[t][i][j] * min), in the
 * layered schedule of Sec. 4 with early termination off. The loss is binary
 * cross-entropy of sigmoid(L) (probability of bit 0, eq. 17) against the
 * transmitted codeword after every iteration:
 *   loss[t] = 1/(T F N) sum_f sum_n softplus(-(1 - 2 cw[f][n]) L_fn after iteration t),
 * so that sum_t loss[t] is the mean per-bit, per-iteration BCE.
 *
 * ldpc_nms_ckpt_bytes: size of the checkpoint buffer for F frames and T
 *   iterations (0 on invalid arguments); the caller allocates it on the device.
 * ldpc_nms_fwd: runs the T iterations on llr (device f32 [F][N]) with target
 *   cw (device u8 [F][N]); writes per-iteration checkpoints into ckpt, loss
 *   (device f32 [T]) and optionally the final posteriors post ([F][N]).
 * ldpc_nms_bwd: hand-written adjoint. From the checkpoints of a forward call
 *   with the same arguments and dloss (device f32 [T], the gradient of the
 *   objective with respect to each loss[t]) computes grad_w (device f32
 *   [T][Mb][Nb], overwritten). Entries of w at zero blocks (-1 in H_bm) get a
 *   zero gradient. Iterations are recomputed from their checkpoints. The last
 *   part of ckpt (past the checkpoints and loss terms) receives each
 *   workgroup's partial gradients, which a second kernel sums in a fixed
 *   order, so grad_w is the same on every run.
 * Both need run-time specialisation (LDPC_ERANGE if LDPC_JIT=0).
 */
size_t ldpc_nms_ckpt_bytes(const int16_t *hbm, int Mb, int Nb, int Z, int64_t F, int T);
int ldpc_nms_fwd(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, const uint8_t *cw, int64_t F, int T,
                 const float *w, void *ckpt, size_t ckpt_bytes, float *loss, float *post, void *stream);
int ldpc_nms_bwd(const int16_t *hbm, int Mb, int Nb, int Z, const uint8_t *cw, int64_t F, int T, const float *w,
                 void *ckpt, size_t ckpt_bytes, const float *dloss, float *grad_w, void *stream);

/*
 * Seeded information bits from Philox4x32-10 (Salmon et al., SC'11):
 * bit k of frame f is bit (k mod 32) of word (k/32 mod 4) of
 * Philox(counter = {k/128, f, 0, 0}, key = {seed low, seed high}).
 *   seed_dev : nullable device u64 [1]; when given, the kernel reads the
 *              seed from it instead of `seed` (so that a captured graph can
 *              be replayed with a new seed written to that buffer)
 *   info : device u8 [F][K]
 */
int ldpc_random_bits(uint64_t seed, const uint64_t *seed_dev, int64_t F, int64_t K, uint8_t *info, void *stream);

/*
 * BPSK over AWGN and the channel LLR (eqs. 16-17):
 *   LLR = ((1 - 2x) + sigma * z) * scale, with scale = 2 / sigma^2 chosen by
 * the caller, evaluated in FP32 without fused multiply-add. z is a standard
 * normal from Box-Muller on Philox(counter = {n/4, f, 1, 0}, key = seed):
 * words (2p, 2p+1) with p = (n mod 4)/2 give u = ((word >> 8) + 1/2) 2^-24,
 * z = sqrt(-2 ln u_a) * (cos for even n, sin for odd n)(2 pi u_b).
 *   seed_dev : nullable device u64 [1] that replaces `seed` when given
 *   cw  : device u8 [F][N] codeword bits,  llr : device f32 [F][N]
 *   sigma_f, scale_f : nullable device f32 [F]; when given (both), frame f
 *         uses sigma_f[f] and scale_f[f] instead of sigma and scale
 */
int ldpc_awgn_llr(uint64_t seed, const uint64_t *seed_dev, const uint8_t *cw, int64_t F, int64_t N, float sigma,
                  float scale, const float *sigma_f, const float *scale_f, float *llr, void *stream);

/*
 * Decoding statistics against the transmitted information bits (the first K
 * bits of each codeword, eq. 1). Adds to counters (device int64 [4], not
 * cleared): [0] information-bit errors, [1] frames with any such error,
 * [2] iterations (if iters is given), [3] frames with ok == 0 (if ok is
 * given). bits: device u8 [F][N]; info: device u8 [F][K].
 */
int ldpc_frame_stats(const uint8_t *bits, const uint8_t *info, const int32_t *iters, const uint8_t *ok, int64_t F,
                     int64_t N, int64_t K, int64_t *counters, void *stream);

/*
 * Measurement utility (no counterpart in the paper): LDS read bandwidth.
 * Launches `blocks` workgroups of 256 threads; each thread reads
 * rounds * 8 16-byte words from a 64 KB LDS buffer and writes a checksum to
 * out[block * 256 + thread] (device f32 [blocks * 256]). Bytes read =
 * blocks * 256 * rounds * 128; time the call on `stream` with events.
 * LDPC_EINVAL unless 1 <= blocks, rounds <= 2^20.
 */
int ldpc_lds_probe(int blocks, int rounds, float *out, void *stream);

/*
 * Fallback: the frames whose ok flag is 0 after a decode are decoded again
 * from their channel LLRs with fresh state by plain min-sum (FP32 weight
 * alpha; int8 offset or wq/16 as for ldpc_decode_i8) with early termination
 * and at most max_iter iterations; their bits, posteriors (if post is given),
 * iteration counts and ok flags are overwritten, the other frames are left
 * as they are. work: device int64 [F + 1] scratch (receives the count and
 * the list of re-decoded frames, in frame order). The list length stays on
 * the device: no host synchronisation.
 */
int ldpc_fallback_f32(const int16_t *hbm, int Mb, int Nb, int Z, const float *llr, int64_t F, int max_iter,
                      float alpha, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok, int64_t *work,
                      void *stream);
int ldpc_fallback_i8(const int16_t *hbm, int Mb, int Nb, int Z, const int8_t *llr, int64_t F, int max_iter, int offset,
                     int wq, uint8_t *bits, int16_t *post, int32_t *iters, uint8_t *ok, int64_t *work, void *stream);

/*
 * Code sets and batched decoding of frames of different codes in one
 * persistent launch (different Z, rate and length).
 *
 * ldpc_codeset_create: compiles `ncodes` base matrices (host pointers
 *   hbm[c], each int16 [Mb[c]][Nb[c]], expansion Z[c]) into device tables on
 *   the current device. Codes with the same block structure share a kernel
 *   body. *out receives an opaque handle owned by the caller (free it with
 *   ldpc_codeset_destroy). At most 1024 codes; each code needs Z <= 256.
 * ldpc_codeset_info: out[8] = {N, K, M, E, dmax, structure class, frames per
 *   work item, number of classes} of code `code`.
 * ldpc_batch_work_bytes: size of the device scratch buffer for F frames.
 * ldpc_decode_batch_f32 / _i8: decodes F frames; frame f belongs to code
 *   code_id[f] (device i32 [F]) and its N values start at element off[f]
 *   (device i64 [F]) of llr, and at the same offset in bits and post; llr,
 *   bits and post (if given) hold n_llr elements each; iters and ok are [F].
 *   Frames are grouped by code on the device and cut into work items that
 *   the workgroups of a persistent grid take from an atomic queue.
 *   Arithmetic and arguments as ldpc_decode_f32 (alpha) / ldpc_decode_i8
 *   (offset, wq; no weight table). A frame whose code id is outside
 *   [0, ncodes), or whose values would not lie inside the n_llr elements
 *   (off[f] < 0 or off[f] + N > n_llr; checked on the device), is not
 *   decoded: its iters entry is set to -1 and its ok entry to 0, its bits and
 *   posteriors are left as they are. No host synchronisation: the call can
 *   be captured in a hipGraph. Calls that share a work buffer must not
 *   overlap.
 */
typedef struct ldpc_codeset ldpc_codeset;
int ldpc_codeset_create(const int16_t *const *hbm, const int *Mb, const int *Nb, const int *Z, int ncodes,
                        ldpc_codeset **out);
void ldpc_codeset_destroy(ldpc_codeset *cs);
int ldpc_codeset_info(const ldpc_codeset *cs, int code, int64_t out[8]);
size_t ldpc_batch_work_bytes(const ldpc_codeset *cs, int64_t F);
int ldpc_decode_batch_f32(const ldpc_codeset *cs, const int32_t *code_id, const int64_t *off, const float *llr,
                          int64_t n_llr, int64_t F, int max_iter, float alpha, int early_term, uint8_t *bits,
                          float *post, int32_t *iters, uint8_t *ok, void *work, size_t work_bytes, void *stream);
int ldpc_decode_batch_i8(const ldpc_codeset *cs, const int32_t *code_id, const int64_t *off, const int8_t *llr,
                         int64_t n_llr, int64_t F, int max_iter, int offset, int wq, int early_term, uint8_t *bits,
                         int16_t *post, int32_t *iters, uint8_t *ok, void *work, size_t work_bytes, void *stream);

/*
 * Allocation-free batched FP32 decode, for callers that cannot allocate
 * device memory during a call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation). Arguments, arithmetic and
 * outputs as ldpc_decode_batch_f32, without the work buffer: the work list
 * lives in a static device array of the library, one per GPU, kept until
 * the process ends, with room for F <= 262144 frames (LDPC_ERANGE beyond).
 * The call allocates nothing and loads no kernel: the code set's batch
 * kernels for the FP32 path at its current layout must already be loaded on
 * this device by an earlier ldpc_decode_batch_f32 or ldpc_codeset_autotune
 * call (FP32), else LDPC_ERANGE. Every call on one GPU shares the one array:
 * calls that overlap on a GPU (on different streams, or from several host
 * threads) race and must be ordered by the caller.
 */
int ldpc_decode_batch_f32_noalloc(const ldpc_codeset *cs, const int32_t *code_id, const int64_t *off,
                                  const float *llr, int64_t n_llr, int64_t F, int max_iter, float alpha,
                                  int early_term, uint8_t *bits, float *post, int32_t *iters, uint8_t *ok,
                                  void *stream);

/*
 * Batch layout autotuner (frames per work item and workgroup size of the
 * persistent kernel). Decodes the caller's batch -- same arguments as
 * ldpc_decode_batch_f32/_i8 for `path` 0/1 -- with alpha 0.75 (FP32) or
 * offset 1 (int8), early termination off, under each candidate layout:
 * workgroups of 192, 256, 384 or 512 threads (those at least as wide as
 * the largest Z of the set), each code's work items holding
 * floor(threads / Z) frames (at most 64), and for 256 and 512 threads also
 * half as many. Keeps the fastest
 * for later batched decodes of `path` with this code set; out[2] receives
 * {threads, divisor} and *ms its time per decode. bits and iters receive the
 * last decode's results. Synchronises `stream`; the code set must not be in
 * use on another stream meanwhile (its tables are rebuilt).
 */
/*
 * ldpc_codeset_set_layout: makes one of the batch autotuner's layouts
 * (threads in {192, 256, 384, 512} with divisor 1, or {256, 512} with
 * divisor 2) the layout of later batched decodes of `path` with this code
 * set, as if the tuner had chosen it (for reproducible runs, and to check
 * every layout the tuner may choose). Rebuilds the path's device tables
 * (allocates device memory); the code set must not be in use on another
 * stream meanwhile. LDPC_EINVAL for another layout, LDPC_ERANGE if a code's
 * Z exceeds the workgroup or its frames do not fit the LDS budget.
 */
int ldpc_codeset_set_layout(ldpc_codeset *cs, int path, int threads, int divisor);
int ldpc_codeset_autotune(ldpc_codeset *cs, int path, const int32_t *code_id, const int64_t *off, const void *llr,
                          int64_t n_llr, int64_t F, int max_iter, uint8_t *bits, int32_t *iters, void *work,
                          size_t work_bytes, int32_t out[2], float *ms, void *stream);

/*
 * The paper's own fixed point (Sec. 5): layered min-sum on int16 values,
 * Q_B-bit LLRs with headroom. Per check row: Q = fix(L - R), the two
 * smallest |Q| and the sign parity in one scan, message R =
 * fix(sgn * ((wq * m + 8) >> 4)) with m the minimum over the other edges,
 * L = fix(Q + R); fix() wraps around to int16 (wrap != 0, the C decoder's
 * arithmetic) or saturates symmetrically at +-32767 (wrap == 0). wq/16 is
 * the normalisation, wq in [1, 31] (16: plain min-sum). llr: device i16
 * [F][N] (see ldpc_quantize_q16); post: nullable device i16 [F][N]; other
 * arguments as ldpc_decode_i8. Needs run-time specialisation.
 *
 * ldpc_quantize_q16: q = clamp(rint(scale * llr), -qmax, qmax), half to
 * even (Q_B = 10: qmax = 1023). llr: device f32 [n], q: device i16 [n].
 */
int ldpc_decode_q16(const int16_t *hbm, int Mb, int Nb, int Z, const int16_t *llr, int64_t F, int max_iter, int wq,
                    int wrap, int early_term, uint8_t *bits, int16_t *post, int32_t *iters, uint8_t *ok, void *stream);
int ldpc_quantize_q16(const float *llr, int16_t *q, int64_t n, float scale, int qmax, void *stream);

/*
 * int8 quantiser for channel LLRs: q = clamp(rint(scale * llr), -127, 127),
 * rounding half to even. llr: device f32 [n], q: device i8 [n].
 */
int ldpc_quantize_i8(const float *llr, int8_t *q, int64_t n, float scale, void *stream);

/*
 * Learned weights in 1/16 steps for the fixed-point decoder (the wq_table of
 * ldpc_decode_i8, Sec. 5 fixed point with a learned normalisation):
 * wq = clamp(rint(16 w), 0, 31), rounding half to even; a NaN weight gives 0.
 * w: device f32 [n], wq: device u8 [n]. Returns LDPC_EINVAL for n < 0 or a
 * null pointer with n > 0.
 */
int ldpc_quantize_weights(const float *w, uint8_t *wq, int64_t n, void *stream);

/* Message for the last failing call on this host thread ("" if none). */
const char *ldpc_last_error(void);

/* Drops cached per-code device tables (safe to call at any time). */
void ldpc_cache_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* LDPC_H */
