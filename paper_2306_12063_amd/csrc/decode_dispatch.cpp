// Picks the compiled decode-kernel shape for a code: the smallest
// (block rows, max degree) variant that holds it.
#include "decode_common.h"

namespace ldpc {

namespace {

// Shapes compiled into the library (one object each). Unused layer and edge
// slots of a larger shape are skipped by uniform branches.
struct Shape {
    int mb, maxd;
};
constexpr Shape kShapes[] = {{4, 20}, {6, 20}, {8, 16}, {12, 12}, {12, 16}, {16, 26}};

int pick_shape(const Sched &sc)
{
    int best = -1;
    for (int s = 0; s < (int)(sizeof(kShapes) / sizeof(kShapes[0])); ++s) {
        if (kShapes[s].mb < sc.Mb || kShapes[s].maxd < sc.dmax)
            continue;
        if (best < 0 || kShapes[s].mb * kShapes[s].maxd < kShapes[best].mb * kShapes[best].maxd)
            best = s;
    }
    return best;
}

}  // namespace

#define LDPC_SHAPE_CASES(RUN, ...)                  \
    switch (pick_shape(sc)) {                       \
    case 0: return RUN<4, 20>(__VA_ARGS__);         \
    case 1: return RUN<6, 20>(__VA_ARGS__);         \
    case 2: return RUN<8, 16>(__VA_ARGS__);         \
    case 3: return RUN<12, 12>(__VA_ARGS__);        \
    case 4: return RUN<12, 16>(__VA_ARGS__);        \
    case 5: return RUN<16, 26>(__VA_ARGS__);        \
    default: return fail(LDPC_ERANGE, "no decode kernel shape for Mb=%d, degree %d", sc.Mb, sc.dmax); \
    }

int launch_decode_f32(const Sched &sc, const DecodeLaunch &lc, const float *llr, const int64_t *fidx, int64_t F,
                      int max_iter, float alpha, int early_term, const float *w, uint8_t *bits, float *post,
                      int32_t *iters, uint8_t *ok, hipStream_t stream)
{
    LDPC_SHAPE_CASES(run_decode_f32, sc, lc, llr, fidx, F, max_iter, alpha, early_term, w, bits, post, iters, ok,
                     stream)
}

int launch_decode_i8(const Sched &sc, const DecodeLaunch &lc, const int8_t *llr, const int64_t *fidx, int64_t F,
                     int max_iter, int offset, int wq, const uint8_t *wq_table, int early_term, uint8_t *bits,
                     int16_t *post, int32_t *iters, uint8_t *ok, hipStream_t stream)
{
    LDPC_SHAPE_CASES(run_decode_i8, sc, lc, llr, fidx, F, max_iter, offset, wq, wq_table, early_term, bits, post,
                     iters, ok, stream)
}

}  // namespace ldpc
