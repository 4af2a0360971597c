// VDF / DDF window kernels for the 5x5 window (instantiations and launcher).
#include "kern_angle.h"
#include "kern_stream_split.h"
#include "batch.h"

namespace vf {

#define VF_ANGLE_CASE(F, MODE, NLO, NHI)                                                   \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI) {                       \
        hipLaunchKernelGGL((angle_kernel<F, 5, MODE, NLO, NHI>), dim3(blocks), dim3(kTileX * angle_tile_y<5>()), \
                           0, (hipStream_t)stream, p);                                     \
        return (int)hipGetLastError();                                                     \
    }

#define VF_ANGLE_MODES(F)          \
    VF_ANGLE_CASE(F, EV_EXACT, 0, 0) \
    VF_ANGLE_CASE(F, EV_PAPER, 5, 5) \
    VF_ANGLE_CASE(F, EV_SPLIT, 2, 2) \
    VF_ANGLE_CASE(F, EV_SPLIT, 3, 3) \
    VF_ANGLE_CASE(F, EV_SPLIT, 4, 4) \
    VF_ANGLE_CASE(F, EV_SPLIT, 5, 5) \
    VF_ANGLE_CASE(F, EV_CHORD, 0, 4) \
    VF_ANGLE_CASE(F, EV_CHORD, 0, 5) \
    VF_ANGLE_CASE(F, EV_CHORD, 0, 6) \
    VF_ANGLE_CASE(F, EV_CHORD, 0, 7)

int launch_angle_w5(int filter, int eval, int n_lo, int n_hi, const KParams& p, int blocks,
                    void* stream) {
    VF_ANGLE_MODES(VF_FILTER_VDF)
    VF_ANGLE_MODES(VF_FILTER_DDF)
    return -1;
}

// DDF runs the two-waves-per-SIMD form (except in exact mode, whose three
// sums per member need all registers), the unrolled VDF kernels the
// three-wave form (see stream_kernel_w)
// The exact-acosf VDF (two sums per member) splits each window's state over
// two waves (kern_stream_split.h): 4096^2 kernel 2.05 -> 1.91 ms. Split DDF
// 5x5 kernels measured slower (chord 1.39 -> 1.86 ms at two waves).
template <int F, int MODE>
constexpr bool split5() { return F == VF_FILTER_VDF && MODE == EV_EXACT; }

template <int F, int MODE>
constexpr int stream5_waves() {
    return F == VF_FILTER_DDF ? (MODE == EV_EXACT ? 0 : 2) : (stream_unrolled<F, 5, MODE>() ? 3 : 0);
}

template <int F, int MODE, int NLO, int NHI>
static void launch_stream5(const KParams& p, int blocks, void* stream) {
    constexpr int WV = stream5_waves<F, MODE>();
    if constexpr (split5<F, MODE>())
        stream_split_launch<2>(stream_split_kernel<2, F, 5, MODE, NLO, NHI>, p, blocks, stream);
    else if constexpr (WV > 0)
        stream_launch(stream_kernel_w<WV, F, 5, MODE, NLO, NHI>, p, blocks, stream);
    else
        stream_launch(stream_kernel<F, 5, MODE, NLO, NHI>, p, blocks, stream);
}

#define VF_STREAM_CASE(F, MODE, NLO, NHI)                                                   \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI) {                        \
        launch_stream5<F, MODE, NLO, NHI>(p, blocks, stream);                               \
        return (int)hipGetLastError();                                                      \
    }

int launch_angle_stream_w5(int filter, int eval, int n_lo, int n_hi, const KParams& p, int blocks,
                            void* stream) {
    VF_STREAM_CASE(VF_FILTER_VDF, EV_EXACT, 0, 0)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_EXACT, 0, 0)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_PAPER, 5, 5)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_PAPER, 5, 5)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_SPLIT, 2, 2)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_SPLIT, 2, 2)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_SPLIT, 3, 3)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_SPLIT, 3, 3)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_SPLIT, 4, 4)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_SPLIT, 4, 4)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_SPLIT, 5, 5)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_SPLIT, 5, 5)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_CHORD, 0, 4)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_CHORD, 0, 4)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_CHORD, 0, 5)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_CHORD, 0, 5)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_CHORD, 0, 6)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_CHORD, 0, 6)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_CHORD, 0, 7)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_CHORD, 0, 7)
    return -1;
}

template <int FILT, int WIN, int MODE, int NLO, int NHI>
__global__ __launch_bounds__(kTileX * angle_tile_y<WIN>()) void angle_batch_kernel(const BatchParams bp) {
    batch_loop(bp, [&](const KParams& p, int tile) { angle_tile<FILT, WIN, MODE, NLO, NHI>(p, tile); });
}



#define VF_BATCH_DIRECT(F, MODE, NLO, NHI)                                                     \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI && !streaming)                \
        return launch_persistent(probe, angle_batch_kernel<F, 5, MODE, NLO, NHI>,                         \
                                 kTileX * angle_tile_y<5>(), bp, num_cus, stream);

template <int F, int MODE, int NLO, int NHI>
static int launch_stream5_batch(bool probe, const BatchParams& bp, int num_cus, void* stream) {
    constexpr int WV = stream5_waves<F, MODE>();
    if constexpr (split5<F, MODE>())
        return launch_persistent(probe, stream_split_batch_kernel<2, F, 5, MODE, NLO, NHI>, 128, bp, num_cus, stream);
    else if constexpr (WV > 0)
        return launch_persistent(probe, stream_batch_kernel_w<WV, F, 5, MODE, NLO, NHI>, 64, bp, num_cus, stream);
    else
        return launch_persistent(probe, stream_batch_kernel<F, 5, MODE, NLO, NHI>, 64, bp, num_cus, stream);
}

#define VF_BATCH_STREAM(F, MODE, NLO, NHI)                                                     \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI && streaming)                 \
        return launch_stream5_batch<F, MODE, NLO, NHI>(probe, bp, num_cus, stream);

// Persistent batch launch. Returns -1 when no kernel matches (the streaming
// combinations are those of the single-image streaming launcher); with
// `probe` set it only reports whether one does (0) and launches nothing.
int launch_angle_batch_w5(int filter, int eval, int n_lo, int n_hi, bool streaming, const BatchParams& bp,
                           int num_cus, void* stream, bool probe) {
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_EXACT, 0, 0)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_EXACT, 0, 0)
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_PAPER, 5, 5)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_PAPER, 5, 5)
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_SPLIT, 2, 2)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_SPLIT, 2, 2)
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_SPLIT, 3, 3)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_SPLIT, 3, 3)
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_SPLIT, 4, 4)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_SPLIT, 4, 4)
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_SPLIT, 5, 5)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_SPLIT, 5, 5)
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_CHORD, 0, 4)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_CHORD, 0, 4)
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_CHORD, 0, 5)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_CHORD, 0, 5)
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_CHORD, 0, 6)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_CHORD, 0, 6)
    VF_BATCH_DIRECT(VF_FILTER_VDF, EV_CHORD, 0, 7)
    VF_BATCH_STREAM(VF_FILTER_VDF, EV_CHORD, 0, 7)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_EXACT, 0, 0)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_EXACT, 0, 0)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_PAPER, 5, 5)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_PAPER, 5, 5)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_SPLIT, 2, 2)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_SPLIT, 2, 2)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_SPLIT, 3, 3)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_SPLIT, 3, 3)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_SPLIT, 4, 4)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_SPLIT, 4, 4)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_SPLIT, 5, 5)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_SPLIT, 5, 5)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_CHORD, 0, 4)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_CHORD, 0, 4)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_CHORD, 0, 5)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_CHORD, 0, 5)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_CHORD, 0, 6)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_CHORD, 0, 6)
    VF_BATCH_DIRECT(VF_FILTER_DDF, EV_CHORD, 0, 7)
    VF_BATCH_STREAM(VF_FILTER_DDF, EV_CHORD, 0, 7)
    return -1;
}

}  // namespace vf
