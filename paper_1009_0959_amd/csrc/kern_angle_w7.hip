// VDF / DDF window kernels for the 7x7 window (instantiations and launcher).
#include "kern_angle.h"
#include "kern_stream_split.h"
#include "batch.h"

namespace vf {

#define VF_ANGLE_CASE(F, MODE, NLO, NHI)                                                   \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI) {                       \
        hipLaunchKernelGGL((angle_kernel<F, 7, MODE, NLO, NHI>), dim3(blocks), dim3(kTileX * angle_tile_y<7>()), \
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

int launch_angle_w7(int filter, int eval, int n_lo, int n_hi, const KParams& p, int blocks,
                    void* stream) {
    VF_ANGLE_MODES(VF_FILTER_VDF)
    VF_ANGLE_MODES(VF_FILTER_DDF)
    return -1;
}

// Streaming 7x7 kernels. The exact-acosf modes sum two (VDF) or three (DDF)
// quantities per member; they, and the DDF modes without a single-wave
// kernel, split each window's state over several waves of a workgroup
// (kern_stream_split.h): the single-wave form needed 512 registers and
// spilled (8192^2 16-bit image: exact VDF 29.6 -> 21.6 ms, exact DDF 81.0 ->
// 40.3 ms; split-approximant DDF 32.0 ms against 120.8 ms in the per-window
// kernel). The approximant VDF and the chord DDF keep the single-wave form,
// at one wave per SIMD (512 registers with AGPRs): held to two waves per SIMD
// the VDF kernel spilled 340 B per lane, about 40 GB of scratch traffic per
// 8192^2 launch, for the same time (10.1 ms). Split over 3, 4 or 7 waves they
// measured slower (VDF 8.7 ms single-wave against 14.9 - 18.3 ms, chord DDF
// 25.4 against 30.3 ms), the barriers and the doubled LDS reads of the fold
// costing more than the spills saved.
template <int F, int MODE>
constexpr int stream7_waves() {
    if (MODE == EV_EXACT) return F == VF_FILTER_DDF ? 7 : 4;
    if (F == VF_FILTER_DDF && MODE != EV_CHORD) return 7;
    return 1;
}

template <int F, int MODE, int NLO, int NHI>
static void launch_stream7(const KParams& p, int blocks, void* stream) {
    constexpr int NW = stream7_waves<F, MODE>();
    if constexpr (NW > 1)
        stream_split_launch<NW>(stream_split_kernel<NW, F, 7, MODE, NLO, NHI>, p, blocks, stream);
    else
        stream_launch(stream_kernel<F, 7, MODE, NLO, NHI>, p, blocks, stream);
}

#define VF_STREAM_CASE(F, MODE, NLO, NHI)                                                   \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI) {                        \
        launch_stream7<F, MODE, NLO, NHI>(p, blocks, stream);                               \
        return (int)hipGetLastError();                                                      \
    }

int launch_angle_stream_w7(int filter, int eval, int n_lo, int n_hi, const KParams& p, int blocks,
                            void* stream) {
    VF_STREAM_CASE(VF_FILTER_VDF, EV_EXACT, 0, 0)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_PAPER, 5, 5)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_SPLIT, 2, 2)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_SPLIT, 3, 3)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_SPLIT, 4, 4)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_SPLIT, 5, 5)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_CHORD, 0, 4)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_CHORD, 0, 5)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_CHORD, 0, 6)
    VF_STREAM_CASE(VF_FILTER_VDF, EV_CHORD, 0, 7)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_EXACT, 0, 0)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_PAPER, 5, 5)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_SPLIT, 2, 2)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_SPLIT, 3, 3)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_SPLIT, 4, 4)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_SPLIT, 5, 5)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_CHORD, 0, 4)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_CHORD, 0, 5)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_CHORD, 0, 6)
    VF_STREAM_CASE(VF_FILTER_DDF, EV_CHORD, 0, 7)
    return -1;
}

template <int FILT, int WIN, int MODE, int NLO, int NHI>
__global__ __launch_bounds__(kTileX * angle_tile_y<WIN>()) void angle_batch_kernel(const BatchParams bp) {
    batch_loop(bp, [&](const KParams& p, int tile) { angle_tile<FILT, WIN, MODE, NLO, NHI>(p, tile); });
}



#define VF_BATCH_DIRECT(F, MODE, NLO, NHI)                                                     \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI && !streaming)                \
        return launch_persistent(probe, angle_batch_kernel<F, 7, MODE, NLO, NHI>,                         \
                                 kTileX * angle_tile_y<7>(), bp, num_cus, stream);

template <int F, int MODE, int NLO, int NHI>
static int launch_stream7_batch(bool probe, const BatchParams& bp, int num_cus, void* stream) {
    constexpr int NW = stream7_waves<F, MODE>();
    if constexpr (NW > 1)
        return launch_persistent(probe, stream_split_batch_kernel<NW, F, 7, MODE, NLO, NHI>, 64 * NW, bp, num_cus,
                                 stream);
    else
        return launch_persistent(probe, stream_batch_kernel<F, 7, MODE, NLO, NHI>, 64, bp, num_cus, stream);
}

#define VF_BATCH_STREAM(F, MODE, NLO, NHI)                                                     \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI && streaming)                 \
        return launch_stream7_batch<F, MODE, NLO, NHI>(probe, bp, num_cus, stream);

// Persistent batch launch. Returns -1 when no kernel matches (the streaming
// combinations are those of the single-image streaming launcher); with
// `probe` set it only reports whether one does (0) and launches nothing.
int launch_angle_batch_w7(int filter, int eval, int n_lo, int n_hi, bool streaming, const BatchParams& bp,
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
