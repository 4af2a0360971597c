// VDF / DDF window kernels for the 3x3 window (instantiations and launcher).
#include "kern_angle.h"
#include "kern_stream.h"

namespace vf {

#define VF_ANGLE_CASE(F, MODE, NLO, NHI)                                                   \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI) {                       \
        hipLaunchKernelGGL((angle_kernel<F, 3, MODE, NLO, NHI>), dim3(blocks), dim3(kTileX * angle_tile_y<3>()), \
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

int launch_angle_w3(int filter, int eval, int n_lo, int n_hi, const KParams& p, int blocks,
                    void* stream) {
    VF_ANGLE_MODES(VF_FILTER_VDF)
    VF_ANGLE_MODES(VF_FILTER_DDF)
    return -1;
}

#define VF_STREAM_CASE(F, MODE, NLO, NHI)                                                   \
    if (filter == F && eval == MODE && n_lo == NLO && n_hi == NHI) {                        \
        hipLaunchKernelGGL((angle_stream_kernel<F, 3, MODE, NLO, NHI>), dim3(blocks), dim3(64), \
                           0, (hipStream_t)stream, p);                                      \
        return (int)hipGetLastError();                                                      \
    }

int launch_angle_stream_w3(int filter, int eval, int n_lo, int n_hi, const KParams& p, int blocks,
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

}  // namespace vf
