// Streaming VDF / DDF kernels of the 7x7 window with the chord approximant
// evaluated by Estrin's scheme or with packed FP16 (instantiations and launcher).
// The occupancy forms are those of the Horner kernels: VDF held to two waves
// per SIMD, DDF unconstrained (see stream_kernel_w).
#include "kern_stream.h"

namespace vf {

template <int F, int NHI, int V>
static void launch_var7(const KParams& p, int blocks, void* stream) {
    if constexpr (F == VF_FILTER_VDF)
        stream_launch(stream_kernel_w<2, F, 7, EV_CHORD, 0, NHI, V>, p, blocks, stream);
    else
        stream_launch(stream_kernel<F, 7, EV_CHORD, 0, NHI, V>, p, blocks, stream);
}

#define VF_STREAM_VAR(F, NHI, V)                                                            \
    if (filter == F && eval == EV_CHORD && n_lo == 0 && n_hi == NHI && variant == V) {      \
        launch_var7<F, NHI, V>(p, blocks, stream);                                          \
        return (int)hipGetLastError();                                                       \
    }

int launch_angle_stream_var_w7(int filter, int eval, int n_lo, int n_hi, int variant, const KParams& p,
                                 int blocks, void* stream) {
    VF_STREAM_VAR(VF_FILTER_VDF, 4, VAR_ESTRIN)
    VF_STREAM_VAR(VF_FILTER_VDF, 4, VAR_F16)
    VF_STREAM_VAR(VF_FILTER_VDF, 5, VAR_ESTRIN)
    VF_STREAM_VAR(VF_FILTER_VDF, 5, VAR_F16)
    VF_STREAM_VAR(VF_FILTER_VDF, 6, VAR_ESTRIN)
    VF_STREAM_VAR(VF_FILTER_VDF, 6, VAR_F16)
    VF_STREAM_VAR(VF_FILTER_VDF, 7, VAR_ESTRIN)
    VF_STREAM_VAR(VF_FILTER_VDF, 7, VAR_F16)
    return -1;
}

}  // namespace vf
