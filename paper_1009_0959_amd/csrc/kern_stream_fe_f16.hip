// Streaming AMNFE, AMNFG and EVMF kernels with the packed-FP16 evaluation of the
// minimax exp / ln1p correction (single image; the tile function and the
// finishers are in kern_stream.h). 7x7 runs the two-waves-per-SIMD form, as
// the FP32 kernels do.
#include "kern_stream.h"

namespace vf {

template <int F, int W>
static void launch_f16(const KParams& p, int blocks, void* stream) {
    if constexpr (W == 7)
        stream_launch(stream_kernel_w<2, F, W, EV_MINIMAX, 0, 0, VAR_F16>, p, blocks, stream);
    else
        stream_launch(stream_kernel<F, W, EV_MINIMAX, 0, 0, VAR_F16>, p, blocks, stream);
}

// Returns -1 when no kernel matches (the FP16 variant exists for the minimax
// approximants only).
int launch_fe_stream_f16(int filter, int window, int eval, const KParams& p, int blocks, void* stream) {
    if (eval != EV_MINIMAX) return -1;
    if (filter == VF_FILTER_AMNFE) {
        if (window == 3) launch_f16<VF_FILTER_AMNFE, 3>(p, blocks, stream);
        else if (window == 5) launch_f16<VF_FILTER_AMNFE, 5>(p, blocks, stream);
        else if (window == 7) launch_f16<VF_FILTER_AMNFE, 7>(p, blocks, stream);
        else return -1;
    } else if (filter == VF_FILTER_AMNFG) {
        if (window == 3) launch_f16<VF_FILTER_AMNFG, 3>(p, blocks, stream);
        else if (window == 5) launch_f16<VF_FILTER_AMNFG, 5>(p, blocks, stream);
        else if (window == 7) launch_f16<VF_FILTER_AMNFG, 7>(p, blocks, stream);
        else return -1;
    } else if (filter == VF_FILTER_EVMF) {
        if (window == 3) launch_f16<VF_FILTER_EVMF, 3>(p, blocks, stream);
        else if (window == 5) launch_f16<VF_FILTER_EVMF, 5>(p, blocks, stream);
        else if (window == 7) launch_f16<VF_FILTER_EVMF, 7>(p, blocks, stream);
        else return -1;
    } else {
        return -1;
    }
    return (int)hipGetLastError();
}

}  // namespace vf
