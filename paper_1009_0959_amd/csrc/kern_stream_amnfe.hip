// Streaming AMNF kernels (exact integer L1 pair sums; exponential or Gaussian
// kernel in the finisher): instantiations and launchers, single image and
// persistent batch (the tile function is in kern_stream.h).
#include "kern_stream.h"

namespace vf {

// 7x7 runs the two-waves-per-SIMD form (see stream_kernel_w)
template <int F, int W, int MODE>
static void launch_fe(const KParams& p, int blocks, void* stream) {
    if constexpr (W == 7)
        stream_launch(stream_kernel_w<2, F, W, MODE, 0, 0>, p, blocks, stream);
    else
        stream_launch(stream_kernel<F, W, MODE, 0, 0>, p, blocks, stream);
}

template <int F, int W, int MODE>
static int launch_fe_batch(bool probe, const BatchParams& bp, int num_cus, void* stream) {
    if constexpr (W == 7)
        return launch_persistent(probe, stream_batch_kernel_w<2, F, W, MODE, 0, 0>, 64, bp, num_cus, stream);
    else
        return launch_persistent(probe, stream_batch_kernel<F, W, MODE, 0, 0>, 64, bp, num_cus, stream);
}

template <int F>
static int launch_fe_any(int window, int eval, const KParams& p, int blocks, void* stream) {
#define VF_FE_STREAM(W, MODE)                                                                 \
    if (window == W && eval == MODE) {                                                        \
        launch_fe<F, W, MODE>(p, blocks, stream);                                             \
        return (int)hipGetLastError();                                                        \
    }
    VF_FE_STREAM(3, EV_EXACT)
    VF_FE_STREAM(3, EV_MINIMAX)
    VF_FE_STREAM(3, EV_PAPER)
    VF_FE_STREAM(5, EV_EXACT)
    VF_FE_STREAM(5, EV_MINIMAX)
    VF_FE_STREAM(5, EV_PAPER)
    VF_FE_STREAM(7, EV_EXACT)
    VF_FE_STREAM(7, EV_MINIMAX)
    VF_FE_STREAM(7, EV_PAPER)
#undef VF_FE_STREAM
    return -1;
}

template <int F>
static int launch_fe_batch_any(int window, int eval, const BatchParams& bp, int num_cus, void* stream, bool probe) {
#define VF_FE_BATCH(W, MODE) \
    if (window == W && eval == MODE) return launch_fe_batch<F, W, MODE>(probe, bp, num_cus, stream);
    VF_FE_BATCH(3, EV_EXACT)
    VF_FE_BATCH(3, EV_MINIMAX)
    VF_FE_BATCH(3, EV_PAPER)
    VF_FE_BATCH(5, EV_EXACT)
    VF_FE_BATCH(5, EV_MINIMAX)
    VF_FE_BATCH(5, EV_PAPER)
    VF_FE_BATCH(7, EV_EXACT)
    VF_FE_BATCH(7, EV_MINIMAX)
    VF_FE_BATCH(7, EV_PAPER)
#undef VF_FE_BATCH
    return -1;
}

int launch_amnfe_stream(int filter, int window, int eval, const KParams& p, int blocks, void* stream) {
    return filter == VF_FILTER_AMNFG ? launch_fe_any<VF_FILTER_AMNFG>(window, eval, p, blocks, stream)
                                     : launch_fe_any<VF_FILTER_AMNFE>(window, eval, p, blocks, stream);
}

// Persistent batch launch (see launch_persistent); -1 when no kernel matches.
int launch_amnfe_stream_batch(int filter, int window, int eval, const BatchParams& bp, int num_cus, void* stream,
                              bool probe) {
    return filter == VF_FILTER_AMNFG ? launch_fe_batch_any<VF_FILTER_AMNFG>(window, eval, bp, num_cus, stream, probe)
                                     : launch_fe_batch_any<VF_FILTER_AMNFE>(window, eval, bp, num_cus, stream, probe);
}

}  // namespace vf
