// AMNFE window kernel: instantiations and launcher (kernel in kern_amnfe.h).
#include "batch.h"
#include "kern_amnfe.h"

namespace vf {

#define VF_AMNFE_CASE(W, MODE)                                                             \
    if (window == W && eval == MODE) {                                                     \
        hipLaunchKernelGGL((amnfe_kernel<W, MODE>), dim3(blocks), dim3(kThreads), 0,       \
                           (hipStream_t)stream, p);                                        \
        return (int)hipGetLastError();                                                     \
    }

int launch_amnfe(int window, int eval, const KParams& p, int blocks, void* stream) {
    VF_AMNFE_CASE(3, EV_EXACT)
    VF_AMNFE_CASE(3, EV_MINIMAX)
    VF_AMNFE_CASE(3, EV_PAPER)
    VF_AMNFE_CASE(5, EV_EXACT)
    VF_AMNFE_CASE(5, EV_MINIMAX)
    VF_AMNFE_CASE(5, EV_PAPER)
    VF_AMNFE_CASE(7, EV_EXACT)
    VF_AMNFE_CASE(7, EV_MINIMAX)
    VF_AMNFE_CASE(7, EV_PAPER)
    return -1;
}

template <int WIN, int MODE>
__global__ __launch_bounds__(kThreads) void amnfe_batch_kernel(const BatchParams bp) {
    batch_loop(bp, [&](const KParams& p, int tile) { amnfe_tile<WIN, MODE>(p, tile); });
}

#define VF_AMNFE_BATCH(W, MODE)                                                            \
    if (window == W && eval == MODE)                                                       \
        return launch_persistent(probe, amnfe_batch_kernel<W, MODE>, kThreads, bp, num_cus, stream);

// Persistent batch launch (see launch_persistent); -1 when no kernel matches.
int launch_amnfe_batch(int window, int eval, const BatchParams& bp, int num_cus, void* stream, bool probe) {
    VF_AMNFE_BATCH(3, EV_EXACT)
    VF_AMNFE_BATCH(3, EV_MINIMAX)
    VF_AMNFE_BATCH(3, EV_PAPER)
    VF_AMNFE_BATCH(5, EV_EXACT)
    VF_AMNFE_BATCH(5, EV_MINIMAX)
    VF_AMNFE_BATCH(5, EV_PAPER)
    VF_AMNFE_BATCH(7, EV_EXACT)
    VF_AMNFE_BATCH(7, EV_MINIMAX)
    VF_AMNFE_BATCH(7, EV_PAPER)
    return -1;
}

}  // namespace vf
