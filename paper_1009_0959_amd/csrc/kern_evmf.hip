// EVMF window kernel: instantiations and launcher (kernel in kern_evmf.h).
#include "batch.h"
#include "kern_evmf.h"

namespace vf {

#define VF_EVMF_CASE(W, MODE)                                                              \
    if (window == W && eval == MODE) {                                                     \
        hipLaunchKernelGGL((evmf_kernel<W, MODE>), dim3(blocks), dim3(kThreads), 0,        \
                           (hipStream_t)stream, p);                                        \
        return (int)hipGetLastError();                                                     \
    }

int launch_evmf(int window, int eval, const KParams& p, int blocks, void* stream) {
    VF_EVMF_CASE(3, EV_EXACT)
    VF_EVMF_CASE(3, EV_PAPER)
    VF_EVMF_CASE(3, EV_MINIMAX)
    VF_EVMF_CASE(5, EV_EXACT)
    VF_EVMF_CASE(5, EV_PAPER)
    VF_EVMF_CASE(5, EV_MINIMAX)
    VF_EVMF_CASE(7, EV_EXACT)
    VF_EVMF_CASE(7, EV_PAPER)
    VF_EVMF_CASE(7, EV_MINIMAX)
    return -1;
}

template <int WIN, int MODE>
__global__ __launch_bounds__(kThreads) void evmf_batch_kernel(const BatchParams bp) {
    batch_loop(bp, [&](const KParams& p, int tile) { evmf_tile<WIN, MODE>(p, tile); });
}

#define VF_EVMF_BATCH(W, MODE)                                                             \
    if (window == W && eval == MODE)                                                       \
        return launch_persistent(probe, evmf_batch_kernel<W, MODE>, kThreads, bp, num_cus, stream);

// Persistent batch launch (see launch_persistent); -1 when no kernel matches.
int launch_evmf_batch(int window, int eval, const BatchParams& bp, int num_cus, void* stream, bool probe) {
    VF_EVMF_BATCH(3, EV_EXACT)
    VF_EVMF_BATCH(3, EV_PAPER)
    VF_EVMF_BATCH(3, EV_MINIMAX)
    VF_EVMF_BATCH(5, EV_EXACT)
    VF_EVMF_BATCH(5, EV_PAPER)
    VF_EVMF_BATCH(5, EV_MINIMAX)
    VF_EVMF_BATCH(7, EV_EXACT)
    VF_EVMF_BATCH(7, EV_PAPER)
    VF_EVMF_BATCH(7, EV_MINIMAX)
    return -1;
}

}  // namespace vf
