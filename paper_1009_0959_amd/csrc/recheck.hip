// FP64 re-check kernel: one wavefront per flagged window, grid-stride over
// this call's re-check list (see recheck_dev.h for what is recomputed).
#include "batch.h"
#include "recheck_dev.h"

namespace vf {
namespace {

template <int FILT>
__global__ __launch_bounds__(64) void recheck_kernel(const KParams p, int eval, int window) {
    extern __shared__ double scratch[];
    if (blockIdx.x == 0 && threadIdx.x == 0) *p.next_count = 0u;
    const uint32_t count = min(*p.flag_count, p.flag_cap);
    for (uint32_t t = blockIdx.x; t < count; t += gridDim.x) {
        const uint32_t pix = p.flag_list[t];
        if (pix >= (uint32_t)p.H * (uint32_t)p.W) continue;   // (never listed by this call's kernel)
        const uint64_t mask = p.flag_mask ? p.flag_mask[t] : ~0ull;
        const int y = (int)(pix / (uint32_t)p.W);
        recheck_window<FILT>(p, rc_image(p), eval, window, y, (int)(pix - (uint32_t)y * (uint32_t)p.W), scratch,
                             threadIdx.x, mask);
    }
}

// VF_PREC_FP64: every window of the image evaluated in FP64 by the same
// window function (one wave per window, grid-stride over the pixels).
template <int FILT>
__global__ __launch_bounds__(64) void fp64_kernel(const KParams p, int eval, int window) {
    extern __shared__ double scratch[];
    const uint32_t total = (uint32_t)p.H * (uint32_t)p.W;
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        const int y = (int)(t / (uint32_t)p.W);
        recheck_window<FILT>(p, rc_image(p), eval, window, y, (int)(t - (uint32_t)y * (uint32_t)p.W), scratch, threadIdx.x);
    }
}

// One launch of K<FILT>::fn for the filter's instantiation, with the FP64
// window scratch in dynamic LDS.
template <template <int> class K, class... A>
int launch_by_filter(int filter, int window, int blocks, void* stream, A... args) {
    const int n = window * window;
    const size_t lds = (size_t)recheck_scratch_doubles(n, filter) * sizeof(double);
    hipStream_t s = (hipStream_t)stream;
    switch (filter) {
    case VF_FILTER_VDF: hipLaunchKernelGGL(K<VF_FILTER_VDF>::fn, dim3(blocks), dim3(64), lds, s, args...); break;
    case VF_FILTER_DDF: hipLaunchKernelGGL(K<VF_FILTER_DDF>::fn, dim3(blocks), dim3(64), lds, s, args...); break;
    case VF_FILTER_AMNFE: hipLaunchKernelGGL(K<VF_FILTER_AMNFE>::fn, dim3(blocks), dim3(64), lds, s, args...); break;
    case VF_FILTER_AMNFG: hipLaunchKernelGGL(K<VF_FILTER_AMNFG>::fn, dim3(blocks), dim3(64), lds, s, args...); break;
    default: hipLaunchKernelGGL(K<VF_FILTER_EVMF>::fn, dim3(blocks), dim3(64), lds, s, args...); break;
    }
    return (int)hipGetLastError();
}

template <int F>
struct Fp64K {
    static constexpr auto fn = fp64_kernel<F>;
};
template <int F>
struct RecheckK {
    static constexpr auto fn = recheck_kernel<F>;
};
template <int F>
struct RecheckBatchK {
    static constexpr auto fn = recheck_batch_kernel<F>;
};
template <int F>
struct OverflowBatchK {
    static constexpr auto fn = overflow_batch_kernel<F>;
};

}  // namespace

int launch_fp64(int filter, int eval, int window, const KParams& p, int blocks, void* stream) {
    return launch_by_filter<Fp64K>(filter, window, blocks, stream, p, eval, window);
}

int launch_recheck(int filter, int eval, int window, const KParams& p, int blocks, void* stream) {
    return launch_by_filter<RecheckK>(filter, window, blocks, stream, p, eval, window);
}

int launch_recheck_batch(int filter, int eval, int window, const BatchParams& bp, int blocks, void* stream) {
    return launch_by_filter<RecheckBatchK>(filter, window, blocks, stream, bp, eval, window);
}

int launch_overflow_batch(int filter, int eval, int window, const BatchParams& bp, uint32_t pixels, int blocks,
                          void* stream) {
    return launch_by_filter<OverflowBatchK>(filter, window, blocks, stream, bp, eval, window, pixels);
}

}  // namespace vf
