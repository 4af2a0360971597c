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
        recheck_window<FILT>(p, eval, window, y, (int)(pix - (uint32_t)y * (uint32_t)p.W), scratch,
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
        recheck_window<FILT>(p, eval, window, y, (int)(t - (uint32_t)y * (uint32_t)p.W), scratch, threadIdx.x);
    }
}

}  // namespace

int launch_fp64(int filter, int eval, int window, const KParams& p, int blocks, void* stream) {
    const int n = window * window;
    const size_t lds = (size_t)recheck_scratch_doubles(n, filter == VF_FILTER_DDF) * sizeof(double);
    hipStream_t s = (hipStream_t)stream;
    switch (filter) {
    case VF_FILTER_VDF:
        hipLaunchKernelGGL(fp64_kernel<VF_FILTER_VDF>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    case VF_FILTER_DDF:
        hipLaunchKernelGGL(fp64_kernel<VF_FILTER_DDF>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    case VF_FILTER_AMNFE:
        hipLaunchKernelGGL(fp64_kernel<VF_FILTER_AMNFE>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    case VF_FILTER_AMNFG:
        hipLaunchKernelGGL(fp64_kernel<VF_FILTER_AMNFG>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    default:
        hipLaunchKernelGGL(fp64_kernel<VF_FILTER_EVMF>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    }
    return (int)hipGetLastError();
}

int launch_recheck(int filter, int eval, int window, const KParams& p, int blocks, void* stream) {
    const int n = window * window;
    const size_t lds = (size_t)recheck_scratch_doubles(n, filter == VF_FILTER_DDF) * sizeof(double);
    hipStream_t s = (hipStream_t)stream;
    switch (filter) {
    case VF_FILTER_VDF:
        hipLaunchKernelGGL(recheck_kernel<VF_FILTER_VDF>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    case VF_FILTER_DDF:
        hipLaunchKernelGGL(recheck_kernel<VF_FILTER_DDF>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    case VF_FILTER_AMNFE:
        hipLaunchKernelGGL(recheck_kernel<VF_FILTER_AMNFE>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    case VF_FILTER_AMNFG:
        hipLaunchKernelGGL(recheck_kernel<VF_FILTER_AMNFG>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    default:
        hipLaunchKernelGGL(recheck_kernel<VF_FILTER_EVMF>, dim3(blocks), dim3(64), lds, s, p, eval, window);
        break;
    }
    return (int)hipGetLastError();
}

int launch_recheck_batch(int filter, int eval, int window, const BatchParams& bp, int blocks, void* stream) {
    const int n = window * window;
    const size_t lds = (size_t)recheck_scratch_doubles(n, filter == VF_FILTER_DDF) * sizeof(double);
    hipStream_t s = (hipStream_t)stream;
    switch (filter) {
    case VF_FILTER_VDF:
        hipLaunchKernelGGL(recheck_batch_kernel<VF_FILTER_VDF>, dim3(blocks), dim3(64), lds, s, bp, eval, window);
        break;
    case VF_FILTER_DDF:
        hipLaunchKernelGGL(recheck_batch_kernel<VF_FILTER_DDF>, dim3(blocks), dim3(64), lds, s, bp, eval, window);
        break;
    case VF_FILTER_AMNFE:
        hipLaunchKernelGGL(recheck_batch_kernel<VF_FILTER_AMNFE>, dim3(blocks), dim3(64), lds, s, bp, eval,
                           window);
        break;
    case VF_FILTER_AMNFG:
        hipLaunchKernelGGL(recheck_batch_kernel<VF_FILTER_AMNFG>, dim3(blocks), dim3(64), lds, s, bp, eval,
                           window);
        break;
    default:
        hipLaunchKernelGGL(recheck_batch_kernel<VF_FILTER_EVMF>, dim3(blocks), dim3(64), lds, s, bp, eval, window);
        break;
    }
    return (int)hipGetLastError();
}

}  // namespace vf
