// Elementwise evaluation of the filters' elementary functions, using the very
// device functions the window kernels inline (for function-error measurements).
#include "kern_common.h"

namespace vf {

template <int MODE, int NLO, int NHI>
__global__ void eval_angle_kernel(const KParams p, const float* in, float* out, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = angle_from_s2<MODE, NLO, NHI>(in[i], p.lo, p.hi);
}

template <int MODE>
__global__ void eval_exp_kernel(const KParams p, const float* in, float* out, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = kernel_exp<MODE>(in[i], p.lo, p.n_lo, p.hi, p.n_hi, p.cutoff);
}

template <int MODE>
__global__ void eval_ent_kernel(const KParams p, const float* in, float* out, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = ent<MODE>(in[i], p.lo, p.n_lo, p.hi, p.n_hi, p.cutoff);
}

// Packed-FP16 variants of exp (AMNFE, AMNFG) and ENT (EVMF): two inputs per thread,
// the same arithmetic as the streaming finishers.
template <int FILT>
__global__ void eval_fe_f16_kernel(const KParams p, const float* in, float* out, int64_t count) {
    const half2_t* h = reinterpret_cast<const half2_t*>(p.lo16);
    const int64_t pairs = (count + 1) / 2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < pairs;
         i += (int64_t)gridDim.x * blockDim.x) {
        const bool two = 2 * i + 1 < count;
        const float a = in[2 * i], b = two ? in[2 * i + 1] : 0.0f;
        float ra, rb;
        if constexpr (FILT == VF_FILTER_AMNFE) {
            const float2 t = corr_pair_f16<0>(a, b, h, p.n_lo);
            ra = a > p.cutoff ? 0.0f : p.lo[0] + t.x;
            rb = b > p.cutoff ? 0.0f : p.lo[0] + t.y;
        } else {
            int xa, xb;
            const float ta = fmaf(frexpf(a, &xa), 2.0f, -1.0f);
            const float tb = fmaf(frexpf(b, &xb), 2.0f, -1.0f);
            const float2 c = corr_pair_f16<0>(ta, tb, h, p.n_lo);
            ra = a > 0.0f ? a * fmaf((float)(xa - 1), kLn2, p.lo[0] + c.x) : 0.0f;
            rb = b > 0.0f ? b * fmaf((float)(xb - 1), kLn2, p.lo[0] + c.y) : 0.0f;
        }
        out[2 * i] = ra;
        if (two) out[2 * i + 1] = rb;
    }
}

int launch_eval_function(int filter, int eval, int n_lo, int n_hi, int variant, const KParams& p,
                         const float* in, float* out, int64_t count, void* stream) {
    const int blocks = (int)((count + 255) / 256 < 4096 ? (count + 255) / 256 : 4096);
    const int nb = blocks > 0 ? blocks : 1;
    hipStream_t s = (hipStream_t)stream;
    if (variant == 2 && is_amnf(filter)) {
        hipLaunchKernelGGL((eval_fe_f16_kernel<VF_FILTER_AMNFE>), dim3(nb), dim3(256), 0, s, p, in, out, count);
        return (int)hipGetLastError();
    }
    if (variant == 2 && filter == VF_FILTER_EVMF) {
        hipLaunchKernelGGL((eval_fe_f16_kernel<VF_FILTER_EVMF>), dim3(nb), dim3(256), 0, s, p, in, out, count);
        return (int)hipGetLastError();
    }
#define VF_EVAL_ANGLE(MODE, NLO, NHI)                                                       \
    if (eval == MODE && n_lo == NLO && n_hi == NHI) {                                       \
        hipLaunchKernelGGL((eval_angle_kernel<MODE, NLO, NHI>), dim3(nb), dim3(256), 0, s, p, \
                           in, out, count);                                                 \
        return (int)hipGetLastError();                                                      \
    }
    if (filter == VF_FILTER_VDF || filter == VF_FILTER_DDF) {
        VF_EVAL_ANGLE(EV_EXACT, 0, 0)
        VF_EVAL_ANGLE(EV_PAPER, 5, 5)
        VF_EVAL_ANGLE(EV_SPLIT, 2, 2)
        VF_EVAL_ANGLE(EV_SPLIT, 3, 3)
        VF_EVAL_ANGLE(EV_SPLIT, 4, 4)
        VF_EVAL_ANGLE(EV_SPLIT, 5, 5)
        VF_EVAL_ANGLE(EV_CHORD, 0, 4)
        VF_EVAL_ANGLE(EV_CHORD, 0, 5)
        VF_EVAL_ANGLE(EV_CHORD, 0, 6)
        VF_EVAL_ANGLE(EV_CHORD, 0, 7)
        return -1;
    }
#undef VF_EVAL_ANGLE
    if (is_amnf(filter)) {
        if (eval == EV_EXACT)
            hipLaunchKernelGGL((eval_exp_kernel<EV_EXACT>), dim3(nb), dim3(256), 0, s, p, in, out, count);
        else if (eval == VF_EVAL_RATIONAL || eval == VF_EVAL_RATFIT)
            hipLaunchKernelGGL((eval_exp_kernel<EV_PAPER>), dim3(nb), dim3(256), 0, s, p, in, out, count);
        else
            hipLaunchKernelGGL((eval_exp_kernel<EV_MINIMAX>), dim3(nb), dim3(256), 0, s, p, in, out, count);
        return (int)hipGetLastError();
    }
    if (eval == EV_EXACT)
        hipLaunchKernelGGL((eval_ent_kernel<EV_EXACT>), dim3(nb), dim3(256), 0, s, p, in, out, count);
    else if (eval == EV_PAPER)
        hipLaunchKernelGGL((eval_ent_kernel<EV_PAPER>), dim3(nb), dim3(256), 0, s, p, in, out, count);
    else
        hipLaunchKernelGGL((eval_ent_kernel<EV_MINIMAX>), dim3(nb), dim3(256), 0, s, p, in, out, count);
    return (int)hipGetLastError();
}

// Zero n words with ordinary vector stores (used in captured graphs, where a
// memset node is avoided).
__global__ void fill_u32_kernel(uint32_t* p, uint32_t n, uint32_t v) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

int launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, void* stream) {
    const uint32_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(nb < 1 ? 1 : (nb > 1024 ? 1024 : nb)), dim3(256), 0,
                       (hipStream_t)stream, p, n, v);
    return (int)hipGetLastError();
}

}  // namespace vf
