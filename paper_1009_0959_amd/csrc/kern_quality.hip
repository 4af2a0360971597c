// Quality criteria of an original image X against a filtered image Y
// (Section 4): MAE and MSE from exact integer sums of |x - y|_1 and
// |x - y|_2^2, NCD from FP64 sums of |x^Lab - y^Lab|_2 and |x^Lab|_2.
//
// CIELAB reading: 8/16-bit values are sRGB scaled to [0, 1] by the type's
// maximum, decoded with the sRGB transfer function, taken to CIE XYZ by the
// sRGB primaries' matrix (four-digit form) and to L*a*b* relative to the
// white that matrix gives the RGB white (its row sums), so white is
// (100, 0, 0); f(t) = t^(1/3) above (6/29)^3, else t (29/6)^2 / 3 + 4/29.
//
// One pass over both images (HBM: 6 or 12 bytes per pixel); each thread
// keeps its four sums, a workgroup folds them in a fixed order, and a second
// single-workgroup kernel folds the workgroup partials in a fixed order, so
// a result depends only on the image and the grid (never on timing).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vf_internal.h"

namespace vf {
namespace {

constexpr int kQThreads = 256;

__device__ __forceinline__ double srgb_linear(double c) {
    return c <= 0.04045 ? c / 12.92 : pow((c + 0.055) / 1.055, 2.4);
}

__device__ __forceinline__ double lab_f(double t) {
    constexpr double eps = (6.0 / 29.0) * (6.0 / 29.0) * (6.0 / 29.0);
    return t > eps ? cbrt(t) : t * ((29.0 / 6.0) * (29.0 / 6.0) / 3.0) + 4.0 / 29.0;
}

// L*, a*, b* of one pixel from its linear RGB
__device__ __forceinline__ void lab_of(double r, double g, double b, double& L, double& A, double& B) {
    constexpr double wx = 0.4124 + 0.3576 + 0.1805, wy = 0.2126 + 0.7152 + 0.0722, wz = 0.0193 + 0.1192 + 0.9505;
    const double X = 0.4124 * r + 0.3576 * g + 0.1805 * b;
    const double Y = 0.2126 * r + 0.7152 * g + 0.0722 * b;
    const double Z = 0.0193 * r + 0.1192 * g + 0.9505 * b;
    const double fx = lab_f(X / wx), fy = lab_f(Y / wy), fz = lab_f(Z / wz);
    L = 116.0 * fy - 16.0;
    A = 500.0 * (fx - fy);
    B = 200.0 * (fy - fz);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// fold one thread's sums over the workgroup (fixed order) into out
__device__ __forceinline__ void block_fold(QualPartial q, QualPartial* out) {
    __shared__ QualPartial s[kQThreads / 64];
    q.l1 = wave_sum(q.l1);
    q.l2sq = wave_sum(q.l2sq);
    q.lab_diff = wave_sum(q.lab_diff);
    q.lab_ref = wave_sum(q.lab_ref);
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) s[wave] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        QualPartial r = s[0];
        for (int w = 1; w < kQThreads / 64; ++w) {
            r.l1 += s[w].l1;
            r.l2sq += s[w].l2sq;
            r.lab_diff += s[w].lab_diff;
            r.lab_ref += s[w].lab_ref;
        }
        *out = r;
    }
}

template <bool U16>
__global__ __launch_bounds__(kQThreads) void quality_partial_kernel(const unsigned char* x, int64_t x_pitch,
                                                                   const unsigned char* y, int64_t y_pitch, int H,
                                                                   int W, QualPartial* parts) {
    // 8-bit values: the 256 decoded levels once per workgroup
    __shared__ double s_lin[U16 ? 1 : 256];
    if constexpr (!U16) {
        s_lin[threadIdx.x] = srgb_linear((double)threadIdx.x / 255.0);
        __syncthreads();
    }
    auto lin = [&](uint32_t v) -> double {
        if constexpr (U16) return srgb_linear((double)v / 65535.0);
        else return s_lin[v];
    };
    QualPartial q{0ull, 0ull, 0.0, 0.0};
    const uint64_t total = (uint64_t)H * (uint64_t)W;
    const uint64_t stride = (uint64_t)gridDim.x * kQThreads;
    for (uint64_t t = (uint64_t)blockIdx.x * kQThreads + threadIdx.x; t < total; t += stride) {
        const uint32_t r = (uint32_t)(t / (uint64_t)W);
        const uint32_t c = (uint32_t)(t - (uint64_t)r * (uint64_t)W);
        uint32_t a[3], b[3];
        if constexpr (U16) {
            const uint16_t* px = reinterpret_cast<const uint16_t*>(x + (int64_t)r * x_pitch) + 3 * c;
            const uint16_t* py = reinterpret_cast<const uint16_t*>(y + (int64_t)r * y_pitch) + 3 * c;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                a[k] = px[k];
                b[k] = py[k];
            }
        } else {
            const unsigned char* px = x + (int64_t)r * x_pitch + 3 * c;
            const unsigned char* py = y + (int64_t)r * y_pitch + 3 * c;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                a[k] = px[k];
                b[k] = py[k];
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t d = (int64_t)a[k] - (int64_t)b[k];
            q.l1 += (unsigned long long)(d < 0 ? -d : d);
            q.l2sq += (unsigned long long)(d * d);
        }
        double La, Aa, Ba, Lb, Ab, Bb;
        lab_of(lin(a[0]), lin(a[1]), lin(a[2]), La, Aa, Ba);
        if (a[0] == b[0] && a[1] == b[1] && a[2] == b[2]) {
            Lb = La;
            Ab = Aa;
            Bb = Ba;
        } else {
            lab_of(lin(b[0]), lin(b[1]), lin(b[2]), Lb, Ab, Bb);
        }
        const double dL = La - Lb, dA = Aa - Ab, dB = Ba - Bb;
        q.lab_diff += sqrt(dL * dL + dA * dA + dB * dB);
        q.lab_ref += sqrt(La * La + Aa * Aa + Ba * Ba);
    }
    block_fold(q, &parts[blockIdx.x]);
}

__global__ __launch_bounds__(kQThreads) void quality_final_kernel(const QualPartial* parts, int n,
                                                                 QualPartial* out) {
    QualPartial q{0ull, 0ull, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += kQThreads) {
        q.l1 += parts[i].l1;
        q.l2sq += parts[i].l2sq;
        q.lab_diff += parts[i].lab_diff;
        q.lab_ref += parts[i].lab_ref;
    }
    block_fold(q, out);
}

}  // namespace

int launch_quality(const unsigned char* x, int64_t x_pitch, const unsigned char* y, int64_t y_pitch, int H, int W,
                   bool u16, int blocks, void* parts, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    QualPartial* p = static_cast<QualPartial*>(parts);
    if (u16)
        hipLaunchKernelGGL(quality_partial_kernel<true>, dim3(blocks), dim3(kQThreads), 0, s, x, x_pitch, y, y_pitch,
                           H, W, p);
    else
        hipLaunchKernelGGL(quality_partial_kernel<false>, dim3(blocks), dim3(kQThreads), 0, s, x, x_pitch, y,
                           y_pitch, H, W, p);
    hipLaunchKernelGGL(quality_final_kernel, dim3(1), dim3(kQThreads), 0, s, p, blocks, p + blocks);
    return (int)hipGetLastError();
}

}  // namespace vf
