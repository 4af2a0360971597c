// FP64 re-check of flagged windows.
//
// The FP32 window kernels append every window whose decision lies within its
// FP32 error bound (two best criteria of distinct vectors too close, an EVMF
// switching test too close to zero, an AMNFE channel too close to a rounding
// boundary, or a zero vector mixed with non-zero ones). This kernel recomputes
// those windows from the definitions in double precision -- the same
// approximant, its FP32 constants widened exactly to double -- and overwrites
// their outputs. Operations are written out one rounding at a time (no fused
// multiply-add: this file is compiled with -ffp-contract=off).
//
// Definitions (paper, Section 3): window members row-major, borders
// replicated; VDF sums of A(x_i, x_j) = acos(cosine) over all j; DDF
// (sum |x_i - x_j|_2)^(1-p) (sum A)^p; AMNFE weighted mean with
// h_i = n^(-kappa/3) sum_j |x_i - x_j|_1, K = exp(-z) (0 above the cutoff);
// EVMF switching test P_C H > -ENT(P_C) and the vector median. Ties: centre
// first, then the lowest index. Cosine conventions: identical, collinear or
// both-zero vectors 1; one zero vector 0.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "vf_internal.h"

#pragma clang fp contract(off)

namespace vf {
namespace {

constexpr int kMaxN = 49;

__device__ double horner64(const double* c, int n, double x) {
    double acc = c[n - 1];
    for (int k = n - 2; k >= 0; --k) acc = acc * x + c[k];
    return acc;
}

__device__ void fetch(const RParams& p, int y, int x, int64_t v[3]) {
    y = y < 0 ? 0 : (y >= p.H ? p.H - 1 : y);
    x = x < 0 ? 0 : (x >= p.W ? p.W - 1 : x);
    const unsigned char* row = p.src + (int64_t)y * p.src_pitch;
    for (int k = 0; k < 3; ++k)
        v[k] = p.u16 ? (int64_t)reinterpret_cast<const uint16_t*>(row)[3 * x + k]
                     : (int64_t)row[3 * x + k];
}

__device__ double cosine64(const int64_t* a, const int64_t* b) {
    const int64_t na = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    const int64_t nb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    if (na == 0 && nb == 0) return 1.0;
    if (na == 0 || nb == 0) return 0.0;
    const int64_t c0 = a[1] * b[2] - a[2] * b[1];
    const int64_t c1 = a[2] * b[0] - a[0] * b[2];
    const int64_t c2 = a[0] * b[1] - a[1] * b[0];
    if (c0 == 0 && c1 == 0 && c2 == 0) return 1.0;
    const double dot = (double)(a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
    double z = dot / (sqrt((double)na) * sqrt((double)nb));
    if (z > 1.0) z = 1.0;
    if (z < -1.0) z = -1.0;
    return z;
}

__device__ double angle64(const RParams& p, double z) {
    switch (p.eval) {
    case EV_EXACT:
        return acos(z);
    case EV_PAPER:
        if (z < 0.5) return horner64(p.lo, p.n_lo, z);
        return horner64(p.hi, p.n_hi, sqrt(1.0 - z));
    case EV_SPLIT:
        if (z >= 0.5) {
            const double s = sqrt(2.0 * (1.0 - z));
            return s * horner64(p.hi, p.n_hi, s * s);
        }
        if (z <= -0.5) {
            const double s = sqrt(2.0 * (1.0 + z));
            return M_PI - s * horner64(p.hi, p.n_hi, s * s);
        }
        return M_PI / 2.0 - z * horner64(p.lo, p.n_lo, z * z);
    default: {   // EV_CHORD: one odd chord polynomial, mirrored for z < 0
        if (z >= 0.0) {
            const double s = sqrt(2.0 * (1.0 - z));
            return s * horner64(p.hi, p.n_hi, s * s);
        }
        const double s = sqrt(2.0 * (1.0 + z));
        return M_PI - s * horner64(p.hi, p.n_hi, s * s);
    }
    }
}

__device__ double dist_l2(const int64_t* a, const int64_t* b) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double d = (double)(a[k] - b[k]);
        s += d * d;
    }
    return sqrt(s);
}

__device__ int64_t dist_l1(const int64_t* a, const int64_t* b) {
    int64_t s = 0;
    for (int k = 0; k < 3; ++k) {
        const int64_t d = a[k] - b[k];
        s += d < 0 ? -d : d;
    }
    return s;
}

__device__ int argmin_tie(const double* s, int n) {
    int best = (n - 1) / 2;
    for (int i = 0; i < n; ++i)
        if (s[i] < s[best]) best = i;
    return best;
}

__device__ double ent64(const RParams& p, double z) {
    if (z <= 0.0) return 0.0;
    switch (p.eval) {
    case EV_EXACT:
        return z * log(z);
    case EV_PAPER:
        if (z < p.cutoff) return 0.0;
        return horner64(p.lo, p.n_lo, z) / horner64(p.hi, p.n_hi, z);
    default: {
        int e;
        double m = frexp(z, &e);
        m *= 2.0;
        e -= 1;
        return z * ((double)e * M_LN2 + horner64(p.lo, p.n_lo, m - 1.0));
    }
    }
}

__device__ void recheck_one(const RParams& p, uint32_t pix) {
    const int y = (int)(pix / (uint32_t)p.W);
    const int x = (int)(pix - (uint32_t)y * (uint32_t)p.W);
    const int w = p.window, r = (w - 1) / 2, n = w * w, C = (n - 1) / 2;
    int64_t v[kMaxN][3];
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) fetch(p, y + dy, x + dx, v[(dy + r) * w + (dx + r)]);
    double S[kMaxN];
    int sel = C;
    int64_t outv[3] = {v[C][0], v[C][1], v[C][2]};
    if (p.filter == VF_FILTER_VDF || p.filter == VF_FILTER_DDF) {
        for (int i = 0; i < n; ++i) {
            double a = 0.0, d = 0.0;
            for (int j = 0; j < n; ++j) {
                a += angle64(p, cosine64(v[i], v[j]));
                if (p.filter == VF_FILTER_DDF) d += dist_l2(v[i], v[j]);
            }
            S[i] = (p.filter == VF_FILTER_DDF) ? pow(d, 1.0 - p.param) * pow(a, p.param) : a;
        }
        sel = argmin_tie(S, n);
        for (int k = 0; k < 3; ++k) outv[k] = v[sel][k];
    } else if (p.filter == VF_FILTER_AMNFE) {
        int64_t S1[kMaxN];
        bool uniform = false;
        for (int i = 0; i < n; ++i) {
            int64_t acc = 0;
            for (int j = 0; j < n; ++j) acc += dist_l1(v[i], v[j]);
            S1[i] = acc;
            uniform |= (acc == 0);
        }
        if (!uniform) {
            double num[3] = {0.0, 0.0, 0.0}, den = 0.0;
            for (int i = 0; i < n; ++i) {
                const double h = p.scale * (double)S1[i];
                const double z = (double)dist_l1(v[C], v[i]) / h;
                double k;
                if (z > p.cutoff) k = 0.0;
                else if (p.eval == EV_EXACT) k = exp(-z);
                else k = horner64(p.lo, p.n_lo, z);
                const double wgt = k / (h * h * h);
                den += wgt;
                for (int c = 0; c < 3; ++c) num[c] += wgt * (double)v[i][c];
            }
            if (den > 0.0) {
                const int64_t maxv = p.u16 ? 65535 : 255;
                for (int c = 0; c < 3; ++c) {
                    double q = floor(num[c] / den + 0.5);
                    if (q < 0.0) q = 0.0;
                    if (q > (double)maxv) q = (double)maxv;
                    outv[c] = (int64_t)q;
                }
            }
        }
    } else {   // EVMF
        double mean[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) mean[k] += (double)v[i][k];
        for (int k = 0; k < 3; ++k) mean[k] /= (double)n;
        double d[kMaxN], D = 0.0;
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double t = (double)v[i][k] - mean[k];
                s += t * t;
            }
            d[i] = sqrt(s);
            D += d[i];
        }
        if (D != 0.0) {
            double H = 0.0;
            for (int j = 0; j < n; ++j) H -= ent64(p, d[j] / D);
            const double PC = d[C] / D;
            const double eC = ent64(p, PC);
            if (PC * H > -eC) {
                for (int i = 0; i < n; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < n; ++j) acc += dist_l2(v[i], v[j]);
                    S[i] = acc;
                }
                sel = argmin_tie(S, n);
                for (int k = 0; k < 3; ++k) outv[k] = v[sel][k];
            }
        }
    }
    unsigned char* row = p.dst + (int64_t)y * p.dst_pitch;
    for (int k = 0; k < 3; ++k) {
        if (p.u16) reinterpret_cast<uint16_t*>(row)[3 * x + k] = (uint16_t)outv[k];
        else row[3 * x + k] = (unsigned char)outv[k];
    }
}

// Grid-stride over the flagged list. Every block reads the count before it
// signals completion; the last block to finish records the count for the
// statistics and clears the counters for the next call.
__global__ __launch_bounds__(64) void recheck_kernel(const RParams p) {
    const uint32_t count = __atomic_load_n(&p.counters[0], __ATOMIC_RELAXED);
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x)
        recheck_one(p, p.flag_list[t]);
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&p.counters[1], 1u);
        last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        p.counters[2] = count;
        atomicExch(&p.counters[0], 0u);
        atomicExch(&p.counters[1], 0u);
    }
}

}  // namespace

int launch_recheck(const RParams& p, int blocks, void* stream) {
    hipLaunchKernelGGL(recheck_kernel, dim3(blocks), dim3(64), 0, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

}  // namespace vf
