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

// One wavefront per flagged window. The members are gathered into LDS as
// exact doubles (integer channel values, their squared norms and the norms'
// square roots); the n^2 pair values are computed by all 64 lanes into an LDS
// matrix; then lane i sums row i over j in index order, and sums that run
// over members (AMNFE weights, EVMF mean, D and H) are taken by lane 0
// serially in member order. Every quantity is therefore computed with the
// operations, in the order, of the plain definition. Integer products are
// formed in double: every one of them is below 2^53, so they are exact.
struct Shared {
    double v[kMaxN][3];
    double nn[kMaxN];     // squared norm (exact integer)
    double sq[kMaxN];     // sqrt of the squared norm
    double S[kMaxN];
    double A[kMaxN];
    double mean[3];
    double D;
    int sw;
};

__device__ double cosine_m(const Shared& sh, int i, int j) {
    const double na = sh.nn[i], nb = sh.nn[j];
    if (na == 0.0 && nb == 0.0) return 1.0;
    if (na == 0.0 || nb == 0.0) return 0.0;
    const double* a = sh.v[i];
    const double* b = sh.v[j];
    const double c0 = a[1] * b[2] - a[2] * b[1];
    const double c1 = a[2] * b[0] - a[0] * b[2];
    const double c2 = a[0] * b[1] - a[1] * b[0];
    if (c0 == 0.0 && c1 == 0.0 && c2 == 0.0) return 1.0;
    const double dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double z = dot / (sh.sq[i] * sh.sq[j]);
    if (z > 1.0) z = 1.0;
    if (z < -1.0) z = -1.0;
    return z;
}

__device__ double l2_m(const Shared& sh, int i, int j) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double d = sh.v[i][k] - sh.v[j][k];
        s += d * d;
    }
    return sqrt(s);
}

__device__ double l1_m(const Shared& sh, int i, int j) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += fabs(sh.v[i][k] - sh.v[j][k]);
    return s;   // exact integer
}

__device__ void recheck_window(const RParams& p, uint32_t pix, Shared& sh, double* PA, double* PD) {
    const int lane = threadIdx.x;
    const int y = (int)(pix / (uint32_t)p.W);
    const int x = (int)(pix - (uint32_t)y * (uint32_t)p.W);
    const int w = p.window, r = (w - 1) / 2, n = w * w, C = (n - 1) / 2;
    if (lane < n) {
        int64_t m[3];
        fetch(p, y + lane / w - r, x + lane % w - r, m);
        for (int k = 0; k < 3; ++k) sh.v[lane][k] = (double)m[k];
        const int64_t na = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
        sh.nn[lane] = (double)na;
        sh.sq[lane] = sqrt((double)na);
    }
    __syncthreads();
    double outv[3] = {sh.v[C][0], sh.v[C][1], sh.v[C][2]};
    if (p.filter == VF_FILTER_VDF || p.filter == VF_FILTER_DDF) {
        const bool ddf = p.filter == VF_FILTER_DDF;
        for (int q = lane; q < n * n; q += 64) {
            const int i = q / n, j = q - (q / n) * n;
            PA[q] = angle64(p, cosine_m(sh, i, j));
            if (ddf) PD[q] = l2_m(sh, i, j);
        }
        __syncthreads();
        if (lane < n) {
            double a = 0.0, d = 0.0;
            for (int j = 0; j < n; ++j) {
                a += PA[lane * n + j];
                if (ddf) d += PD[lane * n + j];
            }
            sh.S[lane] = ddf ? pow(d, 1.0 - p.param) * pow(a, p.param) : a;
        }
        __syncthreads();
        const int sel = argmin_tie(sh.S, n);
        for (int k = 0; k < 3; ++k) outv[k] = sh.v[sel][k];
    } else if (p.filter == VF_FILTER_AMNFE) {
        for (int q = lane; q < n * n; q += 64) {
            const int i = q / n, j = q - (q / n) * n;
            PA[q] = l1_m(sh, i, j);
        }
        __syncthreads();
        if (lane < n) {
            double acc = 0.0;   // exact integer sum
            for (int j = 0; j < n; ++j) acc += PA[lane * n + j];
            sh.S[lane] = acc;
        }
        __syncthreads();
        bool uniform = false;
        for (int i = 0; i < n; ++i) uniform |= (sh.S[i] == 0.0);
        if (!uniform) {
            if (lane < n) {
                const double h = p.scale * sh.S[lane];
                const double z = PA[C * n + lane] / h;
                double k;
                if (z > p.cutoff) k = 0.0;
                else if (p.eval == EV_EXACT) k = exp(-z);
                else k = horner64(p.lo, p.n_lo, z);
                sh.A[lane] = k / (h * h * h);
            }
            __syncthreads();
            double num[3] = {0.0, 0.0, 0.0}, den = 0.0;
            for (int i = 0; i < n; ++i) {
                den += sh.A[i];
                for (int c = 0; c < 3; ++c) num[c] += sh.A[i] * sh.v[i][c];
            }
            if (den > 0.0) {
                const double maxv = p.u16 ? 65535.0 : 255.0;
                for (int c = 0; c < 3; ++c) {
                    double q = floor(num[c] / den + 0.5);
                    if (q < 0.0) q = 0.0;
                    if (q > maxv) q = maxv;
                    outv[c] = q;
                }
            }
        }
    } else {   // EVMF
        if (lane == 0) {
            double m[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < n; ++i)
                for (int k = 0; k < 3; ++k) m[k] += sh.v[i][k];
            for (int k = 0; k < 3; ++k) sh.mean[k] = m[k] / (double)n;
        }
        __syncthreads();
        if (lane < n) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double t = sh.v[lane][k] - sh.mean[k];
                s += t * t;
            }
            sh.A[lane] = sqrt(s);
        }
        __syncthreads();
        if (lane == 0) {
            double D = 0.0;
            for (int i = 0; i < n; ++i) D += sh.A[i];
            sh.D = D;
        }
        __syncthreads();
        const double D = sh.D;
        if (D != 0.0) {
            if (lane < n) sh.S[lane] = ent64(p, sh.A[lane] / D);
            __syncthreads();
            if (lane == 0) {
                double H = 0.0;
                for (int j = 0; j < n; ++j) H -= sh.S[j];
                const double PC = sh.A[C] / D;
                const double eC = ent64(p, PC);
                sh.sw = (PC * H > -eC) ? 1 : 0;
            }
            __syncthreads();
            if (sh.sw) {
                for (int q = lane; q < n * n; q += 64) {
                    const int i = q / n, j = q - (q / n) * n;
                    PA[q] = l2_m(sh, i, j);
                }
                __syncthreads();
                if (lane < n) {
                    double acc = 0.0;
                    for (int j = 0; j < n; ++j) acc += PA[lane * n + j];
                    sh.S[lane] = acc;
                }
                __syncthreads();
                const int sel = argmin_tie(sh.S, n);
                for (int k = 0; k < 3; ++k) outv[k] = sh.v[sel][k];
            }
        }
    }
    if (lane == 0) {
        unsigned char* row = p.dst + (int64_t)y * p.dst_pitch;
        for (int k = 0; k < 3; ++k) {
            if (p.u16) reinterpret_cast<uint16_t*>(row)[3 * x + k] = (uint16_t)outv[k];
            else row[3 * x + k] = (unsigned char)outv[k];
        }
    }
    __syncthreads();
}

// Grid-stride over the flagged list, one window per workgroup (one wave) at a
// time; the dynamic LDS holds the n x n pair matrices. Block 0 clears the
// next call's counter slot.
__global__ __launch_bounds__(64) void recheck_kernel(const RParams p) {
    __shared__ Shared sh;
    extern __shared__ double pairs[];
    const int n = p.window * p.window;
    double* PA = pairs;
    double* PD = pairs + n * n;
    if (blockIdx.x == 0 && threadIdx.x == 0) *p.next_count = 0u;
    const uint32_t count = *p.count;
    for (uint32_t t = blockIdx.x; t < count; t += gridDim.x) recheck_window(p, p.flag_list[t], sh, PA, PD);
}

}  // namespace

int launch_recheck(const RParams& p, int blocks, void* stream) {
    const int n = p.window * p.window;
    const size_t lds = (size_t)n * n * sizeof(double) * (p.filter == VF_FILTER_DDF ? 2 : 1);
    hipLaunchKernelGGL(recheck_kernel, dim3(blocks), dim3(64), lds, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

}  // namespace vf
