// FP64 re-check of one flagged window by one wavefront (device code of the
// re-check kernels, which walk a call's list of flagged windows, of the FP64
// precision mode and of the batch re-check and overflow passes).
//
// The window is recomputed from the definitions in double precision with the
// same approximant (its FP32 constants widened exactly to double), and its
// output overwritten. Operations are written out one rounding at a time (no
// contraction) and every sum runs in member order, as in a plain loop over
// the definition, so the result is bit-identical to a straightforward FP64
// evaluation. Definitions (paper, Section 3): VDF sums of A = arccos(cosine)
// over all members; DDF (sum |x_i - x_j|_2)^(1-p) (sum A)^p; AMNFE weighted
// mean with h_i = n^(-kappa/3) sum_j |x_i - x_j|_1 and K = exp(-z) (0 above
// the cutoff; AMNFG: K = exp(-0.5 |x|_2^2)); EVMF switching test P_C H > -ENT(P_C) and the vector median.
// Ties: centre first, then the lowest index. Cosine conventions: identical,
// collinear or both-zero vectors 1; one zero vector 0. Integer products are
// formed in double; all of them are below 2^53, hence exact.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "vf_internal.h"

namespace vf {

// Candidate members whose rows of pair values the angle filters hold in LDS
// at once: as many as fill four rounds of the wave's 64 lanes (the rows of the
// other filters hold every member).
__host__ __device__ constexpr int recheck_rows(int n, int filter) {
    return (filter == VF_FILTER_VDF || filter == VF_FILTER_DDF) ? (256 / n < n ? (256 / n < 1 ? 1 : 256 / n) : n) : n;
}

// Doubles of LDS scratch one wave needs to re-check an n-member window (the
// angle filters' small row block keeps many waves resident per CU; the
// re-check is bound by the latency of each window's dependent steps).
__host__ __device__ constexpr int recheck_scratch_doubles(int n, int filter) {
    return 7 * n + 8 + recheck_rows(n, filter) * n * (filter == VF_FILTER_DDF ? 2 : 1);
}

struct RView {   // scratch layout
    double* v;    // [n][3]
    double* nn;   // [n] squared norms
    double* sq;   // [n] their square roots
    double* S;    // [n]
    double* A;    // [n]
    double* misc; // [8]: mean[3], D, switch
    double* PA;   // [rows * n] (rows = recheck_rows)
    double* PD;   // [rows * n]
};

__device__ inline RView recheck_view(double* base, int n, int rows) {
    RView r;
    r.v = base;
    r.nn = base + 3 * n;
    r.sq = base + 4 * n;
    r.S = base + 5 * n;
    r.A = base + 6 * n;
    r.misc = base + 7 * n;
    r.PA = base + 7 * n + 8;
    r.PD = r.PA + rows * n;
    return r;
}

__device__ inline double rc_horner(const float* c, int n, double x) {
#pragma clang fp contract(off)
    double acc = (double)c[n - 1];
    for (int k = n - 2; k >= 0; --k) acc = acc * x + (double)c[k];
    return acc;
}

__device__ inline double rc_angle(const KParams& p, int eval, double z) {
#pragma clang fp contract(off)
    switch (eval) {
    case EV_EXACT:
        return acos(z);
    case EV_PAPER:
        if (z < 0.5) return rc_horner(p.lo, p.n_lo, z);
        return rc_horner(p.hi, p.n_hi, sqrt(1.0 - z));
    case EV_SPLIT:
        if (z >= 0.5) {
            const double s = sqrt(2.0 * (1.0 - z));
            return s * rc_horner(p.hi, p.n_hi, s * s);
        }
        if (z <= -0.5) {
            const double s = sqrt(2.0 * (1.0 + z));
            return M_PI - s * rc_horner(p.hi, p.n_hi, s * s);
        }
        return M_PI / 2.0 - z * rc_horner(p.lo, p.n_lo, z * z);
    default: {   // EV_CHORD: one odd chord polynomial, mirrored for z < 0
        if (z >= 0.0) {
            const double s = sqrt(2.0 * (1.0 - z));
            return s * rc_horner(p.hi, p.n_hi, s * s);
        }
        const double s = sqrt(2.0 * (1.0 + z));
        return M_PI - s * rc_horner(p.hi, p.n_hi, s * s);
    }
    }
}

__device__ inline double rc_ent(const KParams& p, int eval, double z) {
#pragma clang fp contract(off)
    if (z <= 0.0 || z < p.cutoff64) return 0.0;   // the cutoff T of Section 3.3, every mode
    switch (eval) {
    case EV_EXACT:
        return z * log(z);
    case EV_PAPER:
        return rc_horner(p.lo, p.n_lo, z) / rc_horner(p.hi, p.n_hi, z);
    default: {
        int e;
        double m = frexp(z, &e);
        m *= 2.0;
        e -= 1;
        return z * ((double)e * M_LN2 + rc_horner(p.lo, p.n_lo, m - 1.0));
    }
    }
}

__device__ inline double rc_cosine(const RView& r, int i, int j) {
#pragma clang fp contract(off)
    const double na = r.nn[i], nb = r.nn[j];
    if (na == 0.0 && nb == 0.0) return 1.0;
    if (na == 0.0 || nb == 0.0) return 0.0;
    const double* a = r.v + 3 * i;
    const double* b = r.v + 3 * j;
    const double c0 = a[1] * b[2] - a[2] * b[1];
    const double c1 = a[2] * b[0] - a[0] * b[2];
    const double c2 = a[0] * b[1] - a[1] * b[0];
    if (c0 == 0.0 && c1 == 0.0 && c2 == 0.0) return 1.0;
    const double dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double z = dot / (r.sq[i] * r.sq[j]);
    if (z > 1.0) z = 1.0;
    if (z < -1.0) z = -1.0;
    return z;
}

__device__ inline double rc_l2(const RView& r, int i, int j) {
#pragma clang fp contract(off)
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double d = r.v[3 * i + k] - r.v[3 * j + k];
        s += d * d;
    }
    return sqrt(s);
}

__device__ inline double rc_l1(const RView& r, int i, int j) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += fabs(r.v[3 * i + k] - r.v[3 * j + k]);
    return s;   // exact integer
}

__device__ inline int rc_argmin(const double* s, int n) {
    int best = (n - 1) / 2;
    for (int i = 0; i < n; ++i)
        if (s[i] < s[best]) best = i;
    return best;
}

// The image a window lies in (the KParams' own for a single image; a batch
// item's otherwise, with the class's KParams: a per-window copy of KParams
// would live in private memory, since the coefficients are indexed at run time).
struct RcImage {
    const unsigned char* src;
    unsigned char* dst;
    int64_t src_pitch, dst_pitch;
    int H, W, u16;
};
__device__ inline RcImage rc_image(const KParams& p) {
    return RcImage{p.src, p.dst, p.src_pitch, p.dst_pitch, p.H, p.W, p.u16};
}

// Re-check the window centred on (y, x) of image im; the whole wave calls this
// with the same arguments. lane = lane index within the wave.
// mask: for the angle filters, the members whose FP32 criterion was within
// the error bound of the minimum (all other members provably have larger
// FP64 criteria, so the oracle's choice is among these); all ones: no such
// information, recompute every member.
template <int FILT>
__device__ void recheck_window(const KParams& p, const RcImage& im, int eval, int window, int y, int x,
                               double* scratch, int lane, uint64_t mask = ~0ull) {
#pragma clang fp contract(off)
    const int w = window, rr = (w - 1) / 2, n = w * w, C = (n - 1) / 2;
    const RView r = recheck_view(scratch, n, recheck_rows(n, FILT));
    if (lane < n) {
        const int yy = min(max(y + lane / w - rr, 0), im.H - 1);
        const int xx = min(max(x + lane % w - rr, 0), im.W - 1);
        const unsigned char* row = im.src + (int64_t)yy * im.src_pitch;
        int64_t m[3];
        for (int k = 0; k < 3; ++k)
            m[k] = im.u16 ? (int64_t)reinterpret_cast<const uint16_t*>(row)[3 * xx + k]
                         : (int64_t)row[3 * xx + k];
        for (int k = 0; k < 3; ++k) r.v[3 * lane + k] = (double)m[k];
        const int64_t na = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
        r.nn[lane] = (double)na;
        r.sq[lane] = sqrt((double)na);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    int sel = C;
    double outq[3];
    bool mean_out = false;
    if constexpr (FILT == VF_FILTER_VDF || FILT == VF_FILTER_DDF) {
        constexpr bool ddf = FILT == VF_FILTER_DDF;
        // FP64 criteria of the candidate members only (every member when the
        // mask carries no information), a block of candidates at a time: the
        // lanes form the block's rows of pair values, then one lane per
        // candidate sums its row in member order
        const uint64_t all = (1ull << n) - 1ull;
        const uint64_t cm = (mask & all) != 0ull ? (mask & all) : all;
        const int k = __popcll(cm);
        const int rows = recheck_rows(n, FILT);
        int* cand = reinterpret_cast<int*>(r.A);   // candidate c -> member index
        if (lane < n && ((cm >> lane) & 1ull)) cand[__popcll(cm & ((1ull << lane) - 1ull))] = lane;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int c0 = 0; c0 < k; c0 += rows) {
            const int kb = min(rows, k - c0);
            for (int q = lane; q < kb * n; q += 64) {
                const int c = q / n, j = q - (q / n) * n;
                const int i = cand[c0 + c];
                r.PA[q] = rc_angle(p, eval, rc_cosine(r, i, j));
                if (ddf) r.PD[q] = rc_l2(r, i, j);
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if (lane < kb) {
                double a = 0.0, d = 0.0;
                for (int j = 0; j < n; ++j) {
                    a += r.PA[lane * n + j];
                    if (ddf) d += r.PD[lane * n + j];
                }
                r.S[cand[c0 + lane]] = ddf ? pow(d, 1.0 - p.param64) * pow(a, p.param64) : a;
            }
            // (the block's rows are read before the next block overwrites them)
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        // the oracle keeps the centre if it is a minimiser, else takes the
        // lowest-index minimiser; every minimiser is a candidate
        sel = ((cm >> C) & 1ull) ? C : __builtin_ctzll(cm);
        for (uint64_t m = cm; m != 0ull; m &= m - 1ull) {
            const int i = __builtin_ctzll(m);
            if (r.S[i] < r.S[sel]) sel = i;
        }
    } else if constexpr (is_amnf(FILT)) {
        for (int q = lane; q < n * n; q += 64) {
            const int i = q / n, j = q - (q / n) * n;
            r.PA[q] = rc_l1(r, i, j);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (lane < n) {
            double acc = 0.0;   // exact integer sum
            for (int j = 0; j < n; ++j) acc += r.PA[lane * n + j];
            r.S[lane] = acc;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        bool uniform = false;
        for (int i = 0; i < n; ++i) uniform |= (r.S[i] == 0.0);
        if (!uniform) {
            if (lane < n) {
                const double h = p.scale64 * r.S[lane];
                double z;
                if constexpr (FILT == VF_FILTER_AMNFG) {
                    // Gaussian kernel: 0.5 |x|_2^2 of x = (x_C - x_i) / h_i
                    double q = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        const double t = (r.v[3 * C + c] - r.v[3 * lane + c]) / h;
                        q += t * t;
                    }
                    z = 0.5 * q;
                } else {
                    z = r.PA[C * n + lane] / h;
                }
                double k;
                if (z > p.cutoff64) k = 0.0;
                else if (eval == EV_EXACT) k = exp(-z);
                else if (eval == EV_PAPER) k = rc_horner(p.lo, p.n_lo, z) / rc_horner(p.hi, p.n_hi, z);
                else k = rc_horner(p.lo, p.n_lo, z);
                r.A[lane] = k / (h * h * h);
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            double num[3] = {0.0, 0.0, 0.0}, den = 0.0;
            for (int i = 0; i < n; ++i) {
                den += r.A[i];
                for (int c = 0; c < 3; ++c) num[c] += r.A[i] * r.v[3 * i + c];
            }
            if (den > 0.0) {
                const double maxv = im.u16 ? 65535.0 : 255.0;
                for (int c = 0; c < 3; ++c) {
                    double q = floor(num[c] / den + 0.5);
                    outq[c] = q < 0.0 ? 0.0 : (q > maxv ? maxv : q);
                }
                mean_out = true;
            }
        }
    } else {   // EVMF
        double mean[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) mean[k] += r.v[3 * i + k];
        for (int k = 0; k < 3; ++k) mean[k] /= (double)n;
        if (lane < n) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double t = r.v[3 * lane + k] - mean[k];
                s += t * t;
            }
            r.A[lane] = sqrt(s);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        double D = 0.0;
        for (int i = 0; i < n; ++i) D += r.A[i];
        if (D != 0.0) {
            if (lane < n) r.S[lane] = rc_ent(p, eval, r.A[lane] / D);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            double H = 0.0;
            for (int j = 0; j < n; ++j) H -= r.S[j];
            const double PC = r.A[C] / D;
            const double eC = rc_ent(p, eval, PC);
            if (PC * H > -eC) {
                for (int q = lane; q < n * n; q += 64) {
                    const int i = q / n, j = q - (q / n) * n;
                    r.PA[q] = rc_l2(r, i, j);
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (lane < n) {
                    double acc = 0.0;
                    for (int j = 0; j < n; ++j) acc += r.PA[lane * n + j];
                    r.S[lane] = acc;
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                sel = rc_argmin(r.S, n);
            }
        }
    }
    if (lane == 0) {
        unsigned char* row = im.dst + (int64_t)y * im.dst_pitch;
        for (int k = 0; k < 3; ++k) {
            const double v = mean_out ? outq[k] : r.v[3 * sel + k];
            if (im.u16) reinterpret_cast<uint16_t*>(row)[3 * x + k] = (uint16_t)v;
            else row[3 * x + k] = (unsigned char)v;
        }
    }
    // the scratch is reused by the next window
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Copy a workgroup's LDS list of n flagged pixels (and, if given, their
// candidate masks) to the global list with one atomic reservation (called by
// every thread of the workgroup; `base` is LDS).
__device__ inline void publish_flags(const KParams& p, const uint32_t* list, uint32_t n, uint32_t* base,
                                     int tid, int nthreads, const uint64_t* masks = nullptr) {
    if (n == 0u) return;
    if (tid == 0) *base = atomicAdd(p.flag_count, n);
    __syncthreads();
    const uint32_t b = *base;
    for (uint32_t e = (uint32_t)tid; e < n; e += (uint32_t)nthreads) {
        if (b + e < p.flag_cap) {
            p.flag_list[b + e] = list[e];
            if (p.flag_item) p.flag_item[b + e] = (uint32_t)p.item;
            if (masks) p.flag_mask[b + e] = masks[e];
        }
    }
    __syncthreads();
}

}  // namespace vf
