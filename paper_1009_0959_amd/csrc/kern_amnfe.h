// AMNF window kernel (Section 3.2, AMNF equation):
//   y = sum_i x_i w_i / sum_j w_j,  w_i = h_i^-3 K((x_C - x_i) / h_i),
//   h_i = n^(-kappa/3) sum_j |x_i - x_j|_1,
// with the exponential kernel K(x) = exp(-|x|_1) (AMNFE) or the Gaussian
// kernel K(x) = exp(-0.5 |x|_2^2) (AMNFG, GAUSS).
// Pair work is one exact integer L1 distance per unordered pair (v_sad_u8 /
// v_sad_u16). Per member, with r_i = n^(kappa/3) / S1_i = 1 / h_i: the EXP
// argument z_i = L1_Ci r_i (AMNFE) or 0.5 |x_C - x_i|_2^2 r_i^2 (AMNFG),
// K = exp(-z_i), and w_i = K / S1_i^3 (the common factor n^(-kappa) of
// h_i^-3 cancels in the ratio). The mean is accumulated relative to x_C,
// y = x_C + sum_i w_i (x_i - x_C) / sum_i w_i, which keeps the FP32 rounding
// proportional to the spread of the window instead of its magnitude.
#pragma once

#include "batch.h"
#include "kern_common.h"
#include "recheck_dev.h"

namespace vf {

template <int WIN, int MODE, bool GAUSS>
__device__ __forceinline__ void amnfe_tile(const KParams& p, const int tile) {
    constexpr int R = (WIN - 1) / 2;
    constexpr int N = WIN * WIN;
    constexpr int C = (N - 1) / 2;
    constexpr int LW = kTileX + 2 * R;
    constexpr int LH = kTileY + 2 * R;
    constexpr int LN = LW * LH;

    __shared__ uint2 sP[LN];
    __shared__ uint32_t s_nflag, s_base;
    __shared__ uint32_t s_flags[kThreads];
    if (threadIdx.x == 0) s_nflag = 0u;
    int tx0, ty0;
    tile_origin(p, tile, tx0, ty0);
    const int u16 = p.u16;
    for (int t = threadIdx.x; t < LN; t += kThreads) {
        const int ly = t / LW;
        const int lx = t - ly * LW;
        const int gy = min(max(ty0 + ly - R, 0), p.H - 1);
        const int gx = min(max(tx0 + lx - R, 0), p.W - 1);
        uint32_t r, g, b;
        load_pixel(p.src + (int64_t)gy * p.src_pitch, gx, u16, r, g, b);
        sP[t] = pack_pixel(r, g, b, u16);
    }
    __syncthreads();

    const int lx = threadIdx.x % kTileX;
    const int ly = threadIdx.x / kTileX;
    const int gx = tx0 + lx;
    const int gy = ty0 + ly;
    // threads past the image edge compute a (discarded) window from the tile
    const bool valid = gx < p.W && gy < p.H;

    uint2 pk[N];
#pragma unroll
    for (int i = 0; i < N; ++i) pk[i] = sP[(ly + i / WIN) * LW + (lx + i % WIN)];

    uint32_t S1[N], L1C[N];
#pragma unroll
    for (int i = 0; i < N; ++i) S1[i] = 0u;
    L1C[C] = 0u;
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = i + 1; j < N; ++j) {
            const uint32_t d = l1_dist(pk[i], pk[j], u16);
            S1[i] += d;
            S1[j] += d;
            if (i == C) L1C[j] = d;
            if (j == C) L1C[i] = d;
        }
    }

    uint2 out = pk[C];
    bool flag = false;
    if (S1[0] != 0u) {   // S1_i = 0 for some i <=> uniform window -> x_C
        float cr, cg, cb;
        unpack_pixel(pk[C], u16, cr, cg, cb);
        float num0 = 0.0f, num1 = 0.0f, num2 = 0.0f, den = 0.0f;
        float ab0 = 0.0f, ab1 = 0.0f, ab2 = 0.0f;
        const bool near_cut_possible = p.zband > 0.0f;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float rs = frcp((float)S1[i]);
            float xr, xg, xb;
            unpack_pixel(pk[i], u16, xr, xg, xb);
            const float d0 = xr - cr, d1 = xg - cg, d2 = xb - cb;
            float z;
            if constexpr (GAUSS) {
                const float t = rs * p.kscale;
                z = 0.5f * fmaf(d0, d0, fmaf(d1, d1, d2 * d2)) * (t * t);
            } else {
                z = (float)L1C[i] * rs * p.kscale;
            }
            // K jumps at the cutoff: an argument within its error of T is decided in FP64
            if (near_cut_possible) flag |= fabsf(z - p.cutoff) <= p.zband;
            const float k = kernel_exp<MODE>(z, p.lo, p.n_lo, p.hi, p.n_hi, p.cutoff);
            const float r3 = rs * rs * rs;
            const float w = k * r3;
            num0 = fmaf(w, d0, num0);
            num1 = fmaf(w, d1, num1);
            num2 = fmaf(w, d2, num2);
            ab0 = fmaf(w, fabsf(d0), ab0);
            ab1 = fmaf(w, fabsf(d1), ab1);
            ab2 = fmaf(w, fabsf(d2), ab2);
            den += w;
        }
        const float maxv = u16 ? 65535.0f : 255.0f;
        const float inv = 1.0f / den;
        const float y[3] = {fmaf(num0, inv, cr), fmaf(num1, inv, cg), fmaf(num2, inv, cb)};
        const float ab[3] = {ab0 * inv, ab1 * inv, ab2 * inv};
        const float dy[3] = {num0 * inv, num1 * inv, num2 * inv};
        uint32_t q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float v = floorf(y[k] + 0.5f);
            // distance of y + 0.5 to the rounding boundaries v and v + 1
            const float frac = (y[k] + 0.5f) - v;
            // each weight within p.wbound units of its exact value moves y by at
            // most 2 wbound u sum w |d| / sum w; the FP32 sums of N terms add 2 N u
            float bound = (2.0f * p.wbound + 2.0f * N) * kU32 * ab[k] + 4.0f * kU32 * fabsf(y[k]) + 1e-6f;
            // approximants: each weight is within the relative p.rho' = r / (1 - r)
            // of its value with K evaluated exactly (r from the Horner or
            // rational evaluation bound over the least K), which moves y by at
            // most p.rho' (sum w |d| / sum w + |y - x_C|)
            if constexpr (MODE != EV_EXACT) bound += 1.01f * p.rho * (ab[k] + fabsf(dy[k]));
            flag |= (frac < bound) || (1.0f - frac < bound);
            q[k] = (uint32_t)fminf(fmaxf(v, 0.0f), maxv);
        }
        flag |= !(den > 0.0f);
        // an approximant that is not positive over the argument range (the
        // host's relative bound is then infinite): weights of either sign,
        // no FP32 bound holds, every window is decided in FP64
        if constexpr (MODE != EV_EXACT) flag |= !(p.rho < 1e29f);
        out = pack_pixel(q[0], q[1], q[2], u16);
    }
    if (valid) store_pixel(p.dst + (int64_t)gy * p.dst_pitch, gx, out, u16);
    if (valid && p.recheck && flag) s_flags[atomicAdd(&s_nflag, 1u)] = (uint32_t)(gy * p.W + gx);
    __syncthreads();
    // one reservation in the re-check list for the whole workgroup
    publish_flags(p, s_flags, s_nflag, &s_base, threadIdx.x, kThreads);
}

template <int WIN, int MODE, bool GAUSS>
__global__ __launch_bounds__(kThreads) void amnfe_kernel(const KParams p) {
    amnfe_tile<WIN, MODE, GAUSS>(p, xcd_tile(blockIdx.x, gridDim.x));
}

template <int WIN, int MODE, bool GAUSS>
__global__ __launch_bounds__(kThreads) void amnfe_batch_kernel(const BatchParams bp) {
    batch_loop(bp, [&](const KParams& p, int tile) { amnfe_tile<WIN, MODE, GAUSS>(p, tile); });
}

// Single-image and persistent batch launchers of one window size and kernel
// (each instantiated in its own translation unit so that the large unrolled
// 7x7 kernels compile in parallel); -1 when no kernel matches.
template <int WIN, bool GAUSS>
int amnfe_launch_w(int eval, const KParams& p, int blocks, void* stream) {
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, p);
        return (int)hipGetLastError();
    };
    switch (eval) {
    case EV_EXACT: return go(amnfe_kernel<WIN, EV_EXACT, GAUSS>);
    case EV_MINIMAX: return go(amnfe_kernel<WIN, EV_MINIMAX, GAUSS>);
    case EV_PAPER: return go(amnfe_kernel<WIN, EV_PAPER, GAUSS>);
    }
    return -1;
}

template <int WIN, bool GAUSS>
int amnfe_batch_launch_w(int eval, const BatchParams& bp, int num_cus, void* stream, bool probe) {
    switch (eval) {
    case EV_EXACT: return launch_persistent(probe, amnfe_batch_kernel<WIN, EV_EXACT, GAUSS>, kThreads, bp, num_cus, stream);
    case EV_MINIMAX:
        return launch_persistent(probe, amnfe_batch_kernel<WIN, EV_MINIMAX, GAUSS>, kThreads, bp, num_cus, stream);
    case EV_PAPER: return launch_persistent(probe, amnfe_batch_kernel<WIN, EV_PAPER, GAUSS>, kThreads, bp, num_cus, stream);
    }
    return -1;
}

}  // namespace vf
