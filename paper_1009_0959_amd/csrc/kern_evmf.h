// EVMF window kernel (Section 3.3, EVF equation):
//   P_i = |x_i - x_bar|_2 / sum_j |x_j - x_bar|_2,
//   beta_i = -P_i log P_i / (-sum_j P_j log P_j),
//   y = argmin_i sum_j |x_i - x_j|_2 if P_C > beta_C, else x(r,c).
// The test is evaluated multiplied through by the non-negative denominator:
// g = P_C H + ENT(P_C) > 0 with H = -sum_j ENT(P_j). The vector-median pair
// loop runs only in lanes whose window switches (or is too close to call).
#pragma once

#include "kern_common.h"
#include "recheck_dev.h"

namespace vf {

template <int WIN, int MODE>
__device__ __forceinline__ void evmf_tile(const KParams& p, const int tile) {
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
    float xr[N], xg[N], xb[N];
    float sr = 0.0f, sg = 0.0f, sb = 0.0f;   // exact integer sums
#pragma unroll
    for (int i = 0; i < N; ++i) {
        pk[i] = sP[(ly + i / WIN) * LW + (lx + i % WIN)];
        unpack_pixel(pk[i], u16, xr[i], xg[i], xb[i]);
        sr += xr[i];
        sg += xg[i];
        sb += xb[i];
    }
    // deviations from the mean, scaled by n: n x_i - sum_j x_j is an exact
    // integer in FP32, so d_i carries only the rounding of one sqrt of a sum
    // of squares; P_i = d_i / sum_j d_j is unchanged by the common factor n
    float d[N];
    float D = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const float a = fmaf((float)N, xr[i], -sr);
        const float b = fmaf((float)N, xg[i], -sg);
        const float c = fmaf((float)N, xb[i], -sb);
        d[i] = fsqrt(fmaf(a, a, fmaf(b, b, c * c)));
        D += d[i];
    }

    uint2 out = pk[C];
    bool flag = false;
    if (D > 0.0f) {   // D = 0 <=> uniform window -> x_C
        const float invD = 1.0f / D;
        float H = 0.0f;
        // ENT jumps at the cutoff T (when T > 0), so a P_i within the FP32
        // error band of T may sit on the other side of it in exact arithmetic
        bool near_cut = false;
        const bool cut_on = p.cutoff > 0.0f;
        const float cut_band = 4.0f * (N + 4) * kU32 * p.cutoff;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const float Pi = d[i] * invD;
            if (cut_on) near_cut |= fabsf(Pi - p.cutoff) <= cut_band;
            H -= ent<MODE>(Pi, p.lo, p.n_lo, p.hi, p.n_hi, p.cutoff);
        }
        const float PC = d[C] * invD;
        const float eC = ent<MODE>(PC, p.lo, p.n_lo, p.hi, p.n_hi, p.cutoff);
        const float g = fmaf(PC, H, eC);
        const float gb = 4.0f * (N + 4) * kU32 * (PC * (H + 2.0f) + fabsf(eC)) + 1e-7f;
        const bool sw = g > 0.0f;
        flag = fabsf(g) <= gb || near_cut;
        if (sw) {
            float S[N];
#pragma unroll
            for (int i = 0; i < N; ++i) S[i] = 0.0f;
#pragma unroll
            for (int i = 0; i < N; ++i) {
#pragma unroll
                for (int j = i + 1; j < N; ++j) {
                    const float a = xr[i] - xr[j], b = xg[i] - xg[j], c = xb[i] - xb[j];
                    const float dd = fsqrt(fmaf(a, a, fmaf(b, b, c * c)));
                    S[i] += dd;
                    S[j] += dd;
                }
            }
            float best = S[C];
            uint2 pb = pk[C];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const bool lt = S[i] < best;
                best = lt ? S[i] : best;
                pb = lt ? pk[i] : pb;
            }
            float s2 = __builtin_inff();
#pragma unroll
            for (int i = 0; i < N; ++i) s2 = !same_pixel(pk[i], pb) ? fminf(s2, S[i]) : s2;
            flag |= (s2 - best) <= (2.0f * N + 8.0f) * kU32 * (best + s2);
            out = pb;
        }
    }
    if (valid) store_pixel(p.dst + (int64_t)gy * p.dst_pitch, gx, out, u16);
    if (valid && p.recheck && flag) s_flags[atomicAdd(&s_nflag, 1u)] = (uint32_t)(gy * p.W + gx);
    __syncthreads();
    // one reservation in the re-check list for the whole workgroup
    publish_flags(p, s_flags, s_nflag, &s_base, threadIdx.x, kThreads);
}

template <int WIN, int MODE>
__global__ __launch_bounds__(kThreads) void evmf_kernel(const KParams p) {
    evmf_tile<WIN, MODE>(p, xcd_tile(blockIdx.x, gridDim.x));
}

}  // namespace vf
