// Angle-criterion window kernels: VDF (Section 3.1, BVDF equation) and DDF
// (the directional-distance filter named in Section 3.1).
#pragma once

#include "kern_common.h"
#include "recheck_dev.h"

namespace vf {

// Output tile height: 4 rows (256 threads), or 2 rows (128 threads) for the
// 7x7 window whose rolled pair loop keeps per-member partial sums in LDS.
template <int WIN>
constexpr int angle_tile_y() { return WIN == 7 ? 2 : kTileY; }

template <int FILT, int WIN, int MODE, int NLO, int NHI>
__device__ __forceinline__ void angle_tile(const KParams& p, const int tile) {
    constexpr int TY = angle_tile_y<WIN>();
    constexpr int NT = kTileX * TY;
    constexpr int R = (WIN - 1) / 2;
    constexpr int N = WIN * WIN;
    constexpr int C = (N - 1) / 2;
    constexpr int LW = kTileX + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int LN = LW * LH;
    constexpr bool DDF = (FILT == VF_FILTER_DDF);
    constexpr bool ROLLED = (WIN == 7);
    constexpr int NACC = 1 + (DDF ? 1 : 0) + (MODE == EV_EXACT ? 1 : 0);

    // LDS: halo tile (unit vectors, packed pixels) and the rolled loop's
    // per-thread partial sums
    constexpr int SMEM = LN * 16 + LN * 8 + (ROLLED ? NACC * N * NT * 4 : 0);
    __shared__ __align__(16) unsigned char smem[SMEM];
    __shared__ uint32_t s_nflag, s_base;
    __shared__ uint32_t s_flags[NT];
    constexpr bool MASKS = writes_masks(FILT, WIN, MODE, false);
    __shared__ uint64_t s_masks[MASKS ? NT : 1];   // candidate members per flagged window
    float4* sU = reinterpret_cast<float4*>(smem);            // w = 1 marks the zero vector
    uint2* sP = reinterpret_cast<uint2*>(smem + LN * 16);    // packed channels
    float* sT = reinterpret_cast<float*>(smem + LN * 24);    // rolled loop partial sums
    if (threadIdx.x == 0) s_nflag = 0u;

    int tx0, ty0;
    {
        const int t = tile;
        const int ty = t / p.tiles_x;
        ty0 = ty * TY;
        tx0 = (t - ty * p.tiles_x) * kTileX;
    }
    const int u16 = p.u16;

    // 1. halo tile -> LDS, with the per-pixel unit vector (FP64 normalisation,
    //    rounded once to FP32)
    for (int t = threadIdx.x; t < LN; t += NT) {
        const int ly = t / LW;
        const int lx = t - ly * LW;
        const int gy = min(max(ty0 + ly - R, 0), p.H - 1);
        const int gx = min(max(tx0 + lx - R, 0), p.W - 1);
        uint32_t r, g, b;
        load_pixel(p.src + (int64_t)gy * p.src_pitch, gx, u16, r, g, b);
        sP[t] = pack_pixel(r, g, b, u16);
        sU[t] = unit_vector(r, g, b);
    }
    __syncthreads();

    const int lx = threadIdx.x % kTileX;
    const int ly = threadIdx.x / kTileX;
    const int gx = tx0 + lx;
    const int gy = ty0 + ly;
    // threads past the image edge compute a (discarded) window from the tile
    const bool valid = gx < p.W && gy < p.H;

    // 2. gather the window (row-major member order)
    float ux[N], uy[N], uz[N];
    float xr[DDF ? N : 1], xg[DDF ? N : 1], xb[DDF ? N : 1];
    bool anyzero = false, allzero = true;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int li = (ly + i / WIN) * LW + (lx + i % WIN);
        const float4 u = sU[li];
        ux[i] = u.x;
        uy[i] = u.y;
        uz[i] = u.z;
        anyzero |= (u.w != 0.0f);
        allzero &= (u.w != 0.0f);
        if constexpr (DDF) unpack_pixel(sP[li], u16, xr[i], xg[i], xb[i]);
    }

    // 3. every unordered pair once; pair value added to both members' sums
    float SA[N], SD[DDF ? N : 1], EA[MODE == EV_EXACT ? N : 1];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        SA[i] = 0.0f;
        if constexpr (DDF) SD[i] = 0.0f;
        if constexpr (MODE == EV_EXACT) EA[i] = 0.0f;
    }
    // exact mode: acosf of the cosine z = 1 - s^2/2 rounded to FP32 (rounding
    // error <= 2^-25) is off by about 2^-25 / sin(theta) <= 1.5 * 2^-25 / s for
    // s^2 >> 2^-24 and by up to sqrt(2^-24) when z rounds to 1; the bound
    // 2^-23 / sqrt(s^2 + 2^-24) covers both, plus 6e-7 for acosf itself
    constexpr float kExactK = 1.1920929e-07f;
    auto pair = [&](float uxi, float uyi, float uzi, float xri, float xgi, float xbi, int j,
                    float& acc_a, float& acc_d, float& acc_e) {
        const float dx = uxi - ux[j];
        const float dy = uyi - uy[j];
        const float dz = uzi - uz[j];
        const float s2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float a = angle_from_s2<MODE, NLO, NHI>(s2, p.lo, p.hi);
        acc_a += a;
        SA[j] += a;
        if constexpr (MODE == EV_EXACT) {
            const float e = s2 > 0.0f ? fmaf(kExactK, frsq(s2 + 5.9604645e-08f), 6.0e-7f) : 0.0f;
            acc_e += e;
            EA[j] += e;
        }
        if constexpr (DDF) {
            const float er = xri - xr[j];
            const float eg = xgi - xg[j];
            const float eb = xbi - xb[j];
            const float d = fsqrt(fmaf(er, er, fmaf(eg, eg, eb * eb)));
            acc_d += d;
            SD[j] += d;
        }
    };
    if constexpr (!ROLLED) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float acc_a = 0.0f, acc_d = 0.0f, acc_e = 0.0f;
#pragma unroll
            for (int j = i + 1; j < N; ++j)
                pair(ux[i], uy[i], uz[i], DDF ? xr[i] : 0.0f, DDF ? xg[i] : 0.0f,
                     DDF ? xb[i] : 0.0f, j, acc_a, acc_d, acc_e);
            SA[i] += acc_a;
            if constexpr (DDF) SD[i] += acc_d;
            if constexpr (MODE == EV_EXACT) EA[i] += acc_e;
        }
    } else {
        // member i is uniform across the wave: its data comes from LDS, its
        // partial sum goes to this thread's LDS slot; members j > i stay in
        // registers (static indices) behind a uniform guard
        const int tid = threadIdx.x;
#pragma nounroll
        for (int i = 0; i < N; ++i) {
            const int li = (ly + i / WIN) * LW + (lx + i % WIN);
            const float4 ui = sU[li];
            float xri = 0.0f, xgi = 0.0f, xbi = 0.0f;
            if constexpr (DDF) unpack_pixel(sP[li], u16, xri, xgi, xbi);
            float acc_a = 0.0f, acc_d = 0.0f, acc_e = 0.0f;
#pragma unroll
            for (int j = 1; j < N; ++j)
                if (j > i) pair(ui.x, ui.y, ui.z, xri, xgi, xbi, j, acc_a, acc_d, acc_e);
            int slot = 0;
            sT[(slot++ * N + i) * NT + tid] = acc_a;
            if constexpr (DDF) sT[(slot++ * N + i) * NT + tid] = acc_d;
            if constexpr (MODE == EV_EXACT) sT[(slot * N + i) * NT + tid] = acc_e;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            int slot = 0;
            SA[i] += sT[(slot++ * N + i) * NT + tid];
            if constexpr (DDF) SD[i] += sT[(slot++ * N + i) * NT + tid];
            if constexpr (MODE == EV_EXACT) EA[i] += sT[(slot * N + i) * NT + tid];
        }
    }

    // 4. criterion per member and its FP32 error bound
    float crit[N], cerr[N];
    const float pexp = p.kscale;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const float ea = (MODE == EV_EXACT) ? EA[i] + N * kU32 * SA[i]
                                            : (N - 1) * p.eta + (N * kU32 + p.rho) * SA[i];
        if constexpr (!DDF) {
            crit[i] = SA[i];
            cerr[i] = ea;
        } else {
            const float ed = (N + 2) * kU32 * SD[i];
            if (pexp == 0.5f) {
                crit[i] = SA[i] * SD[i];
                cerr[i] = SD[i] * ea + SA[i] * ed + 2.0f * kU32 * crit[i];
            } else {
                const float la = __log2f(SA[i]);
                const float ld = __log2f(SD[i]);
                crit[i] = (1.0f - pexp) * ld + pexp * la;
                cerr[i] = 1.4427f * ((1.0f - pexp) * ed / SD[i] + pexp * ea / SA[i]) +
                          4.0f * kU32 * fabsf(crit[i]) + 1e-6f;
            }
        }
    }

    // 5. argmin with the centre-first tie rule; runner-up over distinct vectors
    uint2 pk[N];
#pragma unroll
    for (int i = 0; i < N; ++i) pk[i] = sP[(ly + i / WIN) * LW + (lx + i % WIN)];
    float cb = crit[C], eb = cerr[C];
    uint2 pb = pk[C];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const bool lt = crit[i] < cb;
        cb = lt ? crit[i] : cb;
        eb = lt ? cerr[i] : eb;
        pb = lt ? pk[i] : pb;
    }
    float c2 = __builtin_inff(), e2 = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const bool take = !same_pixel(pk[i], pb) && crit[i] < c2;
        c2 = take ? crit[i] : c2;
        e2 = take ? cerr[i] : e2;
    }

    bool flag = false;
    if (valid) {
        store_pixel(p.dst + (int64_t)gy * p.dst_pitch, gx, pb, u16);
        // near tie (c2 is +inf when every member equals the selected vector),
        // a non-finite criterion, or a zero vector mixed with non-zero ones
        // (the FP32 chord does not encode the zero-vector convention)
        const bool fin = (cb == cb) && (cb > -__builtin_inff());
        const bool tie = (c2 < __builtin_inff()) && (c2 - cb <= eb + e2);
        flag = p.recheck && (!fin || tie || (anyzero && !allzero));
    }
    if (flag) {
        // members whose criterion may still be the minimum: crit_i - e_i <= best + e_best
        uint64_t cmask = ~0ull;
        if (MASKS && (cb == cb) && (cb > -__builtin_inff()) && !(anyzero && !allzero)) {
            cmask = 0ull;
            // widened by 8 ulps for the rounding of the test itself
            const float lim = cb + eb + 8.0f * kU32 * (fabsf(cb) + eb);
#pragma unroll
            for (int i = 0; i < N; ++i) cmask |= (crit[i] - cerr[i] <= lim) ? (1ull << i) : 0ull;
        }
        const uint32_t k = atomicAdd(&s_nflag, 1u);
        s_flags[k] = (uint32_t)(gy * p.W + gx);
        if constexpr (MASKS) s_masks[k] = cmask;
    }
    __syncthreads();

    // 6. one reservation in the re-check list for the whole workgroup
    publish_flags(p, s_flags, s_nflag, &s_base, threadIdx.x, NT, MASKS ? s_masks : nullptr);
}

template <int FILT, int WIN, int MODE, int NLO, int NHI>
__global__ __launch_bounds__(kTileX * angle_tile_y<WIN>()) void angle_kernel(const KParams p) {
    angle_tile<FILT, WIN, MODE, NLO, NHI>(p, xcd_tile(blockIdx.x, gridDim.x));
}

}  // namespace vf
