// Device building blocks of the window kernels (gfx950, wave64).
//
// Data flow of one workgroup (256 threads, output tile 64 x 4 pixels):
//   1. the (4 + 2r) x (64 + 2r) halo tile is read from HBM once (edge pixels
//      replicate, the border rule of the filters) and staged in LDS, together
//      with each pixel's per-pixel preparation (unit vector for the angle
//      criterion, packed integer channels for L1 / L2 / output);
//   2. each thread gathers its n = w^2 window members from LDS into registers
//      and scores the n(n-1)/2 unordered pairs once each, adding the pair
//      value to both members' sums (the symmetric half is never recomputed);
//   3. the per-member criterion, the selection (argmin with the centre-first
//      tie rule, or the weighted mean) and the write-out follow in registers;
//   4. windows whose decision is closer than the FP32 error bound are listed
//      in LDS and re-checked in FP64 by the same workgroup before it exits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "vf_internal.h"

namespace vf {

constexpr float kU32 = 5.9604645e-08f;            // 2^-24, unit roundoff of FP32
constexpr float kHalfPi = 1.57079632679489662f;
constexpr float kLn2 = 0.693147180559945309f;

__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Unit vector of a pixel in FP32 (w = 1 marks the zero vector). The squared
// norm nn is an exact integer in FP64; 1 / sqrt(nn) is the FP64 hardware
// reciprocal square root refined by two Newton steps y <- y (3 - nn y^2) / 2,
// each of which about squares the relative error, so it lies within a few FP64
// ulps of the exact value. Rounded to FP32, 2^29 times coarser, a component
// is therefore the correctly rounded r / |x| except where that lies within a
// few FP64 ulps of an FP32 rounding boundary, and its error stays below 2^-25
// plus that distance (the per-pair bounds assume 2^-24 per component).
__device__ __forceinline__ float4 unit_vector(uint32_t r, uint32_t g, uint32_t b) {
    const double nn = (double)r * r + (double)g * g + (double)b * b;
    if (!(nn > 0.0)) return make_float4(0.0f, 0.0f, 0.0f, 1.0f);
    const double h = 0.5 * nn;
    double y = __builtin_amdgcn_rsq(nn);
#pragma unroll
    for (int k = 0; k < 2; ++k) y *= fma(-h * y, y, 1.5);
    return make_float4((float)(r * y), (float)(g * y), (float)(b * y), 0.0f);
}

// Packed pixel: uint8 -> x = r | g << 8 | b << 16, y = 0;
//               uint16 -> x = r | g << 16, y = b.
__device__ __forceinline__ void load_pixel(const unsigned char* row, int x, int u16, uint32_t& r,
                                           uint32_t& g, uint32_t& b) {
    if (u16) {
        const uint16_t* p = reinterpret_cast<const uint16_t*>(row) + 3 * x;
        r = p[0];
        g = p[1];
        b = p[2];
    } else {
        const uint8_t* p = row + 3 * x;
        r = p[0];
        g = p[1];
        b = p[2];
    }
}

__device__ __forceinline__ uint2 pack_pixel(uint32_t r, uint32_t g, uint32_t b, int u16) {
    return u16 ? make_uint2(r | (g << 16), b) : make_uint2(r | (g << 8) | (b << 16), 0u);
}

__device__ __forceinline__ void unpack_pixel(uint2 v, int u16, float& r, float& g, float& b) {
    if (u16) {
        r = (float)(v.x & 0xffffu);
        g = (float)(v.x >> 16);
        b = (float)v.y;
    } else {
        r = (float)(v.x & 0xffu);
        g = (float)((v.x >> 8) & 0xffu);
        b = (float)(v.x >> 16);
    }
}

__device__ __forceinline__ void store_pixel(unsigned char* row, int x, uint2 v, int u16) {
    if (u16) {
        uint16_t* p = reinterpret_cast<uint16_t*>(row) + 3 * x;
        p[0] = (uint16_t)(v.x & 0xffffu);
        p[1] = (uint16_t)(v.x >> 16);
        p[2] = (uint16_t)v.y;
    } else {
        uint8_t* p = row + 3 * x;
        p[0] = (uint8_t)(v.x & 0xffu);
        p[1] = (uint8_t)((v.x >> 8) & 0xffu);
        p[2] = (uint8_t)(v.x >> 16);
    }
}

// WIDE: one 64-bit compare rather than two 32-bit ones and their
// combination. It changes the kernels' register allocation: the 7x7 DDF
// streaming kernel spills 92 instead of 532 B per lane with it (8192^2
// 16-bit: 29.4 -> 23.2 ms), while the VDF 5x5 / 7x7 streaming kernels, at
// their register limits, start or grow spilling, and the exact 7x7 VDF
// split-wave kernel slowed down: those keep the 32-bit form.
template <bool WIDE = true>
__device__ __forceinline__ bool same_pixel(uint2 a, uint2 b) {
    if constexpr (WIDE) return (((uint64_t)a.y << 32) | a.x) == (((uint64_t)b.y << 32) | b.x);
    return a.x == b.x && a.y == b.y;
}

// L1 distance of two packed pixels (exact integer, v_sad_u8 / v_sad_u16).
__device__ __forceinline__ uint32_t l1_dist(uint2 a, uint2 b, int u16) {
    if (u16) return __builtin_amdgcn_sad_u16(a.x, b.x, __builtin_amdgcn_sad_u16(a.y, b.y, 0u));
    return __builtin_amdgcn_sad_u8(a.x, b.x, 0u);
}

template <int N>
__device__ __forceinline__ float horner(const float* c, float x) {
    float acc = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) acc = fmaf(acc, x, c[k]);
    return acc;
}

// Estrin's scheme: pairs c_2i + c_2i+1 x, then pairs of those with x^2, x^4, ...
// (shorter dependency chains than Horner, one extra multiply per level).
template <int N>
__device__ __forceinline__ float estrin(const float* c, float x) {
    float v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = c[k];
    float xp = x;
#pragma unroll
    for (int n = N; n > 1; n = (n + 1) / 2) {
#pragma unroll
        for (int i = 0; i < n / 2; ++i) v[i] = fmaf(v[2 * i + 1], xp, v[2 * i]);
        if (n & 1) v[n / 2] = v[n - 1];
        xp = xp * xp;
    }
    return v[0];
}

// Polynomial evaluation variants of the angle kernels.
enum : int { VAR_HORNER = 0, VAR_ESTRIN = 1, VAR_F16 = 2 };

template <int N, int V>
__device__ __forceinline__ float poly(const float* c, float x) {
    if constexpr (V == VAR_ESTRIN) return estrin<N>(c, x);
    else return horner<N>(c, x);
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// Packed-FP16 variant of the chord approximant for two pairs at once:
// angle = s (c_0 + t), t = x q(x), x = s^2, q(x) = c_1 + c_2 x + ...; the
// correction t (at most 0.11 over the chord range) is evaluated with packed
// FP16 multiply-adds on both pairs; c_0 s and the final sum stay FP32. h holds
// c_1 .. c_{N-1} rounded to FP16.
template <int N>
__device__ __forceinline__ float2 chord_pair_f16(float s2a, float s2b, float c0, const half2_t* h) {
    const half2_t x = {(_Float16)s2a, (_Float16)s2b};
    half2_t q = h[N - 2];
#pragma unroll
    for (int k = N - 3; k >= 0; --k) q = __builtin_elementwise_fma(q, x, h[k]);   // one rounding each
    const half2_t t = q * x;
    const float sa = fsqrt(s2a), sb = fsqrt(s2b);
    return make_float2(sa * (c0 + (float)t.x), sb * (c0 + (float)t.y));
}

// The correction t(x) = sum_{k>=1} c_k x^k of a polynomial with NC
// coefficients (NC >= 2; 0: the runtime count n) at two arguments at once,
// in packed FP16: the arguments rounded to FP16, h[k - 1] = {c_k, c_k}
// (already FP16 values), Horner with one rounding per step. The caller adds
// c_0 in FP32.
template <int NC>
__device__ __forceinline__ float2 corr_pair_f16(float xa, float xb, const half2_t* h, int n) {
    const half2_t x = {(_Float16)xa, (_Float16)xb};
    half2_t q;
    if constexpr (NC >= 2) {
        q = h[NC - 2];
#pragma unroll
        for (int k = NC - 3; k >= 0; --k) q = __builtin_elementwise_fma(q, x, h[k]);
    } else {
        q = h[n - 2];
        for (int k = n - 3; k >= 0; --k) q = __builtin_elementwise_fma(q, x, h[k]);
    }
    const half2_t t = q * x;
    return make_float2((float)t.x, (float)t.y);
}

// Horner with a runtime coefficient count (per-member functions only).
__device__ __forceinline__ float horner_n(const float* c, int n, float x) {
    float acc = 0.0f;
#pragma unroll
    for (int k = kMaxCoef - 1; k >= 0; --k)
        if (k < n) acc = fmaf(acc, x, c[k]);
    return acc;
}

// The angle between two unit vectors from their squared chord s2 = |u_i - u_j|^2
// = 2 (1 - z) (z the cosine; s2 <= 2 for non-negative RGB vectors).
//   EV_EXACT: acosf of the cosine 1 - s2/2 (Section 3.1 definition).
//   EV_PAPER: Table 1 two-piece form, z < 0.5 -> P_lo(z), else P_hi(tau) with
//             tau = sqrt(1 - z) = sqrt(s2 / 2) (Section 3.1).
//   EV_SPLIT: z >= 0.5 (s2 <= 1) -> s U(s2), s = sqrt(s2) (odd chord fit);
//             else pi/2 - z L(z^2) (odd asin fit).
//   EV_CHORD: s U(s2), one odd chord fit over z in [0, 1].
template <int MODE, int NLO, int NHI, int V = VAR_HORNER>
__device__ __forceinline__ float angle_from_s2(float s2, const float* lo, const float* hi) {
    if constexpr (MODE == EV_EXACT) {
        float z = fmaf(-0.5f, s2, 1.0f);
        return acosf(fmaxf(z, -1.0f));
    } else if constexpr (MODE == EV_PAPER) {
        float tau = fsqrt(0.5f * s2);
        float up = poly<NHI, V>(hi, tau);
        float z = fmaf(-0.5f, s2, 1.0f);
        float dn = poly<NLO, V>(lo, z);
        return s2 <= 1.0f ? up : dn;
    } else if constexpr (MODE == EV_SPLIT) {
        float s = fsqrt(s2);
        float up = s * poly<NHI, V>(hi, s2);
        float z = fmaf(-0.5f, s2, 1.0f);
        float mid = fmaf(-z, poly<NLO, V>(lo, z * z), kHalfPi);
        return s2 <= 1.0f ? up : mid;
    } else {
        float s = fsqrt(s2);
        return s * poly<NHI, V>(hi, s2);
    }
}

// Horner with a compile-time coefficient count NC, or the runtime count n
// when NC = 0.
template <int NC>
__device__ __forceinline__ float horner_k(const float* c, int n, float x) {
    if constexpr (NC > 0) return horner<NC>(c, x);
    else return horner_n(c, n, x);
}

// Call f(std::integral_constant<int, NC>) with NC = n for the coefficient
// counts the exp and ENT approximants use (3 .. 10), else NC = 0 (runtime
// count): callers hoist this uniform switch out of their member loops.
template <class F>
__device__ __forceinline__ auto with_coef_count(int n, F&& f) {
    switch (n) {
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 9: return f(std::integral_constant<int, 9>{});
    case 10: return f(std::integral_constant<int, 10>{});
    default: return f(std::integral_constant<int, 0>{});
    }
}

// K(z) of the AMNFE kernel with the Section 3.2 cutoff (0 above T).
//   EV_EXACT:   expf(-z)
//   EV_PAPER:   the Table 3 rational c(z) / d(z)
//   EV_MINIMAX: the polynomial c(z) (the Table 2 ones and the minimax fits)
template <int MODE, int NC = 0>
__device__ __forceinline__ float kernel_exp(float z, const float* c, int n, const float* d, int nd,
                                            float cutoff) {
    float k;
    if constexpr (MODE == EV_EXACT) k = expf(-z);
    else if constexpr (MODE == EV_PAPER) k = horner_k<NC>(c, n, z) / horner_k<NC>(d, nd, z);
    else k = horner_k<NC>(c, n, z);
    return z > cutoff ? 0.0f : k;
}

// ENT(P) = P ln P of Section 3.3, 0 below the cutoff T (and at 0).
//   EV_EXACT:   P logf(P)
//   EV_PAPER:   Table 4 rational (T >= 0.05)
//   EV_MINIMAX: P = m 2^e (m in [1, 2)): P (e ln 2 + q(m - 1))
// NC: compile-time coefficient count of lo (and, for the rational, of hi), or 0.
template <int MODE, int NC = 0>
__device__ __forceinline__ float ent(float P, const float* lo, int n_lo, const float* hi, int n_hi,
                                     float cutoff) {
    if constexpr (MODE == EV_EXACT) {
        return (P > 0.0f && P >= cutoff) ? P * logf(P) : 0.0f;
    } else if constexpr (MODE == EV_PAPER) {
        float v = horner_k<NC>(lo, n_lo, P) / horner_k<NC>(hi, n_hi, P);
        return P < cutoff ? 0.0f : v;
    } else {
        int e;
        float m = frexpf(P, &e);          // P = m 2^e, m in [0.5, 1)
        float t = fmaf(m, 2.0f, -1.0f);   // 2m - 1 in [0, 1), exact
        float ln = fmaf((float)(e - 1), kLn2, horner_k<NC>(lo, n_lo, t));
        return (P > 0.0f && P >= cutoff) ? P * ln : 0.0f;
    }
}

// Workgroups of a launch are handed to the 8 XCDs round-robin (block b to XCD
// b mod 8). Renumber them so that each XCD works on one contiguous range of
// tiles: neighbouring tiles share the cache lines of their halo columns, and
// only the L2 of one XCD then fetches them. A bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
    constexpr int kXcds = 8;
    const int q = n / kXcds, r = n % kXcds;
    const int x = b % kXcds, i = b / kXcds;
    return x * q + min(x, r) + i;
}

// Tile coordinates of this workgroup.
__device__ __forceinline__ void tile_origin(const KParams& p, int t, int& tx0, int& ty0) {
    const int ty = t / p.tiles_x;
    ty0 = ty * kTileY;
    tx0 = (t - ty * p.tiles_x) * kTileX;
}

}  // namespace vf
