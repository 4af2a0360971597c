// Streaming window kernels of all four filters: every pixel pair scored once
// per image.
//
// A window's member sums S_i = sum_j c(x_i, x_j) (c = the pair criterion:
// the angle A for VDF, plus the Euclidean distance for DDF; the exact L1
// distance for AMNFE, the Euclidean distance for EVMF's vector median) share most of
// their pairs with the neighbouring windows: two pixels at offset (dy, dx)
// with |dy|, |dx| < w lie together in (w - |dy|)(w - |dx|) windows. Scoring
// each such pair once instead of once per window cuts the pair evaluations
// per output pixel from n(n-1)/2 = 36 / 300 / 1176 to 2w(w-1) = 12 / 40 / 84
// for w = 3 / 5 / 7.
//
// Organisation (one wavefront per workgroup):
//   * the wave owns 64 consecutive image columns (lane = column) and walks
//     down a strip of rows; its 64 - 2r middle lanes produce outputs, the r
//     lanes at each side are the horizontal halo;
//   * when input row y arrives, each lane normalises its pixel into an LDS
//     ring of the last w rows and scores its "backward" pairs one row at a
//     time: the 2w - 1 pixels within +-(w - 1) columns of each of the w - 1
//     rows above, then the w - 1 pixels to its left in row y (2w(w - 1)
//     pairs); each row's pair values go through a small LDS plane;
//   * each output lane keeps the w x w member sums of its current window and,
//     per member, its sums against the rows above it (w^2(w-1)/2 values) in
//     registers. Sliding the window down one row drops each kept member's
//     sum that involves the leaving row (nothing is subtracted), then adds
//     the new row: its members' sums are assembled from the pair planes, and
//     the same pair values are added to the kept members they touch.
// Member sums therefore hold pair values of the current window only, and the
// FP32 error bound used for flagging is relative to those sums. Flagged
// windows are collected in LDS and published to the re-check list in blocks
// (one atomic reservation per block), with the mask of the members that may
// still be the minimum where the kernel forms one (writes_masks). The strip
// height comes from the host (sized from the kernel's residency per call).
#pragma once

#include "batch.h"
#include "kern_common.h"
#include "recheck_dev.h"

namespace vf {

// backward offset o of a pixel: o < w - 1: same row, dx = o - (w - 1);
// otherwise row dy = -(1 + (o - (w-1)) / (2w - 1)), dx = (o - (w-1)) % (2w - 1) - (w - 1)
template <int WIN>
constexpr int stream_nb() { return 2 * WIN * (WIN - 1); }
template <int WIN>
constexpr int boff_dy(int o) { return o < WIN - 1 ? 0 : -(1 + (o - (WIN - 1)) / (2 * WIN - 1)); }
template <int WIN>
constexpr int boff_dx(int o) {
    return o < WIN - 1 ? o - (WIN - 1) : (o - (WIN - 1)) % (2 * WIN - 1) - (WIN - 1);
}
template <int WIN>
constexpr int boff_index(int dy, int dx) {
    return dy == 0 ? dx + (WIN - 1) : (WIN - 1) + (-dy - 1) * (2 * WIN - 1) + (dx + WIN - 1);
}

// Step loop unrolled by the window height: for the VDF 3x3 and 5x5 kernels
// (measured 2% faster at 5x5; larger windows and DDF would grow the code or
// the register state beyond what pays).
template <int FILT, int WIN, int MODE>
constexpr bool stream_unrolled() {
    return stream_unrolled_cfg(FILT, WIN, MODE);
}

template <int FILT, int MODE>
constexpr int stream_k() {
    const bool angle = FILT == VF_FILTER_VDF || FILT == VF_FILTER_DDF;
    return 1 + (FILT == VF_FILTER_DDF ? 1 : 0) + (angle && MODE == EV_EXACT ? 1 : 0);
}

// The AMNFE and EVMF outputs below read the window's member sums from LDS
// (sS[i * 64], this lane's column; written just before) and its members from
// the pixel ring through member(j, b), with loops over the window rows kept
// rolled: the register file then holds only the streaming state.

// AMNF output from the window's exact L1 member sums S1 (Section 3.2; the
// same arithmetic as the per-window kernel, kern_amnfe.h): with r_i =
// n^(kappa/3) / S1_i the EXP argument z_i = L1(x_C, x_i) r_i (exponential
// kernel) or 0.5 |x_C - x_i|_2^2 r_i^2 (Gaussian kernel, GAUSS), w_i =
// K(z_i) / S1_i^3, the mean relative to x_C, rounded with floor(v + 0.5).
// Returns whether a channel lies within the FP32 error bound of a rounding
// boundary (p.wbound: the relative error of one weight), or an argument lies
// within p.zband of the cutoff, where K jumps. FP32 approximants (Horner
// polynomial, Table 3 rational): p.rho is a relative bound of every weight
// (the evaluation bound of K over its least value), which moves the mean by at
// most rho (sum w |d| / sum w + |y - x_C|). V = VAR_F16: K = c_0 + t(z) with
// the correction t evaluated for two members at once in packed FP16; its
// absolute error bound p.rho enters the flagging bound through
// |dy| <= rho (sum rs^3 |d| + |y - x_C| sum rs^3) / (den - rho sum rs^3).
template <int WIN, int MODE, int V, bool GAUSS, class Member>
__device__ __forceinline__ bool amnfe_finish(const KParams& p, const float* sS, Member&& member, int oy, int ox) {
    constexpr bool F16 = V == VAR_F16;
    constexpr bool RW = !F16 && MODE != EV_EXACT;   // relative weight bound p.rho enters the flag
    constexpr int N = WIN * WIN;
    constexpr int R = (WIN - 1) / 2;
    const int u16 = p.u16;
    const uint2 pc = member(R, R);
    uint2 out = pc;
    bool flag = false;
    if (sS[0] != 0.0f) {   // S1_i = 0 for some i <=> uniform window -> x_C
        float cr, cg, cb;
        unpack_pixel(pc, u16, cr, cg, cb);
        // the EXP argument of a member from its reciprocal sum and its pixel
        auto arg = [&](float rs, uint2 q, float d0, float d1, float d2, int w16) -> float {
            if constexpr (GAUSS) {
                const float t = rs * p.kscale;
                return 0.5f * fmaf(d0, d0, fmaf(d1, d1, d2 * d2)) * (t * t);
            } else {
                return (float)l1_dist(pc, q, w16) * rs * p.kscale;
            }
        };
        float num0 = 0.0f, num1 = 0.0f, num2 = 0.0f, den = 0.0f;
        float ab0 = 0.0f, ab1 = 0.0f, ab2 = 0.0f;
        float fa0 = 0.0f, fa1 = 0.0f, fa2 = 0.0f, fb = 0.0f;   // FP16: sums of rs^3 |d| and rs^3
        // (u16_tag: the channel width as a constant, the test hoisted out of
        // the member loops)
        auto weights = [&](auto nc_tag, auto u16_tag) -> int {
            constexpr int NC = decltype(nc_tag)::value;
            constexpr int U16 = decltype(u16_tag)::value ? 1 : 0;
            if constexpr (F16) {
                const half2_t* h = reinterpret_cast<const half2_t*>(p.lo16);
#pragma unroll 1
                for (int j = 0; j < WIN; ++j) {
                    float zr[WIN], rr[WIN];
#pragma unroll
                    for (int b = 0; b < WIN; ++b) {
                        rr[b] = frcp(sS[(j * WIN + b) * 64]);
                        const uint2 q = member(j, b);
                        float xr, xg, xb;
                        unpack_pixel(q, u16, xr, xg, xb);
                        zr[b] = arg(rr[b], q, xr - cr, xg - cg, xb - cb, u16);
                    }
#pragma unroll
                    for (int b = 0; b < WIN; b += 2) {
                        const bool two = b + 1 < WIN;
                        const float2 t = corr_pair_f16<NC>(zr[b], two ? zr[b + 1] : 0.0f, h, p.n_lo);
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            if (e == 1 && !two) break;
                            const int bb = b + e;
                            const float k = zr[bb] > p.cutoff ? 0.0f : p.lo[0] + (e == 0 ? t.x : t.y);
                            const float r3 = rr[bb] * rr[bb] * rr[bb];
                            const float w = k * r3;
                            float xr, xg, xb;
                            unpack_pixel(member(j, bb), u16, xr, xg, xb);
                            const float d0 = xr - cr, d1 = xg - cg, d2 = xb - cb;
                            num0 = fmaf(w, d0, num0);
                            num1 = fmaf(w, d1, num1);
                            num2 = fmaf(w, d2, num2);
                            ab0 = fmaf(w, fabsf(d0), ab0);
                            ab1 = fmaf(w, fabsf(d1), ab1);
                            ab2 = fmaf(w, fabsf(d2), ab2);
                            den += w;
                            fa0 = fmaf(r3, fabsf(d0), fa0);
                            fa1 = fmaf(r3, fabsf(d1), fa1);
                            fa2 = fmaf(r3, fabsf(d2), fa2);
                            fb += r3;
                        }
                    }
                }
                return 0;
            }
#pragma unroll 1
            for (int j = 0; j < WIN; ++j) {
#pragma unroll
                for (int b = 0; b < WIN; ++b) {
                    const uint2 q = member(j, b);
                    const float rs = frcp(sS[(j * WIN + b) * 64]);
                    float xr, xg, xb;
                    unpack_pixel(q, U16, xr, xg, xb);
                    const float d0 = xr - cr, d1 = xg - cg, d2 = xb - cb;
                    const float z = arg(rs, q, d0, d1, d2, U16);
                    const float k = kernel_exp<MODE, NC>(z, p.lo, p.n_lo, p.hi, p.n_hi, p.cutoff);
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
            }
            return 0;
        };
        auto run = [&](auto nc_tag) -> int {
            if constexpr (F16) return weights(nc_tag, std::false_type{});   // (runtime width inside)
            else return u16 ? weights(nc_tag, std::true_type{}) : weights(nc_tag, std::false_type{});
        };
        if constexpr (MODE == EV_EXACT) run(std::integral_constant<int, 0>{});
        else with_coef_count(p.n_lo, run);
        if (p.zband > 0.0f) {
            // (only where the argument can reach the cutoff: large kappa) K jumps
            // at T, so an argument within its error bound of T is decided in FP64
#pragma unroll 1
            for (int j = 0; j < WIN; ++j) {
#pragma unroll
                for (int b = 0; b < WIN; ++b) {
                    const uint2 q = member(j, b);
                    float xr, xg, xb;
                    unpack_pixel(q, u16, xr, xg, xb);
                    const float z = arg(frcp(sS[(j * WIN + b) * 64]), q, xr - cr, xg - cg, xb - cb, u16);
                    flag |= fabsf(z - p.cutoff) <= p.zband;
                }
            }
        }
        const float maxv = u16 ? 65535.0f : 255.0f;
        const float inv = 1.0f / den;
        const float y[3] = {fmaf(num0, inv, cr), fmaf(num1, inv, cg), fmaf(num2, inv, cb)};
        const float ab[3] = {ab0 * inv, ab1 * inv, ab2 * inv};
        const float fa[3] = {fa0, fa1, fa2};
        const float dy[3] = {num0 * inv, num1 * inv, num2 * inv};
        const float fden = den - p.rho * fb;   // FP16: lower bound of the exact-K denominator
        if constexpr (F16) flag |= !(fden > 0.0f);
        uint32_t qv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float v = floorf(y[k] + 0.5f);
            const float frac = (y[k] + 0.5f) - v;
            float bound = (2.0f * p.wbound + 2.0f * N) * kU32 * ab[k] + 4.0f * kU32 * fabsf(y[k]) + 1e-6f;
            if constexpr (F16) bound += 1.01f * p.rho * (fa[k] + fabsf(dy[k]) * fb) / fden;
            if constexpr (RW) bound += 1.01f * p.rho * (ab[k] + fabsf(dy[k]));
            flag |= (frac < bound) || (1.0f - frac < bound);
            qv[k] = (uint32_t)fminf(fmaxf(v, 0.0f), maxv);
        }
        flag |= !(den > 0.0f);
        // an approximant that is not positive over the argument range (the
        // host's relative bound is then infinite): weights of either sign,
        // no FP32 bound holds, every window is decided in FP64
        if constexpr (RW) flag |= !(p.rho < 1e29f);
        out = pack_pixel(qv[0], qv[1], qv[2], u16);
    }
    store_pixel(p.dst + (int64_t)oy * p.dst_pitch, ox, out, u16);
    return flag;
}

// EVMF output (Section 3.3): the entropy switch P_C H + ENT(P_C) > 0 from the
// deviations n x_i - sum_j x_j (exact integers in FP32), in the same order and
// arithmetic as the per-window kernel (kern_evmf.h); where it switches, the
// vector median is the argmin of the window's L2 member sums S2 (centre
// first, then lowest index) with the runner-up over distinct vectors checked
// against the FP32 bound. V = VAR_F16: ln(1 + t) = c_0 + t(t) with the
// correction evaluated for two members at once in packed FP16; its absolute
// bound p.rho moves H by at most rho sum P_j = rho and ENT(P_C) by P_C rho,
// so the switching test by at most 2 P_C rho.
// memberf(j, b): the member's channels as floats (the pair phase's ring);
// wsum: the window's channel sums (exact integers).
template <int WIN, int MODE, int V, class Member, class MemberF, class StoreSums>
__device__ __forceinline__ bool evmf_finish(const KParams& p, float* sS, Member&& member, MemberF&& memberf,
                                            float3 wsum, StoreSums&& store_sums, int oy, int ox) {
    constexpr bool F16 = V == VAR_F16;
    constexpr int N = WIN * WIN;
    constexpr int R = (WIN - 1) / 2;
    constexpr int C = (N - 1) / 2;
    const int u16 = p.u16;
    const uint2 pc = member(R, R);
    const float sr = wsum.x, sg = wsum.y, sb = wsum.z;
    auto dev = [&](float4 x) -> float {
        const float a = fmaf((float)N, x.x, -sr);
        const float b = fmaf((float)N, x.y, -sg);
        const float c = fmaf((float)N, x.z, -sb);
        return fsqrt(fmaf(a, a, fmaf(b, b, c * c)));
    };
    // the deviations go to this lane's LDS column (the member sums are
    // written there only if the window switches)
    float D = 0.0f;
#pragma unroll 1
    for (int j = 0; j < WIN; ++j) {
#pragma unroll
        for (int b = 0; b < WIN; ++b) {
            const float d = dev(memberf(j, b));
            sS[(j * WIN + b) * 64] = d;
            D += d;
        }
    }
    uint2 out = pc;
    bool flag = false;
    if (D > 0.0f) {   // D = 0 <=> uniform window -> x_C
        const float invD = 1.0f / D;
        const float PC = sS[C * 64] * invD;
        float H = 0.0f, eC = 0.0f;
        // ENT jumps at the cutoff T (when T > 0), so a P_j within the FP32
        // error band of T may sit on the other side of it in exact arithmetic
        bool near_cut = false;
        const bool cut_on = p.cutoff > 0.0f;
        const float cut_band = 4.0f * (N + 4) * kU32 * p.cutoff;
        auto entropy = [&](auto nc_tag) -> int {
            constexpr int NC = decltype(nc_tag)::value;
            if constexpr (F16) {
                // P = m 2^e (m in [0.5, 1)): ENT = P ((e - 1) ln 2 + c_0 + t(2m - 1))
                const half2_t* h = reinterpret_cast<const half2_t*>(p.lo16);
                auto ent_pair = [&](float Pa, float Pb, float& ea, float& eb) {
                    int xa, xb;
                    const float ta = fmaf(frexpf(Pa, &xa), 2.0f, -1.0f);
                    const float tb = fmaf(frexpf(Pb, &xb), 2.0f, -1.0f);
                    const float2 c = corr_pair_f16<NC>(ta, tb, h, p.n_lo);
                    ea = (Pa > 0.0f && Pa >= p.cutoff) ? Pa * fmaf((float)(xa - 1), kLn2, p.lo[0] + c.x) : 0.0f;
                    eb = (Pb > 0.0f && Pb >= p.cutoff) ? Pb * fmaf((float)(xb - 1), kLn2, p.lo[0] + c.y) : 0.0f;
                    if (cut_on) near_cut |= (fabsf(Pa - p.cutoff) <= cut_band) || (fabsf(Pb - p.cutoff) <= cut_band);
                };
#pragma unroll 1
                for (int j = 0; j < WIN; ++j) {
                    float Pr[WIN];
#pragma unroll
                    for (int b = 0; b < WIN; ++b) Pr[b] = sS[(j * WIN + b) * 64] * invD;
#pragma unroll
                    for (int b = 0; b < WIN; b += 2) {
                        float ea, eb;
                        ent_pair(Pr[b], b + 1 < WIN ? Pr[b + 1] : 0.0f, ea, eb);
                        H -= ea;
                        if (b + 1 < WIN) H -= eb;
                    }
                }
                float unused;
                ent_pair(PC, 0.0f, eC, unused);
                return 0;
            }
#pragma unroll 1
            for (int j = 0; j < WIN; ++j) {
#pragma unroll
                for (int b = 0; b < WIN; ++b) {
                    const float Pm = sS[(j * WIN + b) * 64] * invD;
                    if (cut_on) near_cut |= fabsf(Pm - p.cutoff) <= cut_band;
                    H -= ent<MODE, NC>(Pm, p.lo, p.n_lo, p.hi, p.n_hi, p.cutoff);
                }
            }
            eC = ent<MODE, NC>(PC, p.lo, p.n_lo, p.hi, p.n_hi, p.cutoff);
            return 0;
        };
        // (the paper's rational has numerator and denominator of equal length)
        if constexpr (MODE == EV_EXACT) entropy(std::integral_constant<int, 0>{});
        else with_coef_count(p.n_lo, entropy);
        const float g = fmaf(PC, H, eC);
        float gb = 4.0f * (N + 4) * kU32 * (PC * (H + 2.0f) + fabsf(eC)) + 1e-7f;
        if constexpr (F16) gb += 2.01f * PC * p.rho;
        flag = fabsf(g) <= gb || near_cut;
        if (g > 0.0f) {
            store_sums();
            // one pass: the best (centre first, then lowest index) and the
            // runner-up over members distinct from the best so far (when the
            // best moves to a distinct vector, the old best, the least of those
            // seen, becomes the runner-up; when it moves to an equal one,
            // nothing changes)
            float best = sS[C * 64];
            uint2 pb = pc;
            float s2 = __builtin_inff();
#pragma unroll 1
            for (int j = 0; j < WIN; ++j) {
#pragma unroll
                for (int b = 0; b < WIN; ++b) {
                    const float v = sS[(j * WIN + b) * 64];
                    const uint2 q = member(j, b);
                    const bool diff = !same_pixel(q, pb);
                    const bool lt = v < best;
                    s2 = (lt && diff) ? best : ((!lt && diff) ? fminf(s2, v) : s2);
                    best = lt ? v : best;
                    pb = lt ? q : pb;
                }
            }
            // sums of n - 1 correctly rounded distances (row sums, then their
            // sum: additions only)
            flag |= (s2 < __builtin_inff()) && (s2 - best) <= (2.0f * N + 8.0f * WIN + 8.0f) * kU32 * (best + s2);
            out = pb;
        }
    }
    store_pixel(p.dst + (int64_t)oy * p.dst_pitch, ox, out, u16);
    return flag;
}

// The w sums out[k] = x[k] + ... + x[k + w - 1] (k = 0 .. w - 1) of 2w - 1
// values, without subtraction: every box holds the centre x[w - 1]; out[k] =
// (x[k] + .. + x[w - 2] + x[w - 1]) + (x[w] + .. + x[k + w - 1]), from the
// left suffix and the right prefix sums about the centre (4w - 6 additions).
template <int WIN>
__device__ __forceinline__ void box_sums(const float (&x)[2 * WIN - 1], float (&out)[WIN]) {
    constexpr int C = WIN - 1;
    float lsuf[WIN], rpre[WIN];   // lsuf[k] = x[k] + .. + x[C - 1]; rpre[k] = x[C + 1] + .. + x[C + k]
    lsuf[C - 1] = x[C - 1];
#pragma unroll
    for (int k = C - 2; k >= 0; --k) lsuf[k] = x[k] + lsuf[k + 1];
    rpre[1] = x[C + 1];
#pragma unroll
    for (int k = 2; k <= C; ++k) rpre[k] = rpre[k - 1] + x[C + k];
    out[0] = lsuf[0] + x[C];
    out[C] = x[C] + rpre[C];
#pragma unroll
    for (int k = 1; k < C; ++k) out[k] = (lsuf[k] + x[C]) + rpre[k];
}

// The streaming kernels run one wavefront per workgroup, whose LDS accesses
// are performed in program order: handing values between lanes within a step
// needs only that the compiler keep that order (wavefront-scope fences, no
// code), not a workgroup barrier with its wait for every LDS access in flight.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int FILT, int WIN, int MODE, int NLO, int NHI, int V = VAR_HORNER>
__device__ __forceinline__ void stream_tile(const KParams& p, const int tile) {
    static_assert(V == VAR_HORNER || MODE == EV_CHORD ||
                      (V == VAR_F16 && MODE == EV_MINIMAX &&
                       (is_amnf(FILT) || FILT == VF_FILTER_EVMF)),
                  "evaluation variants: chord angle (Estrin, FP16), minimax exp / ln (FP16)");
    constexpr bool F16 = (V == VAR_F16) && MODE == EV_CHORD;   // packed FP16 chord angles
    constexpr int R = (WIN - 1) / 2;
    constexpr int N = WIN * WIN;
    constexpr int C = (N - 1) / 2;
    constexpr int OUTW = 64 - 2 * R;
    constexpr bool DDF = (FILT == VF_FILTER_DDF);
    constexpr bool ANG = (FILT == VF_FILTER_VDF || DDF);   // angle filters
    constexpr bool AMN = is_amnf(FILT);                    // pair value: exact L1 distance
    constexpr bool EVM = (FILT == VF_FILTER_EVMF);         // pair value: L2 distance
    constexpr bool EXA = ANG && (MODE == EV_EXACT);
    constexpr bool WIDE_CMP = !(FILT == VF_FILTER_VDF && WIN >= 5);   // see same_pixel
    constexpr int K = stream_k<FILT, MODE>();   // quantities: angle [, distance] [, error]
    constexpr int KD = 1;                        // index of the distance
    constexpr int KE = DDF ? 2 : 1;              // index of the exact-mode error estimate
    constexpr int NB = stream_nb<WIN>();
    constexpr float kExactK = 1.1920929e-07f;    // 2^-23, see angle_kernel

    // rings of the last w rows, padded by w - 1 columns on each side so that
    // every lane's backward neighbours are addressable without clamping (the
    // edge lanes' out-of-strip pairs are never read by an output lane)
    constexpr int PAD = WIN - 1;
    constexpr int RW = 64 + 2 * PAD;
    // angle filters: unit vectors (w = 1 marks the zero vector); EVMF: the pixels as floats
    __shared__ float4 sU[(ANG || EVM) ? WIN : 1][(ANG || EVM) ? RW : 1];
    __shared__ float4 sF[DDF ? WIN : 1][DDF ? RW : 1];   // DDF: the pixels as floats
    __shared__ uint2 sP[WIN][RW];    // packed pixels
    constexpr int NDX = 2 * WIN - 1;
    // sC: this lane's pair values against one row, dx = -(w-1)..(w-1);
    // sS (AMNFE / EVMF): this step's member sums, read back only by the lane
    // that wrote them. The two are never live together within a step (the
    // wave's LDS accesses stay in program order), so they share storage: one
    // workgroup more per CU for the finishers' kernels.
    constexpr int SCS = (AMN || EVM) ? (N > K * NDX ? N : K * NDX) : K * NDX;
    __shared__ float sCS[SCS][64];
    float (*const sC)[NDX][64] = reinterpret_cast<float (*)[NDX][64]>(&sCS[0][0]);
    float (*const sS)[64] = sCS;
    static_assert(!EVM || N - 3 >= K * NDX, "EVMF column sums need three rows of sCS beyond the pair rows");
    // flagged windows held before publishing (a step adds at most 64; 96
    // keeps the 5x5 DDF kernel at two workgroups per SIMD within the LDS)
    constexpr int FCAP = 96;
    __shared__ uint32_t s_flags[FCAP];
    // candidate members of each flagged window (angle filters, not unrolled)
    constexpr bool MASKS = writes_masks(FILT, WIN, MODE, true);
    __shared__ uint64_t s_masks[MASKS ? FCAP : 1];
    __shared__ uint32_t s_base;

    // packed FP16 variant: c_1 .. c_{m-1} as FP16 pairs (exact: the host rounded them)
    half2_t h16[F16 ? NHI - 1 : 1];
    if constexpr (F16) {
#pragma unroll
        for (int k = 0; k < NHI - 1; ++k) h16[k] = half2_t{(_Float16)p.hi[k + 1], (_Float16)p.hi[k + 1]};
    }
    const int L = threadIdx.x;
    const int sx = tile % p.tiles_x;
    const int sy = tile / p.tiles_x;
    const int X = sx * OUTW - R;           // image column of lane 0
    const int Y0 = sy * p.strip_rows;      // first output row of the strip
    const int rows_out = min(p.strip_rows, p.H - Y0);
    const int gxl = min(max(X + L, 0), p.W - 1);
    const bool out_lane = (L >= R) && (L < 64 - R) && (X + L < p.W);
    const int u16 = p.u16;
    uint32_t nflag = 0u;   // wave-uniform
    auto flush = [&]() {
        publish_flags(p, s_flags, nflag, &s_base, L, 64, MASKS ? s_masks : nullptr);
        nflag = 0u;
    };

    // Window state per member (j, b): S[k][j][b], its sum against its own
    // row and the rows below, and Rk[k][j][b][jj] (jj < j) for the rows
    // above. Each step the window's top row leaves and every kept member's
    // Rk shifts down one, dropping the entry of the leaving row. Every sum
    // thus holds pair values of the current window only, and no pair value
    // is ever subtracted: the FP32 rounding stays relative to the window's
    // own sums. (Sliding one sum by subtracting the leaving row's partial
    // would leave in it the rounding of values from rows no longer in the
    // window, the padding rows above a strip's first row included.)
    // When a member enters (the window's last row), its sums against the
    // rows above become suffix sums, Rk[..][jj] over rows jj .. j - 1, so its
    // criterion sum is S + Rk[..][0]. (Keeping Rk[..][jj] as the sum against
    // row jj alone and adding them all at the output is the other exact form;
    // it measured slower in every kernel: 7x7 DDF 29 against 49 ms, 7x7 VDF
    // 9.7 against 9.2 ms at one wave per SIMD.)
    // Box-sum fold of the rows above (below): 4w - 6 additions per w box sums
    // instead of w (w - 1), for two more LDS hand-overs per row. Measured at
    // w = 7 (16-bit 8192^2 chord-11: VDF 12.9 -> 10.3 ms, DDF 23.3 -> 16.7 ms;
    // AMNFE / EVMF 4096^2 2.15 -> 1.65 ms, 4.00 -> 2.87 ms) and 1-3% faster at
    // w = 5 with the lane's own pair values kept in registers; at w = 3 it
    // saves nothing.
    constexpr bool BOXFOLD = WIN >= 5;
    float S[K][WIN][WIN];
    float Rk[K][WIN][WIN][WIN];    // Rk[k][j][b][jj]: member (j, b) against rows jj .. j - 1
    // member i's criterion sum of quantity k (i a constant after unrolling:
    // every index folds to a constant, registers, not private memory)
    auto msum = [&](int k, int i) -> float {
        const int j = i / WIN, b = i % WIN;
        return j > 0 ? S[k][j][b] + Rk[k][j][b][0] : S[k][j][b];
    };
    float4 colsum = make_float4(0.0f, 0.0f, 0.0f, 0.0f);   // EVMF: this column's channel sums over the ring
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int j = 0; j < WIN; ++j)
#pragma unroll
            for (int b = 0; b < WIN; ++b) {
                S[k][j][b] = 0.0f;
#pragma unroll
                for (int jj = 0; jj < j; ++jj) Rk[k][j][b][jj] = 0.0f;
            }

    // Every ring slot and pad starts as the zero pixel, so the pairs scored
    // against rows above the strip's first row during the first w - 1 steps
    // are finite; they enter only the state of members and rows that leave
    // the window before any output is formed.
    for (int c = L; c < RW; c += 64)
#pragma unroll
        for (int j = 0; j < WIN; ++j) {
            if constexpr (ANG || EVM) sU[j][c] = make_float4(0.0f, 0.0f, 0.0f, ANG ? 1.0f : 0.0f);
            if constexpr (DDF) sF[j][c] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            sP[j][c] = make_uint2(0u, 0u);
        }
    __syncthreads();
    uint32_t zero_rows = 0u;   // bit j: a zero pixel among the wave's pixels of ring row j
    const int steps = rows_out + WIN - 1;
    // one step: input row t arrives in ring slot rs = t mod w
    auto step = [&](const int t, const int rs) {
        // ---- 1. new input row into the ring
        {
            const int gy = min(max(Y0 - R + t, 0), p.H - 1);
            uint32_t r, g, b;
            load_pixel(p.src + (int64_t)gy * p.src_pitch, gxl, u16, r, g, b);
            sP[rs][L + PAD] = pack_pixel(r, g, b, u16);
            if constexpr (ANG) {
                const bool z = (r | g | b) == 0u;
                zero_rows = (zero_rows & ~(1u << rs)) | (__any(z) ? (1u << rs) : 0u);
                sU[rs][L + PAD] = unit_vector(r, g, b);
                if constexpr (DDF) {
                    float fr, fg, fb;
                    unpack_pixel(sP[rs][L + PAD], u16, fr, fg, fb);
                    sF[rs][L + PAD] = make_float4(fr, fg, fb, 0.0f);
                }
            } else if constexpr (EVM) {
                float fr, fg, fb;
                unpack_pixel(sP[rs][L + PAD], u16, fr, fg, fb);
                // this column's channel sums over the ring's w rows: the row
                // leaving the ring out, the new row in (exact integers)
                const float4 old = sU[rs][L + PAD];
                colsum.x += fr - old.x;
                colsum.y += fg - old.y;
                colsum.z += fb - old.z;
                sU[rs][L + PAD] = make_float4(fr, fg, fb, 0.0f);
                // published in the last three rows of the finishers' LDS,
                // which the pair rows never reach and the finisher overwrites
                // only after reading them
                sCS[N - 3][L] = colsum.x;
                sCS[N - 2][L] = colsum.y;
                sCS[N - 1][L] = colsum.z;
            }
        }
        wave_sync();

        // ---- 2. shift the window state down one row (each kept member drops
        //         its sum that starts at the leaving row)
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int j = 0; j < WIN - 1; ++j)
#pragma unroll
                for (int b = 0; b < WIN; ++b) {
                    S[k][j][b] = S[k][j + 1][b];
#pragma unroll
                    for (int jj = 0; jj < j; ++jj) Rk[k][j][b][jj] = Rk[k][j + 1][b][jj + 1];
                }
#pragma unroll
            for (int a = 0; a < WIN; ++a) S[k][WIN - 1][a] = 0.0f;
        }

        // ---- 3. one row at a time (the w - 1 rows above, then the new row
        //         itself): score this lane's pixel against that row's pixels
        //         within +-(w-1) columns, then fold the pair values of the
        //         window's new members into the sums
        float4 me = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if constexpr (ANG || EVM) me = sU[rs][L + PAD];
        const uint2 mp = sP[rs][L + PAD];
        float4 mf = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if constexpr (DDF) mf = sF[rs][L + PAD];
#pragma unroll
        for (int js = 0; js < WIN; ++js) {
            const int dy = js - (WIN - 1);          // -(w-1) .. 0
            const int qs = (rs + WIN + dy) % WIN;
            constexpr int dummy = 0;
            (void)dummy;
            const int ndx = (dy == 0) ? WIN - 1 : NDX;   // same row: only the pixels to the left
            // this lane's pair values go to its LDS column and, for the box-sum
            // fold, stay in registers as well
            float pv[K][NDX];
            auto put = [&](int k, int o, float v) {
                sC[k][o][L] = v;
                pv[k][o] = v;
            };
            if constexpr (F16) {
                // squared chords in FP32, then the angles two at a time
                float s2v[NDX + 1];
#pragma unroll
                for (int o = 0; o < NDX; ++o) {
                    if (o >= ndx) break;
                    const float4 uq = sU[qs][L + PAD + o - (WIN - 1)];
                    const float ex = me.x - uq.x, ey = me.y - uq.y, ez = me.z - uq.z;
                    s2v[o] = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
                }
#pragma unroll
                for (int o = 0; o < NDX; o += 2) {
                    if (o >= ndx) break;
                    const bool two = o + 1 < ndx;
                    const float2 th = chord_pair_f16<NHI>(s2v[o], two ? s2v[o + 1] : 0.0f, p.hi[0], h16);
                    put(0, o, th.x);
                    if (two) put(0, o + 1, th.y);
                }
            }
#pragma unroll
            for (int o = 0; o < NDX; ++o) {
                if (o >= ndx) break;
                const int dx = o - (WIN - 1);
                if constexpr (AMN) {
                    // exact integer; sums of these stay exact in FP32 (below 2^24)
                    put(0, o, (float)l1_dist(mp, sP[qs][L + PAD + dx], u16));
                    continue;
                }
                if constexpr (EVM) {
                    const float4 q = sU[qs][L + PAD + dx];
                    const float er = me.x - q.x, eg = me.y - q.y, eb = me.z - q.z;
                    put(0, o, fsqrt(fmaf(er, er, fmaf(eg, eg, eb * eb))));
                    continue;
                }
                const float4 uq = sU[qs][L + PAD + dx];
                const float ex = me.x - uq.x, ey = me.y - uq.y, ez = me.z - uq.z;
                const float s2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
                if constexpr (!F16) put(0, o, angle_from_s2<MODE, NLO, NHI, V>(s2, p.lo, p.hi));
                if constexpr (DDF) {
                    const float4 q = sF[qs][L + PAD + dx];
                    const float er = mf.x - q.x, eg = mf.y - q.y, eb = mf.z - q.z;
                    put(KD, o, fsqrt(fmaf(er, er, fmaf(eg, eg, eb * eb))));
                }
                if constexpr (EXA)
                    put(KE, o, s2 > 0.0f ? fmaf(kExactK, frsq(s2 + 5.9604645e-08f), 6.0e-7f) : 0.0f);
            }
            wave_sync();
            if (dy < 0 && BOXFOLD) {
                // new members a (lanes L - R + a) against row js of the window,
                // and the kept members b of row js against the new row, as box
                // sums: lane l forms the w sums of w consecutive values of its
                // backward pair values v_l[o] (its own pixel against row js,
                // dx = o - (w-1)) and of its forward values f_l[e] =
                // v_{l+d}[w-1-d], d = e - (w-1) (row js's pixel against the new
                // row); new member a takes B_{w-1-a} of lane L - R + a and kept
                // member b adds F_{w-1-b} of lane L - R + b. Each box shares
                // the centre value e = w - 1 and is (left suffix + centre) +
                // right prefix, so no value outside a box enters its sum.
                float Bx[K][WIN], Fx[K][WIN];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    float v[NDX], f[NDX];
#pragma unroll
                    for (int e = 0; e < NDX; ++e) {
                        v[e] = pv[k][e];
                        f[e] = sC[k][NDX - 1 - e][min(max(L + e - (WIN - 1), 0), 63)];
                    }
                    box_sums<WIN>(v, Bx[k]);
                    box_sums<WIN>(f, Fx[k]);
                }
                // (every lane has read the plane before it is overwritten)
                wave_sync();
                // published sums: plane (k < R ? k : k - 1) for B_k, and w - 1
                // more for F_k; B_R and F_R stay with their lane
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int c = 0; c < WIN; ++c) {
                        if (c == R) continue;
                        const int pl = c < R ? c : c - 1;
                        sC[k][pl][L] = Bx[k][c];
                        sC[k][WIN - 1 + pl][L] = Fx[k][c];
                    }
                wave_sync();
#pragma unroll
                for (int a = 0; a < WIN; ++a) {
                    const int la = min(max(L - R + a, 0), 63);
                    const int c = WIN - 1 - a;
                    const int pl = c < R ? c : c - 1;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        Rk[k][WIN - 1][a][js] = a == R ? Bx[k][c] : sC[k][pl][la];
                        S[k][js][a] += a == R ? Fx[k][c] : sC[k][WIN - 1 + pl][la];
                    }
                }
            } else if (dy < 0) {
                // new members a (lanes L - R + a) against row js of the window
#pragma unroll
                for (int a = 0; a < WIN; ++a) {
                    const int la = min(max(L - R + a, 0), 63);
                    float racc[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) racc[k] = 0.0f;
#pragma unroll
                    for (int b = 0; b < WIN; ++b) {
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            const float cv = sC[k][b - a + WIN - 1][la];
                            racc[k] += cv;
                            S[k][js][b] += cv;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k) Rk[k][WIN - 1][a][js] = racc[k];
                }
            } else {
                // pairs inside the new row
#pragma unroll
                for (int a = 1; a < WIN; ++a) {
                    const int la = min(max(L - R + a, 0), 63);
#pragma unroll
                    for (int b = 0; b < a; ++b) {
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            const float cv = sC[k][b - a + WIN - 1][la];
                            S[k][WIN - 1][a] += cv;
                            S[k][WIN - 1][b] += cv;
                        }
                    }
                }
            }
            wave_sync();
        }
        // the new members' row sums become suffix sums (rows jj .. w - 2)
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int a = 0; a < WIN; ++a)
#pragma unroll
                for (int jj = WIN - 3; jj >= 0; --jj) Rk[k][WIN - 1][a][jj] += Rk[k][WIN - 1][a][jj + 1];

        // ---- 4. output: the window with rows t - w + 1 .. t is complete
        if (t >= WIN - 1) {
            const int oy = Y0 + t - (WIN - 1);
            bool flag = false;
            uint64_t cmask = ~0ull;   // candidate members of a flagged window
            if (out_lane && oy < p.H) {
                // member i sits in ring slot (t - (w-1) + i / w) % w, column L - R + i % w
                const int slot0 = rs + 1 == WIN ? 0 : rs + 1;   // ring slot of the window's top row
                auto member = [&](int i) -> uint2 {
                    const int j = i / WIN;
                    const int slot = slot0 + j >= WIN ? slot0 + j - WIN : slot0 + j;
                    return sP[slot][L - R + (i - j * WIN) + PAD];
                };
                if constexpr (AMN || EVM) {
                    // the rolled finishers read this lane's member sums from LDS
                    auto store_sums = [&]() {
#pragma unroll
                        for (int i = 0; i < N; ++i) sS[i][L] = msum(0, i);
                    };
                    auto member2 = [&](int j, int b) -> uint2 {
                        const int slot = slot0 + j >= WIN ? slot0 + j - WIN : slot0 + j;
                        return sP[slot][L - R + b + PAD];
                    };
                    if constexpr (AMN) {
                        store_sums();
                        flag = amnfe_finish<WIN, MODE, V, FILT == VF_FILTER_AMNFG>(p, &sS[0][L], member2, oy, X + L);
                    } else {
                        auto member2f = [&](int j, int b) -> float4 {
                            const int slot = slot0 + j >= WIN ? slot0 + j - WIN : slot0 + j;
                            return sU[slot][L - R + b + PAD];
                        };
                        // the window's channel sums: the w column sums around this lane
                        float3 wsum = make_float3(0.0f, 0.0f, 0.0f);
#pragma unroll
                        for (int b = 0; b < WIN; ++b) {
                            wsum.x += sCS[N - 3][L - R + b];
                            wsum.y += sCS[N - 2][L - R + b];
                            wsum.z += sCS[N - 1][L - R + b];
                        }
                        flag = evmf_finish<WIN, MODE, V>(p, &sS[0][L], member2, member2f, wsum, store_sums, oy,
                                                         X + L);
                    }
                } else {
                // criterion and its FP32 error bound e_i = e0 + e1 * crit_i (+ e2_i)
                // 7x7 DDF selects in one pass over the members (below): its
                // two sums per member leave no room for per-member arrays
                // (spills 207 -> 113, 4096^2 kernel 7.9 -> 6.4 ms); the other
                // kernels keep the arrays (5x5 DDF measured 4% faster with them)
                constexpr bool ONEPASS = DDF && WIN == 7;
                constexpr int NA = ONEPASS ? 1 : N;
                float crit[NA], cerr[NA];
                const float pexp = p.kscale;
                constexpr float kSum0 = (N + 4 * WIN) * kU32;
                const float kSum = kSum0 + p.rho;   // summation + relative per-pair term
                // (DDF: the exponent test is uniform; it selects one of two
                // straight-line member loops rather than branching per member)
                auto crit_err = [&](auto half_tag, float sa, float sd, float se, float& c, float& e) {
                    constexpr bool HALF = decltype(half_tag)::value;
                    const float ea = (EXA ? se : (N - 1) * p.eta) + kSum * sa;
                    if constexpr (!DDF) {
                        c = sa;
                        e = ea;
                    } else {
                        const float ed = (kSum0 + 2.0f * kU32) * sd;
                        if constexpr (HALF) {
                            c = sa * sd;
                            e = sd * ea + sa * ed + 2.0f * kU32 * c;
                        } else {
                            const float la2 = __log2f(sa);
                            const float ld2 = __log2f(sd);
                            c = (1.0f - pexp) * ld2 + pexp * la2;
                            e = 1.4427f * ((1.0f - pexp) * ed / sd + pexp * ea / sa) + 4.0f * kU32 * fabsf(c) +
                                1e-6f;
                        }
                    }
                };
                auto se_of = [&](int i) -> float {
                    if constexpr (EXA) return msum(KE, i);
                    else return 0.0f;
                };
                constexpr bool AFFINE = !DDF && !EXA;   // cerr = e0 + kSum * crit
                float cb, eb, c2 = __builtin_inff(), e2 = 0.0f;
                bool near_tie = false;   // (threshold form of the tie test)
                uint2 pb;
                // zero vectors mixed with non-zero ones are flagged too; the
                // test runs as a scan of its own, only when a ring row of the
                // wave holds a zero pixel (folded into the selection passes
                // the compiler evaluates it for every window, two operations
                // per member)
                bool anyzero = false, allzero = true;
                const bool check_zero = zero_rows != 0u;
                auto zero_scan = [&]() {
                    if (check_zero) {
#pragma unroll
                        for (int i = 0; i < N; ++i) {
                            const uint2 q = member(i);
                            const bool z = (q.x | q.y) == 0u;
                            anyzero |= z;
                            allzero &= z;
                        }
                    }
                };
                auto sd_of = [&](int i) -> float {
                    if constexpr (DDF) return msum(KD, i);
                    else return 0.0f;
                };
                if constexpr (!ONEPASS) {
                    auto all_crit = [&](auto half_tag) {
#pragma unroll
                        for (int i = 0; i < N; ++i)
                            crit_err(half_tag, msum(0, i), sd_of(i), se_of(i), crit[i], cerr[i]);
                    };
                    if (!DDF || pexp == 0.5f) all_crit(std::true_type{});
                    else all_crit(std::false_type{});
                    // argmin (centre first, then lowest index) by index; the
                    // selected pixel is read back from the ring
                    cb = crit[C];
                    eb = cerr[C];
                    int bi = C;
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        const bool lt = crit[i] < cb;
                        cb = lt ? crit[i] : cb;
                        if constexpr (!AFFINE) eb = lt ? cerr[i] : eb;
                        bi = lt ? i : bi;
                    }
                    pb = member(bi);
                    // (threshold form for the kernels without candidate masks:
                    // one compare less per member; the 7x7 kernel keeps the
                    // runner-up, whose spills grew with the other form)
                    if constexpr (AFFINE && !MASKS) {
                        // a member distinct from the selected vector ties when
                        // crit_i - cb <= eb + e_i, e_i = E0 + kSum crit_i, i.e.
                        // crit_i <= (cb + eb + E0) / (1 - kSum); the threshold
                        // takes 1 + kSum + 2 kSum^2 >= 1 / (1 - kSum) (kSum <= 1/2)
                        // and 4 ulps for its own rounding, so it flags every
                        // window the runner-up test would (a bound of kSum > 1/2
                        // flags every window with two distinct vectors)
                        const float e0 = (N - 1) * p.eta;
                        eb = e0 + kSum * cb;
                        const float thr = kSum <= 0.5f
                                              ? (cb + eb + e0) * (1.0f + fmaf(2.0f * kSum, kSum, kSum) + 4.0f * kU32)
                                              : __builtin_inff();
#pragma unroll
                        for (int i = 0; i < N; ++i) {
                            const uint2 q = member(i);
                            near_tie |= !same_pixel<WIDE_CMP>(q, pb) && crit[i] <= thr;
                        }
                    } else {
                        // runner-up over members distinct from the selected vector
#pragma unroll
                        for (int i = 0; i < N; ++i) {
                            const uint2 q = member(i);
                            const bool take = !same_pixel<WIDE_CMP>(q, pb) && crit[i] < c2;
                            c2 = take ? crit[i] : c2;
                            if constexpr (!AFFINE) e2 = take ? cerr[i] : e2;
                        }
                        if constexpr (AFFINE) {
                            eb = (N - 1) * p.eta + kSum * cb;
                            e2 = (N - 1) * p.eta + kSum * c2;
                        }
                    }
                } else {
                    // one pass, no per-member arrays: the best (centre first,
                    // then lowest index) and the runner-up over members distinct
                    // from the best so far (when the best moves to a distinct
                    // vector, the old best, the least of those seen, becomes the
                    // runner-up; when it moves to an equal one, nothing changes)
                    auto pass = [&](auto half_tag) {
                        crit_err(half_tag, msum(0, C), sd_of(C), se_of(C), cb, eb);
                        pb = member(C);
#pragma unroll
                        for (int i = 0; i < N; ++i) {
                            float c, e;
                            crit_err(half_tag, msum(0, i), sd_of(i), se_of(i), c, e);
                            const uint2 q = member(i);
                            const bool diff = !same_pixel<WIDE_CMP>(q, pb);
                            const bool lt = c < cb;
                            const bool old_up = lt && diff;
                            const bool new_up = !lt && diff && c < c2;
                            c2 = old_up ? cb : (new_up ? c : c2);
                            e2 = old_up ? eb : (new_up ? e : e2);
                            cb = lt ? c : cb;
                            eb = lt ? e : eb;
                            pb = lt ? q : pb;
                        }
                    };
                    if (!DDF || pexp == 0.5f) pass(std::true_type{});
                    else pass(std::false_type{});
                }
                zero_scan();
                const bool zero_mix = anyzero && !allzero;
                store_pixel(p.dst + (int64_t)oy * p.dst_pitch, X + L, pb, u16);
                if (p.recheck) {
                    const bool fin = (cb == cb) && (cb > -__builtin_inff());
                    // c2 stays +inf when every member equals the selected vector
                    const bool tie = near_tie || ((c2 < __builtin_inff()) && (c2 - cb <= eb + e2));
                    flag = !fin || tie || zero_mix;
                    if (MASKS && flag && fin && !zero_mix) {
                        // members whose criterion may still be the minimum:
                        // crit_i - e_i <= best + e_best, widened by 8 ulps for
                        // the rounding of this test.
                        cmask = 0ull;
                        const float lim = cb + eb + 8.0f * kU32 * (fabsf(cb) + eb);
                        if constexpr (!ONEPASS) {
#pragma unroll
                            for (int i = 0; i < N; ++i) cmask |= (crit[i] - cerr[i] <= lim) ? (1ull << i) : 0ull;
                        } else {
                            auto mask_pass = [&](auto half_tag) {
#pragma unroll
                                for (int i = 0; i < N; ++i) {
                                    float c, e;
                                    crit_err(half_tag, msum(0, i), sd_of(i), se_of(i), c, e);
                                    cmask |= (c - e <= lim) ? (1ull << i) : 0ull;
                                }
                            };
                            if (!DDF || pexp == 0.5f) mask_pass(std::true_type{});
                            else mask_pass(std::false_type{});
                        }
                    }
                }
                }
                flag = flag && p.recheck;
            }
            // wave-aggregated append to the LDS list; published when half full
            const unsigned long long mask = __ballot(flag);
            if (flag) {
                const unsigned long long below = mask & ((1ull << L) - 1ull);
                s_flags[nflag + (uint32_t)__popcll(below)] = (uint32_t)(oy * p.W + X + L);
                if constexpr (MASKS) s_masks[nflag + (uint32_t)__popcll(below)] = cmask;
            }
            nflag += (uint32_t)__popcll(mask);
            if (nflag > FCAP - 64) {
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                flush();
            }
        }
        wave_sync();
    };
    if constexpr (stream_unrolled<FILT, WIN, MODE>()) {
        // w steps per iteration: ring slots are constants and the shifts of the
        // window state become register renames
        for (int t0 = 0; t0 < steps; t0 += WIN) {
#pragma unroll
            for (int k = 0; k < WIN; ++k) {
                if (t0 + k >= steps) break;
                step(t0 + k, k);
            }
        }
    } else {
        for (int t = 0; t < steps; ++t) step(t, t % WIN);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (nflag != 0u) flush();
}

// Launch a single-image streaming kernel (one wave per workgroup), or, while
// the host has set occupancy_query(), store its resident workgroups per CU
// there and launch nothing (how the host sizes strips for a call).
template <class Kern>
inline void stream_launch(Kern kernel, const KParams& p, int blocks, void* stream) {
    if (int* q = occupancy_query()) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(q, kernel, 64, 0) != hipSuccess) *q = 0;
        return;
    }
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(64), 0, (hipStream_t)stream, p);
}

template <int FILT, int WIN, int MODE, int NLO, int NHI, int V = VAR_HORNER>
__global__ __launch_bounds__(64) void stream_kernel(const KParams p) {
    stream_tile<FILT, WIN, MODE, NLO, NHI, V>(p, xcd_tile(blockIdx.x, gridDim.x));
}

// Persistent batch form: workgroups pull strips of the class's images.
template <int FILT, int WIN, int MODE, int NLO, int NHI>
__global__ __launch_bounds__(64) void stream_batch_kernel(const BatchParams bp) {
    batch_loop(bp, [&](const KParams& p, int tile) { stream_tile<FILT, WIN, MODE, NLO, NHI>(p, tile); });
}

// The same kernels held to WAVES waves per SIMD (at most 512 / WAVES
// registers, any excess spilled). Used where the unconstrained kernel needs
// more and the constrained one measured faster: 5x5 DDF at two waves (1.85 ms
// against 2.85 ms on a 4096 x 4096 image), 7x7 VDF, AMNFE and EVMF at two
// (the uneven batch 16% faster), and the unrolled 5x5 VDF at three (it needs
// 178 registers otherwise, i.e. two waves).
template <int WAVES, int FILT, int WIN, int MODE, int NLO, int NHI, int V = VAR_HORNER>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WAVES))) void stream_kernel_w(const KParams p) {
    stream_tile<FILT, WIN, MODE, NLO, NHI, V>(p, xcd_tile(blockIdx.x, gridDim.x));
}

template <int WAVES, int FILT, int WIN, int MODE, int NLO, int NHI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WAVES))) void stream_batch_kernel_w(
    const BatchParams bp) {
    batch_loop(bp, [&](const KParams& p, int tile) { stream_tile<FILT, WIN, MODE, NLO, NHI>(p, tile); });
}

}  // namespace vf
