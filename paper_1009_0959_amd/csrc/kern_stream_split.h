// Streaming angle-filter kernels (VDF, DDF) with the window state split over
// NW waves of one workgroup.
//
// The single-wave streaming kernel (kern_stream.h) keeps, per output lane,
// the member sums S of its window and the row partials Rk of every member
// against each row above it: w^2 (w + 1) / 2 values per summed quantity, 196
// for a 7x7 VDF and 392 for a 7x7 DDF, more than a wave's registers hold at
// any useful occupancy (the 7x7 kernels spilled 107 and 113 registers, and
// their scratch traffic was about 30 GB per 8192^2 launch). Here the NW waves
// of a workgroup walk the same 64-column strip together, and wave v keeps the
// state of the members in window columns [v w / NW, (v + 1) w / NW) only:
//   * each new input row is scored once: wave v evaluates every pixel's pair
//     values for its share of the 2w - 1 column offsets of a row, into the
//     shared LDS plane of that row;
//   * each wave folds the plane into the sums of its own members: the new
//     row's members of its columns against the whole row (their row partial),
//     and its kept members against the whole new row;
//   * at the output, each wave selects among its own members (best, and the
//     runner-up over members distinct from it, in one pass); waves 1.. hand
//     theirs to wave 0 through LDS, which combines them (least criterion, the
//     centre on ties, else the lowest window index), writes the pixel and
//     keeps the near-tie list with the candidate masks.
// Pair values, sums, selections, error bounds and re-check lists are those of
// the single-wave kernel; only the summation order of a member's sum differs
// (each wave adds a row's w pair values as one partial sum), which the FP32
// bound covers.
#pragma once

#include "kern_stream.h"

namespace vf {

// Window columns [B0, B1) whose members wave V of NW keeps.
template <int WIN, int NW, int V>
struct SplitCols {
    static constexpr int B0 = V * WIN / NW;
    static constexpr int B1 = (V + 1) * WIN / NW;
    static constexpr int BW = B1 - B0;
};

// Call f(integral_constant<V>) for the wave index wv in [V0, NW) (wave-uniform).
template <int V, int NW, class F>
__device__ __forceinline__ void split_dispatch(int wv, F& f) {
    if constexpr (V + 1 == NW) {
        f(std::integral_constant<int, V>{});
    } else {
        if (wv == V) f(std::integral_constant<int, V>{});
        else split_dispatch<V + 1, NW>(wv, f);
    }
}

// Fields of one wave's local selection handed to wave 0 (LDS, per lane).
enum : int { SX_CB, SX_EB, SX_C2, SX_E2, SX_BI, SX_PBX, SX_PBY, SX_P2X, SX_P2Y, SX_Z, SX_FIELDS };

template <int FILT, int WIN, int MODE, int NLO, int NHI, int NW>
__device__ __forceinline__ void stream_tile_split(const KParams& p, const int tile) {
    static_assert(FILT == VF_FILTER_VDF || FILT == VF_FILTER_DDF, "angle filters only");
    static_assert(NW >= 2 && NW <= WIN, "two or more waves, each keeping at least one column");
    constexpr int R = (WIN - 1) / 2;
    constexpr int N = WIN * WIN;
    constexpr int C = (N - 1) / 2;
    constexpr int OUTW = 64 - 2 * R;
    constexpr bool DDF = (FILT == VF_FILTER_DDF);
    constexpr bool EXA = (MODE == EV_EXACT);
    // the 64-bit pixel compare slowed the exact 7x7 VDF kernel (21.6 -> 39.4 ms on 8192^2 16-bit)
    constexpr bool WIDE_CMP = !(FILT == VF_FILTER_VDF && WIN == 7);
    constexpr int K = stream_k<FILT, MODE>();   // angle [, distance] [, exact-mode error estimate]
    constexpr int KD = 1;
    constexpr int KE = DDF ? 2 : 1;
    constexpr int NDX = 2 * WIN - 1;
    constexpr int OPW = (NDX + NW - 1) / NW;     // column offsets a wave scores per row
    constexpr int PAD = WIN - 1;
    constexpr int RW = 64 + 2 * PAD;
    constexpr float kExactK = 1.1920929e-07f;    // 2^-23 (the exact-mode per-pair estimate)
    constexpr bool MASKS = writes_masks(FILT, WIN, MODE, true);
    constexpr int BW0 = SplitCols<WIN, NW, 0>::BW;
    constexpr int NLOW = N - WIN * BW0;          // members kept by waves 1..

    __shared__ float4 sU[WIN][RW];                          // unit vectors (w = 1: zero vector)
    __shared__ float4 sF[DDF ? WIN : 1][DDF ? RW : 1];      // DDF: the pixels as floats
    __shared__ uint2 sP[WIN][RW];                           // packed pixels
    __shared__ float sC[K][NDX][64];                        // one row's pair values
    __shared__ uint32_t sX[NW - 1][SX_FIELDS][64];          // waves 1..: local selections
    __shared__ float sLow[MASKS ? NLOW : 1][64];            // waves 1..: crit - err of their members
    constexpr int FCAP = 96;
    __shared__ uint32_t s_flags[FCAP];
    __shared__ uint64_t s_masks[MASKS ? FCAP : 1];

    const int L = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int sx = tile % p.tiles_x;
    const int sy = tile / p.tiles_x;
    const int X = sx * OUTW - R;
    const int Y0 = sy * p.strip_rows;
    const int rows_out = min(p.strip_rows, p.H - Y0);
    const int gxl = min(max(X + L, 0), p.W - 1);
    const bool out_lane = (L >= R) && (L < 64 - R) && (X + L < p.W);
    const int u16 = p.u16;
    const int steps = rows_out + WIN - 1;

    // every ring slot starts as a finite copy of a real pixel (see stream_tile)
    for (int c = (int)threadIdx.x; c < RW; c += 64 * NW)
#pragma unroll
        for (int j = 0; j < WIN; ++j) {
            sU[j][c] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
            if constexpr (DDF) sF[j][c] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            sP[j][c] = make_uint2(0u, 0u);
        }
    __syncthreads();

    auto run = [&](auto wv_tag) {
        constexpr int WV = decltype(wv_tag)::value;
        constexpr int B0 = SplitCols<WIN, NW, WV>::B0;
        constexpr int BW = SplitCols<WIN, NW, WV>::BW;
        constexpr bool OWNS_C = (C % WIN) >= B0 && (C % WIN) < B0 + BW;
        // as in stream_tile: S against the member's own row and the rows
        // below, Rk suffix sums against the rows above; no pair value is
        // ever subtracted
        float S[K][WIN][BW];
        float Rk[K][WIN][BW][WIN];   // Rk[k][j][bl][jj]: member (j, B0 + bl) against rows jj .. j - 1
        auto msum = [&](int k, int j, int bl) -> float {
            return j > 0 ? S[k][j][bl] + Rk[k][j][bl][0] : S[k][j][bl];
        };
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < WIN; ++j)
#pragma unroll
                for (int bl = 0; bl < BW; ++bl) {
                    S[k][j][bl] = 0.0f;
#pragma unroll
                    for (int jj = 0; jj < j; ++jj) Rk[k][j][bl][jj] = 0.0f;
                }
        uint32_t zero_rows = 0u;   // bit j: a zero pixel among the strip's pixels of ring row j
        uint32_t nflag = 0u;       // wave 0: windows held in the LDS flag list
        auto flush = [&]() {
            // one reservation in the re-check list for the wave's held windows
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            uint32_t base = 0u;
            if (L == 0) base = atomicAdd(p.flag_count, nflag);
            base = (uint32_t)__shfl((int)base, 0);
            for (uint32_t e = (uint32_t)L; e < nflag; e += 64u) {
                if (base + e < p.flag_cap) {
                    p.flag_list[base + e] = s_flags[e];
                    if (p.flag_item) p.flag_item[base + e] = (uint32_t)p.item;
                    if constexpr (MASKS) p.flag_mask[base + e] = s_masks[e];
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            nflag = 0u;
        };

        for (int t = 0; t < steps; ++t) {
            const int rs = t % WIN;   // ring slot of input row t
            // ---- 1. the new input row into the ring (wave 0: packed pixels and
            //         unit vectors; the last wave: DDF's float pixels)
            {
                const int gy = min(max(Y0 - R + t, 0), p.H - 1);
                uint32_t r, g, b;
                load_pixel(p.src + (int64_t)gy * p.src_pitch, gxl, u16, r, g, b);
                const bool z = (r | g | b) == 0u;
                zero_rows = (zero_rows & ~(1u << rs)) | (__any(z) ? (1u << rs) : 0u);
                if constexpr (WV == 0) {
                    sP[rs][L + PAD] = pack_pixel(r, g, b, u16);
                    sU[rs][L + PAD] = unit_vector(r, g, b);
                }
                if constexpr (DDF && WV == NW - 1) sF[rs][L + PAD] = make_float4((float)r, (float)g, (float)b, 0.0f);
            }
            __syncthreads();

            // ---- 2. shift the kept state down one row
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int j = 0; j < WIN - 1; ++j)
#pragma unroll
                    for (int bl = 0; bl < BW; ++bl) {
                        S[k][j][bl] = S[k][j + 1][bl];
#pragma unroll
                        for (int jj = 0; jj < j; ++jj) Rk[k][j][bl][jj] = Rk[k][j + 1][bl][jj + 1];
                    }
#pragma unroll
                for (int bl = 0; bl < BW; ++bl) S[k][WIN - 1][bl] = 0.0f;
            }

            // ---- 3. one row at a time: score this wave's share of the pairs,
            //         then fold the whole row's values into the kept sums
            const float4 me = sU[rs][L + PAD];
            float4 mf = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if constexpr (DDF) mf = sF[rs][L + PAD];
#pragma unroll
            for (int js = 0; js < WIN; ++js) {
                const int dy = js - (WIN - 1);
                const int qs = (rs + WIN + dy) % WIN;
                const int ndx = (dy == 0) ? WIN - 1 : NDX;
#pragma unroll
                for (int oo = 0; oo < OPW; ++oo) {
                    const int o = WV * OPW + oo;
                    if (o >= ndx) break;
                    const int dx = o - (WIN - 1);
                    const float4 uq = sU[qs][L + PAD + dx];
                    const float ex = me.x - uq.x, ey = me.y - uq.y, ez = me.z - uq.z;
                    const float s2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
                    sC[0][o][L] = angle_from_s2<MODE, NLO, NHI>(s2, p.lo, p.hi);
                    if constexpr (DDF) {
                        const float4 q = sF[qs][L + PAD + dx];
                        const float er = mf.x - q.x, eg = mf.y - q.y, eb = mf.z - q.z;
                        sC[KD][o][L] = fsqrt(fmaf(er, er, fmaf(eg, eg, eb * eb)));
                    }
                    if constexpr (EXA)
                        sC[KE][o][L] = s2 > 0.0f ? fmaf(kExactK, frsq(s2 + 5.9604645e-08f), 6.0e-7f) : 0.0f;
                }
                __syncthreads();
                if (dy < 0) {
                    // the new row's members of this wave's columns against row js
#pragma unroll
                    for (int al = 0; al < BW; ++al) {
                        const int a = B0 + al;
                        const int la = min(max(L - R + a, 0), 63);
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            float racc = 0.0f;
#pragma unroll
                            for (int b = 0; b < WIN; ++b) racc += sC[k][b - a + WIN - 1][la];
                            Rk[k][WIN - 1][al][js] = racc;
                        }
                    }
                    // this wave's members of row js against the new row
#pragma unroll
                    for (int bl = 0; bl < BW; ++bl) {
                        const int b = B0 + bl;
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            float acc = 0.0f;
#pragma unroll
                            for (int a = 0; a < WIN; ++a) acc += sC[k][b - a + WIN - 1][min(max(L - R + a, 0), 63)];
                            S[k][js][bl] += acc;
                        }
                    }
                } else {
                    // pairs inside the new row, for the members of this wave's columns
#pragma unroll
                    for (int bl = 0; bl < BW; ++bl) {
                        const int c = B0 + bl;
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            float acc = 0.0f;
#pragma unroll
                            for (int b = 0; b < c; ++b) acc += sC[k][b - c + WIN - 1][min(max(L - R + c, 0), 63)];
#pragma unroll
                            for (int a = c + 1; a < WIN; ++a) acc += sC[k][c - a + WIN - 1][min(max(L - R + a, 0), 63)];
                            S[k][WIN - 1][bl] += acc;
                        }
                    }
                }
                __syncthreads();
            }

            // the new members' row sums become suffix sums (rows jj .. w - 2)
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int al = 0; al < BW; ++al)
#pragma unroll
                    for (int jj = WIN - 3; jj >= 0; --jj) Rk[k][WIN - 1][al][jj] += Rk[k][WIN - 1][al][jj + 1];

            // ---- 4. output: the window with rows t - w + 1 .. t is complete
            if (t >= WIN - 1) {
                const int oy = Y0 + t - (WIN - 1);
                const int slot0 = rs + 1 == WIN ? 0 : rs + 1;   // ring slot of the window's top row
                auto member = [&](int j, int b) -> uint2 {
                    const int slot = slot0 + j >= WIN ? slot0 + j - WIN : slot0 + j;
                    return sP[slot][L - R + b + PAD];
                };
                const float pexp = p.kscale;
                constexpr float kSum0 = (N + 4 * WIN) * kU32;
                const float kSum = kSum0 + p.rho;
                auto crit_err = [&](auto half_tag, int j, int bl, float& c, float& e) {
                    constexpr bool HALF = decltype(half_tag)::value;
                    const float sa = msum(0, j, bl);
                    const float se = EXA ? msum(KE, j, bl) : 0.0f;
                    const float ea = (EXA ? se : (N - 1) * p.eta) + kSum * sa;
                    if constexpr (!DDF) {
                        c = sa;
                        e = ea;
                    } else {
                        const float sd = msum(KD, j, bl);
                        const float ed = (kSum0 + 2.0f * kU32) * sd;
                        if constexpr (HALF) {
                            c = sa * sd;
                            e = sd * ea + sa * ed + 2.0f * kU32 * c;
                        } else {
                            const float la2 = __log2f(sa);
                            const float ld2 = __log2f(sd);
                            c = (1.0f - pexp) * ld2 + pexp * la2;
                            e = 1.4427f * ((1.0f - pexp) * ed / sd + pexp * ea / sa) + 4.0f * kU32 * fabsf(c) + 1e-6f;
                        }
                    }
                };
                // local selection in window order: best (the centre first when
                // this wave keeps it, else its first member, so that the best
                // is always a member even when criteria are not finite) and
                // the runner-up over members distinct from the best so far
                float cb, eb, c2 = __builtin_inff(), e2 = 0.0f;
                int bi;
                uint2 pb, p2 = make_uint2(0xffffffffu, 0xffffffffu);
                bool anyzero = false, allzero = true;
                const bool check_zero = zero_rows != 0u;
                auto pass = [&](auto half_tag) {
                    constexpr int J0 = OWNS_C ? C / WIN : 0;
                    constexpr int BL0 = OWNS_C ? C % WIN - B0 : 0;
                    crit_err(half_tag, J0, BL0, cb, eb);
                    bi = J0 * WIN + B0 + BL0;
                    pb = member(J0, B0 + BL0);
#pragma unroll
                    for (int j = 0; j < WIN; ++j)
#pragma unroll
                        for (int bl = 0; bl < BW; ++bl) {
                            float c, e;
                            crit_err(half_tag, j, bl, c, e);
                            const uint2 q = member(j, B0 + bl);
                            const bool diff = !same_pixel<WIDE_CMP>(q, pb);
                            const bool lt = c < cb;
                            const bool old_up = lt && diff;
                            const bool new_up = !lt && diff && c < c2;
                            c2 = old_up ? cb : (new_up ? c : c2);
                            e2 = old_up ? eb : (new_up ? e : e2);
                            p2.x = old_up ? pb.x : (new_up ? q.x : p2.x);
                            p2.y = old_up ? pb.y : (new_up ? q.y : p2.y);
                            cb = lt ? c : cb;
                            eb = lt ? e : eb;
                            pb = lt ? q : pb;
                            bi = lt ? j * WIN + B0 + bl : bi;
                            if (check_zero) {
                                const bool zq = (q.x | q.y) == 0u;
                                anyzero |= zq;
                                allzero &= zq;
                            }
                        }
                };
                const bool half = !DDF || pexp == 0.5f;
                if (half) pass(std::true_type{});
                else pass(std::false_type{});
                if constexpr (WV > 0) {
                    uint32_t* xs = &sX[WV - 1][0][0];
                    xs[SX_CB * 64 + L] = __float_as_uint(cb);
                    xs[SX_EB * 64 + L] = __float_as_uint(eb);
                    xs[SX_C2 * 64 + L] = __float_as_uint(c2);
                    xs[SX_E2 * 64 + L] = __float_as_uint(e2);
                    xs[SX_BI * 64 + L] = (uint32_t)bi;
                    xs[SX_PBX * 64 + L] = pb.x;
                    xs[SX_PBY * 64 + L] = pb.y;
                    xs[SX_P2X * 64 + L] = p2.x;
                    xs[SX_P2Y * 64 + L] = p2.y;
                    xs[SX_Z * 64 + L] = (anyzero ? 1u : 0u) | (allzero ? 2u : 0u);
                    if constexpr (MASKS) {
                        // lower ends crit - err of this wave's members, for wave 0's masks
                        auto lows = [&](auto half_tag) {
#pragma unroll
                            for (int j = 0; j < WIN; ++j)
#pragma unroll
                                for (int bl = 0; bl < BW; ++bl) {
                                    float c, e;
                                    crit_err(half_tag, j, bl, c, e);
                                    sLow[j * (WIN - BW0) + (B0 + bl - BW0)][L] = c - e;
                                }
                        };
                        if (half) lows(std::true_type{});
                        else lows(std::false_type{});
                    }
                }
                __syncthreads();
                if constexpr (WV == 0) {
                    // combine the waves' selections: least criterion, the centre
                    // on ties, else the lowest window index; the runner-up is the
                    // least criterion over members distinct from the winner
#pragma unroll
                    for (int w = 1; w < NW; ++w) {
                        const uint32_t* xs = &sX[w - 1][0][0];
                        const float cbw = __uint_as_float(xs[SX_CB * 64 + L]);
                        const float ebw = __uint_as_float(xs[SX_EB * 64 + L]);
                        const float c2w = __uint_as_float(xs[SX_C2 * 64 + L]);
                        const float e2w = __uint_as_float(xs[SX_E2 * 64 + L]);
                        const int biw = (int)xs[SX_BI * 64 + L];
                        const uint2 pbw = make_uint2(xs[SX_PBX * 64 + L], xs[SX_PBY * 64 + L]);
                        const uint2 p2w = make_uint2(xs[SX_P2X * 64 + L], xs[SX_P2Y * 64 + L]);
                        const uint32_t zw = xs[SX_Z * 64 + L];
                        anyzero |= (zw & 1u) != 0u;
                        allzero &= (zw & 2u) != 0u;
                        const bool take = cbw < cb || (cbw == cb && (biw == C || (bi != C && biw < bi)));
                        if (take) {
                            // the previous waves' least member distinct from the new winner
                            const bool pdiff = !same_pixel<WIDE_CMP>(pb, pbw);
                            const float cp = pdiff ? cb : c2, ep = pdiff ? eb : e2;
                            const uint2 pp = pdiff ? pb : p2;
                            const bool w2 = c2w < cp;
                            c2 = w2 ? c2w : cp;
                            e2 = w2 ? e2w : ep;
                            p2 = w2 ? p2w : pp;
                            cb = cbw;
                            eb = ebw;
                            bi = biw;
                            pb = pbw;
                        } else {
                            const bool wdiff = !same_pixel<WIDE_CMP>(pbw, pb);
                            const float cw = wdiff ? cbw : c2w, ew = wdiff ? ebw : e2w;
                            const uint2 pw = wdiff ? pbw : p2w;
                            const bool w2 = cw < c2;
                            c2 = w2 ? cw : c2;
                            e2 = w2 ? ew : e2;
                            p2 = w2 ? pw : p2;
                        }
                    }
                    bool flag = false;
                    uint64_t cmask = ~0ull;
                    if (out_lane && oy < p.H) {
                        const bool zero_mix = anyzero && !allzero;
                        store_pixel(p.dst + (int64_t)oy * p.dst_pitch, X + L, pb, u16);
                        if (p.recheck) {
                            const bool fin = (cb == cb) && (cb > -__builtin_inff()) && (cb < __builtin_inff());
                            // c2 stays +inf when every member equals the selected vector
                            const bool tie = (c2 < __builtin_inff()) && (c2 - cb <= eb + e2);
                            flag = !fin || tie || zero_mix;
                            if (MASKS && flag && fin && !zero_mix) {
                                // members whose criterion may still be the minimum:
                                // crit_i - e_i <= best + e_best, widened by 8 ulps
                                cmask = 0ull;
                                const float lim = cb + eb + 8.0f * kU32 * (fabsf(cb) + eb);
                                auto mask_pass = [&](auto half_tag) {
#pragma unroll
                                    for (int j = 0; j < WIN; ++j)
#pragma unroll
                                        for (int bl = 0; bl < BW0; ++bl) {
                                            float c, e;
                                            crit_err(half_tag, j, bl, c, e);
                                            cmask |= (c - e <= lim) ? (1ull << (j * WIN + bl)) : 0ull;
                                        }
                                };
                                if (half) mask_pass(std::true_type{});
                                else mask_pass(std::false_type{});
#pragma unroll
                                for (int j = 0; j < WIN; ++j)
#pragma unroll
                                    for (int b = BW0; b < WIN; ++b)
                                        cmask |= (sLow[j * (WIN - BW0) + (b - BW0)][L] <= lim) ? (1ull << (j * WIN + b))
                                                                                            : 0ull;
                            }
                        }
                    }
                    flag = flag && p.recheck;
                    // wave-aggregated append to the LDS list; published when nearly full
                    const unsigned long long mask = __ballot(flag);
                    if (flag) {
                        const uint32_t slot = nflag + (uint32_t)__popcll(mask & ((1ull << L) - 1ull));
                        s_flags[slot] = (uint32_t)(oy * p.W + X + L);
                        if constexpr (MASKS) s_masks[slot] = cmask;
                    }
                    nflag += (uint32_t)__popcll(mask);
                    if (nflag > FCAP - 64) flush();
                }
            }
            __syncthreads();
        }
        if constexpr (WV == 0) {
            if (nflag != 0u) flush();
        }
    };
    // every wave runs the same number of steps and barriers
    split_dispatch<0, NW>(wv, run);
}

template <int NW, int FILT, int WIN, int MODE, int NLO, int NHI>
__global__ __launch_bounds__(64 * NW) void stream_split_kernel(const KParams p) {
    stream_tile_split<FILT, WIN, MODE, NLO, NHI, NW>(p, xcd_tile(blockIdx.x, gridDim.x));
}

template <int NW, int FILT, int WIN, int MODE, int NLO, int NHI>
__global__ __launch_bounds__(64 * NW) void stream_split_batch_kernel(const BatchParams bp) {
    batch_loop(bp, [&](const KParams& p, int tile) { stream_tile_split<FILT, WIN, MODE, NLO, NHI, NW>(p, tile); });
}

// Launch a split kernel (NW waves per workgroup), or, while the host has set
// occupancy_query(), store its resident workgroups per CU there scaled to
// single-wave strips (the strip sizing counts one strip per resident
// workgroup) and launch nothing.
template <int NW, class Kern>
inline void stream_split_launch(Kern kernel, const KParams& p, int blocks, void* stream) {
    if (int* q = occupancy_query()) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(q, kernel, 64 * NW, 0) != hipSuccess) *q = 0;
        return;
    }
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(64 * NW), 0, (hipStream_t)stream, p);
}

}  // namespace vf
