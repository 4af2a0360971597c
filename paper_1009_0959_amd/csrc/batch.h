// Persistent batch kernels: many images of uneven size with one filter class
// (filter, window, approximant) per launch. Workgroups pull tiles from a work
// counter; the tiles of all images are numbered consecutively with the
// images sorted largest first, so the biggest images start first and the
// small ones fill the tail (longest-processing-time order).
#pragma once

#include "kern_common.h"
#include "recheck_dev.h"

namespace vf {

__device__ inline int batch_find(const BatchParams& bp, uint32_t w) {
    int lo = 0, hi = bp.nitems - 1;   // last item whose first tile is <= w
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bp.items[mid].first_tile <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline RcImage rc_image(const BatchItem& it) {
    return RcImage{it.src, it.dst, it.src_pitch, it.dst_pitch, it.H, it.W, it.u16};
}

__device__ inline void batch_apply(KParams& p, const BatchItem& it) {
    p.src = it.src;
    p.dst = it.dst;
    p.src_pitch = it.src_pitch;
    p.dst_pitch = it.dst_pitch;
    p.H = it.H;
    p.W = it.W;
    p.u16 = it.u16;
    p.tiles_x = it.tiles_x;
    p.item = it.index;
}

// Workgroup loop: take the next tile, run it, until the work runs out (every
// workgroup leaves after the counter passes the total).
template <class TileFn>
__device__ inline void batch_loop(const BatchParams& bp, TileFn&& fn) {
    __shared__ uint32_t s_work;
    for (;;) {
        if (threadIdx.x == 0) s_work = atomicAdd(bp.counter, 1u);
        __syncthreads();
        const uint32_t w = s_work;
        __syncthreads();
        if (w >= bp.total) break;
        const BatchItem it = bp.items[batch_find(bp, w)];
        KParams p = bp.base;
        batch_apply(p, it);
        fn(p, (int)(w - it.first_tile));
        __syncthreads();
    }
}

// Launch a persistent kernel with as many workgroups as the device keeps
// resident at once (but no more than there are tiles). With `probe` set,
// launch nothing and report success.
template <class K>
inline int launch_persistent(bool probe, K kernel, int threads, const BatchParams& bp, int num_cus,
                             void* stream) {
    if (probe) return 0;
    if (int* q = occupancy_query()) {   // residency query: launch nothing
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(q, kernel, threads, 0) != hipSuccess) *q = 0;
        return 0;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const uint64_t want = (uint64_t)per_cu * (uint64_t)(num_cus > 0 ? num_cus : 1);
    const int blocks = (int)(want < bp.total ? want : (bp.total > 0 ? bp.total : 1));
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(threads), 0, (hipStream_t)stream, bp);
    return (int)hipGetLastError();
}

// FP64 re-check of the class's listed windows (item and pixel per entry).
// When the class flagged more windows than its list holds, the overflow pass
// below evaluates every window of the class instead, and this one does nothing.
template <int FILT>
__global__ __launch_bounds__(64) void recheck_batch_kernel(const BatchParams bp, int eval, int window) {
    extern __shared__ double scratch[];
    const uint32_t count = *bp.base.flag_count;
    if (count > bp.base.flag_cap) return;
    for (uint32_t t = blockIdx.x; t < count; t += gridDim.x) {
        const uint32_t item = bp.base.flag_item[t];
        if (item >= (uint32_t)bp.nitems) continue;   // never listed; keeps every access in bounds
        const RcImage im = rc_image(bp.items[item]);
        const uint32_t pix = bp.base.flag_list[t];
        if (pix >= (uint32_t)im.H * (uint32_t)im.W) continue;
        const uint64_t mask = bp.base.flag_mask ? bp.base.flag_mask[t] : ~0ull;
        const int y = (int)(pix / (uint32_t)im.W);
        recheck_window<FILT>(bp.base, im, eval, window, y, (int)(pix - (uint32_t)y * (uint32_t)im.W), scratch,
                             threadIdx.x, mask);
    }
}

__device__ inline int batch_find_pixel(const BatchParams& bp, uint32_t t) {
    int lo = 0, hi = bp.nitems - 1;   // last item whose first pixel is <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bp.items[mid].first_pixel <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Overflow pass: when the class flagged more windows than its re-check list
// holds (the list lost entries), every window of the class is evaluated in
// FP64, one wave per window, grid-stride over the class's `pixels` pixels in
// item-table order. Otherwise every wave leaves at once.
template <int FILT>
__global__ __launch_bounds__(64) void overflow_batch_kernel(const BatchParams bp, int eval, int window,
                                                            uint32_t pixels) {
    extern __shared__ double scratch[];
    if (*bp.base.flag_count <= bp.base.flag_cap) return;
    for (uint32_t t = blockIdx.x; t < pixels; t += gridDim.x) {
        const BatchItem& it = bp.items[batch_find_pixel(bp, t)];
        const RcImage im = rc_image(it);
        const uint32_t local = t - it.first_pixel;
        if (local >= (uint32_t)im.H * (uint32_t)im.W) continue;   // (the prefix covers every pixel once)
        const int y = (int)(local / (uint32_t)im.W);
        recheck_window<FILT>(bp.base, im, eval, window, y, (int)(local - (uint32_t)y * (uint32_t)im.W), scratch,
                             threadIdx.x);
    }
}

}  // namespace vf
