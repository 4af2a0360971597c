// C ABI of the vf library: contexts, argument validation, kernel dispatch,
// the FP64 re-check submission, statistics and error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"


namespace vf {

thread_local std::string g_last_error;

vf_status set_error(vf_status st, const char* msg) {
    g_last_error = msg ? msg : "";
    return st;
}

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = (hipSetDevice(dev) == hipSuccess);
}

DeviceGuard::~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
}

vf_status hip_fail(hipError_t e, const char* what) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    return set_error(VF_EHIP, buf);
}

bool inject_hip_error(const char* site) {
    const char* v = std::getenv("VF_INJECT_HIP_ERROR");
    return v && std::strcmp(v, site) == 0;
}

vf_status validate_image(const vf_image* img) {
    if (!img) return set_error(VF_EINVAL, "image is null");
    if (!img->src || !img->dst) return set_error(VF_EINVAL, "null src or dst");
    if (img->dtype != VF_U8 && img->dtype != VF_U16) return set_error(VF_EINVAL, "dtype must be VF_U8 or VF_U16");
    if (img->height < 1 || img->width < 1) return set_error(VF_EINVAL, "height and width must be >= 1");
    if ((uint64_t)img->height * (uint64_t)img->width >= (1ull << 32))
        return set_error(VF_EUNSUPPORTED, "images of 2^32 or more pixels are not supported");
    const int64_t es = img->dtype == VF_U16 ? 2 : 1;
    const int64_t row = 3 * (int64_t)img->width * es;
    if (img->src_pitch < row || img->dst_pitch < row) return set_error(VF_EINVAL, "pitch smaller than a row");
    if (img->dtype == VF_U16 && ((img->src_pitch | img->dst_pitch) & 1))
        return set_error(VF_EINVAL, "uint16 pitches must be even");
    const char* s0 = (const char*)img->src;
    const char* s1 = s0 + (img->height - 1) * img->src_pitch + row;
    const char* d0 = (const char*)img->dst;
    const char* d1 = d0 + (img->height - 1) * img->dst_pitch + row;
    if (s0 < d1 && d0 < s1) return set_error(VF_EINVAL, "src and dst overlap");
    return VF_OK;
}

static vf_status ensure_capacity(vf_context* ctx, uint64_t pixels) {
    if (ctx->flag_cap >= pixels) return VF_OK;
    if (ctx->flag_list) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        (void)hipFree(ctx->flag_list);
        (void)hipFree(ctx->flag_mask);
        ctx->flag_list = nullptr;
        ctx->flag_mask = nullptr;
        ctx->flag_cap = 0;
    }
    hipError_t e = hipMalloc((void**)&ctx->flag_list, pixels * sizeof(uint32_t));
    if (e == hipSuccess) {
        e = hipMalloc((void**)&ctx->flag_mask, pixels * sizeof(uint64_t));
        if (e != hipSuccess) (void)hipFree(ctx->flag_list);
    }
    if (e != hipSuccess) {
        ctx->flag_list = nullptr;
        ctx->flag_mask = nullptr;
        return set_error(VF_ENOMEM, "cannot allocate the re-check list");
    }
    ctx->flag_cap = pixels;
    return VF_OK;
}

int*& occupancy_query() {
    thread_local int* q = nullptr;
    return q;
}

void fill_kparams(const vf_image* img, const Prepared& P, KParams* k) {
    std::memset(k, 0, sizeof(*k));
    k->src = (const unsigned char*)img->src;
    k->dst = (unsigned char*)img->dst;
    k->src_pitch = img->src_pitch;
    k->dst_pitch = img->dst_pitch;
    k->H = img->height;
    k->W = img->width;
    k->tiles_x = (img->width + kTileX - 1) / kTileX;
    k->u16 = img->dtype == VF_U16;
    std::memcpy(k->lo, P.lo, sizeof(P.lo));
    std::memcpy(k->hi, P.hi, sizeof(P.hi));
    k->n_lo = P.n_lo;
    k->n_hi = P.n_hi;
    k->eta = P.eta;
    k->rho = (float)P.rho;
    if (P.variant == 2 && (is_amnf(P.filter) || P.filter == VF_FILTER_EVMF)) {
        for (int i = 1; i < P.n_lo; ++i) {
            const _Float16 h = (_Float16)P.lo[i];   // exact: the coefficient was rounded to FP16
            uint16_t bits;
            std::memcpy(&bits, &h, sizeof(bits));
            k->lo16[i - 1] = (uint32_t)bits | ((uint32_t)bits << 16);
        }
    }
    k->kscale = P.kscale;
    k->cutoff = P.cutoff;
    k->param64 = P.param;
    k->scale64 = std::pow((double)(P.window * P.window), -P.param / 3.0);
    k->cutoff64 = P.cutoff64;
    k->wbound = P.wbound;
    k->zband = P.zband;
}

namespace {

// one wave per flagged window; the count is known only on the device,
// blocks beyond it exit at once
vf_status launch_recheck_call(vf_context* ctx, int filter, int emode, int window, const KParams& k,
                              uint64_t pixels, void* stream) {
    const uint64_t want = pixels / 64;
    const int rblocks = (int)(want < 1 ? 1 : (want > 16384 ? 16384 : want));
    const int rc = inject_hip_error("recheck") ? (int)hipErrorLaunchFailure
                                               : launch_recheck(filter, emode, window, k, rblocks, stream);
    if (rc != 0) {
        // the window kernel counted into this call's slot and the next slot
        // was never cleared: the next call re-zeroes the whole ring first
        ctx->counters_dirty = true;
        return hip_fail((hipError_t)rc, "re-check kernel launch");
    }
    ctx->last_slot = ctx->slot;
    ctx->slot = (ctx->slot + 1) % kCounterSlots;
    return VF_OK;
}

}  // namespace

// Strip height for a streaming call from the kernel's residency: with `slots`
// waves resident on the device (workgroups per CU x CUs) and strips_x column
// strips, a call of R rounds cuts every column into floor(R slots / strips_x)
// strips; each wave then steps through rows + w - 1 image rows. Take the R
// in 1..16 whose rounds x steps is least: with 64-row strips a 4096^2 5x5
// call needs 4416 waves against 3072 slots, so its second round ran 44% full.
// 3x3 windows take at least three rounds: their short steps measured 10%
// faster in many short strips (4096^2 VDF: 0.23 ms at 16-24 rows, 0.26 ms at
// the single full round's 46).
int auto_strip_rows(int H, int strips_x, int window, int64_t slots) {
    if (slots < 1 || strips_x < 1) return 64;
    int best_rows = 64;
    int64_t best_cost = -1;
    for (int r = window == 3 ? 3 : 1; r <= 16; ++r) {
        const int64_t chunks = (int64_t)r * slots / strips_x;
        if (chunks < 1) continue;
        int rows = (int)((H + chunks - 1) / chunks);
        rows = rows < 1 ? 1 : (rows > 4096 ? 4096 : rows);
        const int64_t tasks = (int64_t)strips_x * ((H + rows - 1) / rows);
        const int64_t rounds = (tasks + slots - 1) / slots;
        const int64_t cost = rounds * (rows + window - 1);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best_rows = rows;
        }
    }
    return best_rows;
}

static int eval_mode(int filter, int eval) {
    (void)filter;
    return eval;   // vf_eval values and kernel modes coincide
}

vf_status launch_window_kernels(const vf_image* img, int filter, int window, const Prepared& P, uint32_t flags,
                                int strip_rows, int num_cus, uint64_t* mask_array, KParams& k, void* stream,
                                WindowLaunch* out) {
    uint64_t blocks_launched = 0;
    const int mode = eval_mode(filter, P.eval);
    const bool angle = (filter == VF_FILTER_VDF || filter == VF_FILTER_DDF);
    int rc = -1, tile_w = kTileX, tile_h = kTileY;
    bool streaming = false;
    if (P.variant != 0 && (flags & VF_DIRECT))
        return set_error(VF_EUNSUPPORTED, "Estrin and packed FP16 evaluation run in the streaming kernels only");
    if (!(flags & VF_DIRECT)) {
        // streaming kernel: one wave per 64-column strip (64 - 2r output columns)
        const int outw = 64 - (window - 1);
        k.tiles_x = (img->width + outw - 1) / outw;
        k.flag_mask = writes_masks(filter, window, mode, true) ? mask_array : nullptr;
        auto launch = [&](int blocks) -> int {
            if (P.variant != 0)
                return angle ? launch_angle_stream_var(window, filter, mode, P.n_lo, P.n_hi, P.variant, k, blocks,
                                                       stream)
                             : launch_fe_stream_f16(filter, window, mode, k, blocks, stream);
            if (angle) return launch_angle_stream(window, filter, mode, P.n_lo, P.n_hi, k, blocks, stream);
            if (is_amnf(filter)) return launch_amnfe_stream(filter, window, amnfe_mode(mode), k, blocks, stream);
            return launch_evmf_stream(window, mode, k, blocks, stream);
        };
        if (strip_rows <= 0 && filter == VF_FILTER_EVMF) {
            // EVMF's sized strips measured slower (4096^2 5x5: 2.41 ms at 111
            // rows against 1.58 ms at 64), so it keeps the fixed height
            strip_rows = 64;
        } else if (strip_rows <= 0) {
            // size the strips from the residency of the kernel this call runs
            int per_cu = 0;
            occupancy_query() = &per_cu;
            const int q = launch(0);
            occupancy_query() = nullptr;
            strip_rows = q < 0 ? 64 : auto_strip_rows(img->height, k.tiles_x, window, (int64_t)per_cu * num_cus);
        }
        k.strip_rows = strip_rows;
        const int strips_y = (img->height + k.strip_rows - 1) / k.strip_rows;
        blocks_launched = (uint64_t)k.tiles_x * strips_y;
        rc = launch(k.tiles_x * strips_y);
        if (rc < 0 && P.variant != 0) return set_error(VF_EUNSUPPORTED, "no streaming kernel for this evaluation variant");
        if (rc >= 0) {
            streaming = true;
            tile_w = outw;
            tile_h = k.strip_rows;
        }
    }
    if (!streaming) {
        k.tiles_x = (img->width + kTileX - 1) / kTileX;
        // 7x7 angle kernels use 64 x 2 tiles (see kern_angle.h), all others 64 x 4
        tile_h = (angle && window == 7) ? 2 : kTileY;
        const int blocks = k.tiles_x * ((img->height + tile_h - 1) / tile_h);
        blocks_launched = (uint64_t)blocks;
        k.flag_mask = writes_masks(filter, window, mode, false) ? mask_array : nullptr;
        if (angle) rc = launch_angle(filter, window, mode, P.n_lo, P.n_hi, k, blocks, stream);
        else if (is_amnf(filter)) rc = launch_amnfe(filter, window, amnfe_mode(mode), k, blocks, stream);
        else rc = launch_evmf(window, mode, k, blocks, stream);
    }
    if (rc < 0) return set_error(VF_EUNSUPPORTED, "no kernel for this filter/window/approximant");
    if (rc != 0) return hip_fail((hipError_t)rc, "window kernel launch");
    out->blocks = blocks_launched;
    out->tile_w = tile_w;
    out->tile_h = tile_h;
    out->streaming = streaming;
    out->mode = mode;
    return VF_OK;
}

vf_status run_filter(vf_context* ctx, const vf_image* img, int filter, int window, double param,
                     const vf_approx* ap_in, void* stream, int strip_override) {
    if (!ctx) return set_error(VF_EINVAL, "context is null");
    vf_status st = validate_image(img);
    if (st != VF_OK) return st;
    if (!ap_in) return set_error(VF_EINVAL, "approx is null");
    // the pending call's list and counter slot are still live: a new call
    // would count into the same slot and its re-check would read the old list
    if (ctx->pending)
        return set_error(VF_EINVAL, "a deferred re-check is pending: call vf_recheck_pending first");
    vf_approx tuned_ap = *ap_in;
    int strip_rows = strip_override > 0 ? strip_override : ctx->strip_rows;
    if (ap_in->flags & VF_TUNED) apply_tuned(ctx, filter, window, img->dtype, &tuned_ap, &strip_rows, false);
    const vf_approx* ap = &tuned_ap;
    Prepared P;
    if ((st = prepare(filter, window, param, ap, &P)) != VF_OK) return st;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return set_error(VF_EHIP, "hipSetDevice failed");
    if (ctx->counters_dirty) {
        hipError_t e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipMemset(ctx->counters, 0, kCounterSlots * sizeof(uint32_t));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "re-zeroing the re-check counters after a failed call");
        ctx->counters_dirty = false;
        ctx->slot = 0;
    }
    const uint64_t pixels = (uint64_t)img->height * (uint64_t)img->width;
    if (P.variant == 3) {
        // every window in FP64: one wave per window, no re-check list
        KParams k;
        fill_kparams(img, P, &k);
        const int emode = is_amnf(filter) ? amnfe_mode(P.eval) : P.eval;
        const int blocks = (int)(pixels < 65536 ? pixels : 65536);
        const int rc = launch_fp64(filter, emode, window, k, blocks, stream);
        if (rc != 0) return hip_fail((hipError_t)rc, "FP64 window kernel launch");
        ctx->last_batch = false;
        ctx->last_windows = pixels;
        ctx->last_blocks = (uint64_t)blocks;
        ctx->last_tile_w = 1;
        ctx->last_tile_h = 1;
        ctx->last_recheck = false;
        ctx->last_streaming = false;
        return VF_OK;
    }
    const bool recheck = !(ap->flags & VF_NO_RECHECK);
    if (recheck && (st = ensure_capacity(ctx, pixels)) != VF_OK) return st;

    KParams k;
    fill_kparams(img, P, &k);
    k.recheck = recheck ? 1 : 0;
    k.flag_list = ctx->flag_list;
    k.flag_count = ctx->counters + ctx->slot;
    k.next_count = ctx->counters + (ctx->slot + 1) % kCounterSlots;
    k.flag_cap = (uint32_t)(recheck ? pixels : 0);
    WindowLaunch wl;
    st = inject_hip_error("window")
             ? hip_fail(hipErrorLaunchFailure, "window kernel launch")
             : launch_window_kernels(img, filter, window, P, ap->flags, strip_rows, ctx->num_cus, ctx->flag_mask, k,
                                     stream, &wl);
    if (st != VF_OK) {
        if (st == VF_EHIP) ctx->counters_dirty = true;
        return st;
    }
    const int mode = wl.mode;
    ctx->pending = false;
    ctx->last_batch = false;
    if (recheck) {
        const int emode = is_amnf(filter) ? amnfe_mode(mode) : mode;
        if (ap->flags & VF_DEFER_RECHECK) {
            ctx->pending = true;
            ctx->pend_k = k;
            ctx->pend_filter = filter;
            ctx->pend_mode = emode;
            ctx->pend_window = window;
            ctx->pend_pixels = pixels;
        } else if ((st = launch_recheck_call(ctx, filter, emode, window, k, pixels, stream)) != VF_OK) {
            return st;
        }
    }
    ctx->last_windows = pixels;
    ctx->last_blocks = wl.blocks;
    ctx->last_tile_w = wl.tile_w;
    ctx->last_tile_h = wl.tile_h;
    ctx->last_recheck = recheck;
    ctx->last_streaming = wl.streaming;
    return VF_OK;
}

int launch_angle(int filter, int window, int eval, int n_lo, int n_hi, const KParams& p, int blocks,
                 void* stream);
int launch_angle_stream(int window, int filter, int eval, int n_lo, int n_hi, const KParams& p,
                        int blocks, void* stream);

}  // namespace vf

namespace vf {
int launch_angle_w3(int, int, int, int, const KParams&, int, void*);
int launch_angle_w5(int, int, int, int, const KParams&, int, void*);
int launch_angle_w7(int, int, int, int, const KParams&, int, void*);
int launch_angle_stream_w3(int, int, int, int, const KParams&, int, void*);
int launch_angle_stream_w5(int, int, int, int, const KParams&, int, void*);
int launch_angle_stream_w7(int, int, int, int, const KParams&, int, void*);

int launch_angle_stream_var_w3(int, int, int, int, int, const KParams&, int, void*);
int launch_angle_stream_var_w5(int, int, int, int, int, const KParams&, int, void*);
int launch_angle_stream_var_w7(int, int, int, int, int, const KParams&, int, void*);

int launch_angle_stream_var(int window, int filter, int eval, int n_lo, int n_hi, int variant,
                            const KParams& p, int blocks, void* stream) {
    switch (window) {
    case 3: return launch_angle_stream_var_w3(filter, eval, n_lo, n_hi, variant, p, blocks, stream);
    case 5: return launch_angle_stream_var_w5(filter, eval, n_lo, n_hi, variant, p, blocks, stream);
    case 7: return launch_angle_stream_var_w7(filter, eval, n_lo, n_hi, variant, p, blocks, stream);
    }
    return -1;
}

int launch_angle_stream(int window, int filter, int eval, int n_lo, int n_hi, const KParams& p,
                        int blocks, void* stream) {
    switch (window) {
    case 3: return launch_angle_stream_w3(filter, eval, n_lo, n_hi, p, blocks, stream);
    case 5: return launch_angle_stream_w5(filter, eval, n_lo, n_hi, p, blocks, stream);
    case 7: return launch_angle_stream_w7(filter, eval, n_lo, n_hi, p, blocks, stream);
    }
    return -1;
}

int launch_angle(int filter, int window, int eval, int n_lo, int n_hi, const KParams& p, int blocks,
                 void* stream) {
    switch (window) {
    case 3: return launch_angle_w3(filter, eval, n_lo, n_hi, p, blocks, stream);
    case 5: return launch_angle_w5(filter, eval, n_lo, n_hi, p, blocks, stream);
    case 7: return launch_angle_w7(filter, eval, n_lo, n_hi, p, blocks, stream);
    }
    return -1;
}
}  // namespace vf

using namespace vf;

extern "C" {

vf_status vf_create(int32_t device, vf_context** out) {
    if (!out) return set_error(VF_EINVAL, "out is null");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return set_error(VF_EINVAL, "no such device");
    DeviceGuard dg(device);
    if (!dg.ok) return set_error(VF_EHIP, "hipSetDevice failed");
    vf_context* ctx = new vf_context();   // value-initialised: every scalar member is zero
    ctx->device = device;
    ctx->strip_rows = 0;   // streaming strip height sized per call from occupancy (auto_strip_rows)
    if (hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        ctx->num_cus < 1)
        ctx->num_cus = 1;
    if (const char* env = std::getenv("VF_STRIP_ROWS")) {
        const int v = std::atoi(env);
        if (v >= 1 && v <= 4096) ctx->strip_rows = v;
    }
    e = hipMalloc((void**)&ctx->counters, kCounterSlots * sizeof(uint32_t));
    if (e != hipSuccess) {
        delete ctx;
        return set_error(VF_ENOMEM, "cannot allocate counters");
    }
    e = hipMemset(ctx->counters, 0, kCounterSlots * sizeof(uint32_t));
    if (e != hipSuccess) {
        (void)hipFree(ctx->counters);
        delete ctx;
        return hip_fail(e, "hipMemset");
    }
    *out = ctx;
    return VF_OK;
}

vf_status vf_destroy(vf_context* ctx) {
    if (!ctx) return VF_OK;
    DeviceGuard dg(ctx->device);
    (void)hipDeviceSynchronize();
    batch_release(ctx);
    if (ctx->qual_ws) (void)hipFree(ctx->qual_ws);
    if (ctx->flag_list) (void)hipFree(ctx->flag_list);
    if (ctx->flag_mask) (void)hipFree(ctx->flag_mask);
    if (ctx->counters) (void)hipFree(ctx->counters);
    delete ctx;
    return VF_OK;
}

vf_status vf_filter_vdf(vf_context* ctx, const vf_image* img, int32_t window, const vf_approx* approx,
                        void* hip_stream) {
    return run_filter(ctx, img, VF_FILTER_VDF, window, 0.0, approx, hip_stream);
}

vf_status vf_filter_ddf(vf_context* ctx, const vf_image* img, int32_t window, double p,
                        const vf_approx* approx, void* hip_stream) {
    return run_filter(ctx, img, VF_FILTER_DDF, window, p, approx, hip_stream);
}

vf_status vf_filter_fuzzy_exp(vf_context* ctx, const vf_image* img, int32_t window, double kappa,
                              int32_t kernel, const vf_approx* approx, void* hip_stream) {
    if (kernel != VF_KERNEL_EXP && kernel != VF_KERNEL_GAUSS)
        return set_error(VF_EINVAL, "kernel must be VF_KERNEL_EXP or VF_KERNEL_GAUSS");
    return run_filter(ctx, img, kernel == VF_KERNEL_GAUSS ? VF_FILTER_AMNFG : VF_FILTER_AMNFE, window, kappa,
                      approx, hip_stream);
}

vf_status vf_filter_log(vf_context* ctx, const vf_image* img, int32_t window, double cutoff,
                        const vf_approx* approx, void* hip_stream) {
    return run_filter(ctx, img, VF_FILTER_EVMF, window, cutoff, approx, hip_stream);
}

vf_status vf_filter_batch(vf_context* ctx, const vf_batch_item* items, int32_t count, void* hip_stream) {
    return run_batch(ctx, items, count, hip_stream);
}

vf_status vf_recheck_pending(vf_context* ctx, void* hip_stream) {
    if (!ctx) return set_error(VF_EINVAL, "context is null");
    if (!ctx->pending) return VF_OK;
    DeviceGuard dg(ctx->device);
    ctx->pending = false;
    return launch_recheck_call(ctx, ctx->pend_filter, ctx->pend_mode, ctx->pend_window, ctx->pend_k,
                               ctx->pend_pixels, hip_stream);
}

vf_status vf_minimax_coeffs(int32_t func, double a, double b, int32_t degree, int32_t basis,
                            double* coeffs_out, double* err_out) {
    return minimax_coeffs(func, a, b, degree, basis, coeffs_out, err_out);
}

vf_status vf_minimax_rational(int32_t func, double a, double b, int32_t n, int32_t m, double* num_out,
                              double* den_out, double* err_out) {
    return minimax_rational(func, a, b, n, m, num_out, den_out, err_out);
}

vf_status vf_get_approximant(int32_t filter, int32_t window, double param, const vf_approx* approx,
                             float* lo, int32_t* n_lo, float* hi, int32_t* n_hi, double* eps_out) {
    Prepared P;
    vf_status st = prepare(filter, window, param, approx, &P);
    if (st != VF_OK) return st;
    if (lo) std::memcpy(lo, P.lo, sizeof(P.lo));
    if (hi) std::memcpy(hi, P.hi, sizeof(P.hi));
    if (n_lo) *n_lo = P.n_lo;
    if (n_hi) *n_hi = P.n_hi;
    if (eps_out) *eps_out = P.eps;
    return VF_OK;
}

vf_status vf_eval_function(vf_context* ctx, int32_t filter, int32_t window, double param,
                           const vf_approx* approx, const float* in, float* out, int64_t count,
                           void* hip_stream) {
    if (!ctx) return set_error(VF_EINVAL, "context is null");
    if (count < 0 || (count > 0 && (!in || !out))) return set_error(VF_EINVAL, "bad arrays");
    Prepared P;
    vf_status st = prepare(filter, window, param, approx, &P);
    if (st != VF_OK) return st;
    if (P.variant == 3) return set_error(VF_EUNSUPPORTED, "FP64 precision evaluates whole windows only");
    if (count == 0) return VF_OK;
    DeviceGuard dg(ctx->device);
    KParams k;
    vf_image dummy{};
    dummy.height = dummy.width = 1;
    fill_kparams(&dummy, P, &k);
    int rc = launch_eval_function(filter, P.eval, P.n_lo, P.n_hi, P.variant, k, in, out, count, hip_stream);
    if (rc < 0) return set_error(VF_EUNSUPPORTED, "no evaluator for this approximant");
    if (rc != 0) return hip_fail((hipError_t)rc, "evaluation kernel launch");
    return VF_OK;
}

vf_status vf_get_stats(vf_context* ctx, vf_stats* out) {
    if (!ctx || !out) return set_error(VF_EINVAL, "null argument");
    DeviceGuard dg(ctx->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    uint64_t flagged = 0;
    if (ctx->last_batch) {
        vf_status st = batch_flagged(ctx, &flagged);
        if (st != VF_OK) return st;
    } else if (ctx->last_recheck) {
        uint32_t f = 0;
        e = hipMemcpy(&f, ctx->counters + ctx->last_slot, sizeof(f), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
        flagged = f;
    }
    std::memset(out, 0, sizeof(*out));
    out->windows = ctx->last_windows;
    out->flagged = flagged;
    out->streaming = ctx->last_streaming ? 1 : 0;
    out->tile_w = ctx->last_tile_w;
    out->tile_h = ctx->last_tile_h;
    out->workgroups = (int32_t)(ctx->last_blocks > 0x7fffffff ? 0x7fffffff : ctx->last_blocks);
    return VF_OK;
}

const char* vf_status_string(int32_t status) {
    switch (status) {
    case VF_OK: return "ok";
    case VF_EINVAL: return "invalid argument";
    case VF_EDOMAIN: return "interval outside the function's domain";
    case VF_ENOCONV: return "Remez exchange did not converge";
    case VF_EHIP: return "HIP runtime error";
    case VF_ENOMEM: return "out of device memory";
    case VF_EUNSUPPORTED: return "unsupported combination";
    }
    return "unknown status";
}

const char* vf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
