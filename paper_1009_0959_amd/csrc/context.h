// Host-side context of the vf library and the helpers its translation units
// share (argument validation, error reporting, kernel parameter set-up).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "vf_internal.h"

namespace vf {
struct BatchGraph;   // cached batch submission (batch_host.cpp)

// One autotuned configuration: for calls with this filter, window, dtype and
// evaluation kind, the kernel, tile height, degree, scheme and precision that
// ran fastest on the tuning sample within the caller's error target.
struct TuneEntry {
    int filter, window, dtype, eval;
    int direct;        // 1: per-window kernel, 0: streaming kernel
    int strip_rows;    // streaming: output rows per strip
    int degree, scheme, precision;
    double ms, func_err;
};
}

struct vf_context {
    int device;
    uint32_t* counters;     // device: kCounterSlots per-call flagged counts
    uint32_t* flag_list;    // device: flagged pixel indices
    uint64_t* flag_mask;    // device: candidate members of each flagged window (angle filters)
    uint64_t flag_cap;
    int slot;               // counter slot of the next call with a re-check
    int last_slot;
    uint64_t last_blocks;
    uint64_t last_windows;
    int last_tile_w, last_tile_h;
    bool last_recheck;
    bool last_streaming;
    bool pending;           // a VF_DEFER_RECHECK call awaits vf_recheck_pending
    vf::KParams pend_k;
    int pend_filter, pend_mode, pend_window;
    uint64_t pend_pixels;
    int strip_rows;         // output rows per strip of the streaming kernels (0: sized per call)
    int num_cus;            // compute units of the device (persistent grids)
    vf::BatchGraph* batch;  // last batch submission (graph, tables, workspace)
    bool last_batch;        // the last call was vf_filter_batch
    std::vector<vf::TuneEntry> tuned;   // autotuned configurations (tune.cpp)
    uint64_t tune_gen;      // bumped whenever `tuned` changes (cached batch graphs compare it)
    void* qual_ws;          // device: quality-criteria partials (kQualMaxBlocks + 1), allocated on first use
    bool counters_dirty;    // a call failed after its window kernel: the counter ring is re-zeroed first
};

namespace vf {

// Makes `dev` current for the scope and restores the previous device.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

vf_status hip_fail(hipError_t e, const char* what);
// Test hook: true when the environment variable VF_INJECT_HIP_ERROR names
// `site` ("window", "recheck" or "batch"); that launch then reports
// hipErrorLaunchFailure without launching, exercising the VF_EHIP path.
bool inject_hip_error(const char* site);
vf_status validate_image(const vf_image* img);
void fill_kparams(const vf_image* img, const Prepared& P, KParams* k);

// The window kernel of one filter call (api.cpp): the streaming kernel, or the
// per-window kernel with VF_DIRECT or where no streaming kernel exists, on the
// re-check workspace already set in k (flag list, counters, capacity); sets
// k's strip and mask fields. strip_rows <= 0: sized from the kernel's
// residency on num_cus compute units.
struct WindowLaunch {
    uint64_t blocks;
    int tile_w, tile_h;
    bool streaming;
    int mode;
};
vf_status launch_window_kernels(const vf_image* img, int filter, int window, const Prepared& P, uint32_t flags,
                                int strip_rows, int num_cus, uint64_t* mask_array, KParams& k, void* stream,
                                WindowLaunch* out);
int auto_strip_rows(int H, int strips_x, int window, int64_t slots);

// One filter call (api.cpp); strip_override > 0 replaces the streaming tile height.
vf_status run_filter(vf_context* ctx, const vf_image* img, int filter, int window, double param,
                     const vf_approx* ap, void* stream, int strip_override = 0);

// Replace degree, scheme, precision, kernel choice (VF_DIRECT) and tile height by
// the tuned entry for (filter, window, dtype, eval), if there is one (tune.cpp).
// For batches the scheme and precision stay Horner / FP32.
bool apply_tuned(const vf_context* ctx, int filter, int window, int dtype, vf_approx* ap, int* strip_rows,
                 bool batch);

// Batch submission (batch_host.cpp).
vf_status run_batch(vf_context* ctx, const vf_batch_item* items, int32_t count, void* stream);
vf_status batch_flagged(vf_context* ctx, uint64_t* flagged);
void batch_release(vf_context* ctx);

}  // namespace vf
