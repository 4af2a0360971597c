// Batch submission: many images of uneven size, each with its own filter,
// window and approximant, as one captured HIP graph.
//
// Images are grouped into classes (same filter, window, parameter and
// approximant); each class is one persistent kernel whose workgroups pull
// tiles from an atomic counter over a table sorted largest image first, then
// the class's FP64 re-check kernel and its overflow pass (every window in
// FP64, which runs only when the class flagged more windows than its capped
// re-check list holds). The graph starts with a fill kernel that clears the
// classes' tile and flag counters (no memset node), then forks into up to
// four branches, each a chain of classes (heaviest first, spread over the
// branches longest-processing-time first), so that one class's tail overlaps
// the next class's start; the branches join before the graph ends. It is
// captured on context-owned streams of default priority, instantiated once
// and launched on the caller's stream; a later call with the same item list
// (pointers, sizes, filters) launches the cached graph again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "context.h"

namespace vf {

struct BatchClass {
    int filter, window;
    double param;
    vf_approx ap;             // after the tuned configuration is applied
    int strip_rows;           // streaming tile height of the class
    Prepared P;
    int mode;                 // kernel evaluation mode
    bool streaming;
    bool recheck;
    std::vector<int> members; // item indices, largest first
    uint64_t pixels;
    uint64_t tiles;
    size_t table_off;         // first BatchItem of the class in the device table
    size_t flag_off;          // first slot of the class in the re-check lists
    uint64_t flag_cap;        // its slots in the re-check lists
    int branch;               // graph branch (capture stream) that runs the class
};

constexpr int kMaxBranches = 4;

struct BatchGraph {
    std::vector<vf_batch_item> items;   // signature of the captured submission
    int strip_rows = 0;
    uint64_t tune_gen = 0;              // tuned configurations the graph was built with
    long cap_env = -1, streams_env = -1;   // VF_BATCH_FLAG_CAP / VF_BATCH_STREAMS it was built with
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture = nullptr;      // branch 0; branches 1.. fork from it
    hipStream_t forks[kMaxBranches] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kMaxBranches] = {};
    void* ws = nullptr;                 // tables, counters and re-check lists
    size_t ws_bytes = 0;
    uint32_t* counters = nullptr;       // 2 per class: next tile, flagged windows
    int nclasses = 0;
    uint64_t pixels = 0;
    bool any_recheck = false;
    bool any_streaming = false;
    uint64_t tiles = 0;
};

namespace {

constexpr uint32_t kFlagMask = VF_NO_RECHECK | VF_DIRECT | VF_TUNED;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// A non-negative integer from the environment, or -1 when unset or malformed.
long env_count(const char* name) {
    const char* v = std::getenv(name);
    if (!v || !*v) return -1;
    char* end = nullptr;
    const long n = std::strtol(v, &end, 10);
    return (*end == '\0' && n >= 0) ? n : -1;
}

// Re-check list slots of a class: an eighth of its windows (half for the
// exact-function kernels, whose FP32 bounds flag more windows), at least 2^16
// and at most all of them. VF_BATCH_FLAG_CAP, when set, replaces the rule
// (it forces the overflow pass in tests).
uint64_t flag_capacity(const BatchClass& c) {
    if (!c.recheck) return 0;
    const long forced = env_count("VF_BATCH_FLAG_CAP");
    if (forced >= 0) return std::min<uint64_t>((uint64_t)forced, c.pixels);
    const uint64_t share = c.mode == EV_EXACT ? c.pixels / 2 : c.pixels / 8;
    return std::min<uint64_t>(c.pixels, std::max<uint64_t>(share, 1u << 16));
}

// Graph branches: VF_BATCH_STREAMS (1 .. 4) when set, else 4; never more than
// there are classes.
int branch_count(int nclasses) {
    const long forced = env_count("VF_BATCH_STREAMS");
    const int want = (forced >= 1 && forced <= kMaxBranches) ? (int)forced : kMaxBranches;
    return std::max(1, std::min(want, nclasses));
}

bool same_class(const BatchClass& c, const vf_batch_item& it, const vf_approx& a, int strip_rows) {
    return c.filter == it.filter && c.window == it.window &&
           std::memcmp(&c.param, &it.param, sizeof(double)) == 0 && c.ap.eval == a.eval &&
           c.ap.degree == a.degree && c.ap.precision == a.precision && c.ap.scheme == a.scheme &&
           (c.ap.flags & kFlagMask) == (a.flags & kFlagMask) && c.strip_rows == strip_rows;
}

bool same_items(const std::vector<vf_batch_item>& a, const vf_batch_item* b, int32_t n) {
    if ((int32_t)a.size() != n) return false;
    for (int32_t i = 0; i < n; ++i) {
        const vf_batch_item& x = a[i];
        const vf_batch_item& y = b[i];
        if (x.img.src != y.img.src || x.img.dst != y.img.dst || x.img.height != y.img.height ||
            x.img.width != y.img.width || x.img.src_pitch != y.img.src_pitch ||
            x.img.dst_pitch != y.img.dst_pitch || x.img.dtype != y.img.dtype || x.filter != y.filter ||
            x.window != y.window || std::memcmp(&x.param, &y.param, sizeof(double)) != 0 ||
            x.approx.eval != y.approx.eval || x.approx.degree != y.approx.degree ||
            x.approx.precision != y.approx.precision || x.approx.scheme != y.approx.scheme ||
            (x.approx.flags & kFlagMask) != (y.approx.flags & kFlagMask))
            return false;
    }
    return true;
}

// No destination may overlap any source or another destination: the batch
// runs its images concurrently, so results could otherwise depend on order.
vf_status check_overlaps(const vf_batch_item* items, int32_t n) {
    struct Range {
        uintptr_t a, b;
        bool dst;
    };
    std::vector<Range> r;
    r.reserve(2 * (size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const vf_image& im = items[i].img;
        const int64_t row = 3 * (int64_t)im.width * (im.dtype == VF_U16 ? 2 : 1);
        const uintptr_t s = (uintptr_t)im.src, d = (uintptr_t)im.dst;
        r.push_back({s, s + (uintptr_t)((im.height - 1) * im.src_pitch + row), false});
        r.push_back({d, d + (uintptr_t)((im.height - 1) * im.dst_pitch + row), true});
    }
    std::sort(r.begin(), r.end(), [](const Range& x, const Range& y) { return x.a < y.a; });
    uintptr_t end_all = 0, end_dst = 0;
    for (const Range& x : r) {
        if (x.dst ? x.a < end_all : x.a < end_dst)
            return set_error(VF_EINVAL, "a batch destination overlaps a source or another destination");
        end_all = std::max(end_all, x.b);
        if (x.dst) end_dst = std::max(end_dst, x.b);
    }
    return VF_OK;
}

int angle_batch(int window, int filter, int mode, const Prepared& P, bool streaming, const BatchParams& bp,
                int num_cus, void* stream, bool probe) {
    switch (window) {
    case 3: return launch_angle_batch_w3(filter, mode, P.n_lo, P.n_hi, streaming, bp, num_cus, stream, probe);
    case 5: return launch_angle_batch_w5(filter, mode, P.n_lo, P.n_hi, streaming, bp, num_cus, stream, probe);
    case 7: return launch_angle_batch_w7(filter, mode, P.n_lo, P.n_hi, streaming, bp, num_cus, stream, probe);
    }
    return -1;
}

int class_launch(const BatchClass& c, const BatchParams& bp, int num_cus, void* stream, bool probe) {
    if (c.filter == VF_FILTER_VDF || c.filter == VF_FILTER_DDF)
        return angle_batch(c.window, c.filter, c.mode, c.P, c.streaming, bp, num_cus, stream, probe);
    if (is_amnf(c.filter))
        return c.streaming ? launch_amnfe_stream_batch(c.filter, c.window, c.mode, bp, num_cus, stream, probe)
                           : launch_amnfe_batch(c.filter, c.window, c.mode, bp, num_cus, stream, probe);
    return c.streaming ? launch_evmf_stream_batch(c.window, c.mode, bp, num_cus, stream, probe)
                       : launch_evmf_batch(c.window, c.mode, bp, num_cus, stream, probe);
}

// Tile geometry of one image in a class (must match the tile decoding of the
// class's kernel).
void tile_grid(const BatchClass& c, int H, int W, int strip_rows, int* tiles_x, uint64_t* tiles) {
    if (c.streaming) {
        const int outw = 64 - (c.window - 1);
        *tiles_x = (W + outw - 1) / outw;
        *tiles = (uint64_t)*tiles_x * (uint64_t)((H + strip_rows - 1) / strip_rows);
        return;
    }
    const bool angle = c.filter == VF_FILTER_VDF || c.filter == VF_FILTER_DDF;
    const int th = (angle && c.window == 7) ? 2 : kTileY;
    *tiles_x = (W + kTileX - 1) / kTileX;
    *tiles = (uint64_t)*tiles_x * (uint64_t)((H + th - 1) / th);
}

void destroy_graph(BatchGraph* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->exec = nullptr;
    g->graph = nullptr;
    g->items.clear();
}

// Build the classes, the device tables and the graph for `items`.
vf_status build_graph(vf_context* ctx, const vf_batch_item* items, int32_t n) {
    BatchGraph* g = ctx->batch;
    std::vector<BatchClass> classes;
    for (int32_t i = 0; i < n; ++i) {
        const vf_batch_item& it = items[i];
        vf_approx a = it.approx;
        int strip = ctx->strip_rows;   // 0: sized per class below
        if (a.flags & VF_TUNED) apply_tuned(ctx, it.filter, it.window, it.img.dtype, &a, &strip, true);
        size_t c = 0;
        while (c < classes.size() && !same_class(classes[c], it, a, strip)) ++c;
        if (c == classes.size()) {
            BatchClass k{};
            k.filter = it.filter;
            k.window = it.window;
            k.param = it.param;
            k.ap = a;
            k.ap.flags &= kFlagMask;
            k.strip_rows = strip;
            vf_status st = prepare(it.filter, it.window, it.param, &a, &k.P);
            if (st != VF_OK) return st;
            if (k.P.variant != 0)
                return set_error(VF_EUNSUPPORTED, "batches evaluate with Horner's scheme in FP32 (FP64 re-check)");
            k.mode = k.P.eval;
            if (is_amnf(k.filter)) k.mode = amnfe_mode(k.mode);
            k.recheck = !(a.flags & VF_NO_RECHECK);
            BatchParams none{};
            k.streaming = false;
            if (!(a.flags & VF_DIRECT)) {
                k.streaming = true;   // probe the streaming kernel of the class
                k.streaming = class_launch(k, none, 1, nullptr, true) == 0;
            }
            if (class_launch(k, none, 1, nullptr, true) != 0)
                return set_error(VF_EUNSUPPORTED, "no kernel for this filter/window/approximant");
            classes.push_back(k);
        }
        classes[c].members.push_back(i);
    }

    // streaming classes without a set height: the one of 16 .. 256 rows whose
    // tiles, handed out to the kernel's resident waves, finish soonest
    // (rounds of tiles x rows stepped per tile)
    for (BatchClass& c : classes) {
        if (!c.streaming || c.strip_rows > 0) continue;
        if (c.filter == VF_FILTER_EVMF) {   // as for single calls: the fixed height measured faster
            c.strip_rows = 64;
            continue;
        }
        int per_cu = 0;
        BatchParams none{};
        occupancy_query() = &per_cu;
        class_launch(c, none, 1, nullptr, false);
        occupancy_query() = nullptr;
        const uint64_t slots = (uint64_t)(per_cu > 0 ? per_cu : 1) * (uint64_t)(ctx->num_cus > 0 ? ctx->num_cus : 1);
        uint64_t best_cost = 0;
        c.strip_rows = 64;
        for (int rows : {16, 24, 32, 48, 64, 96, 128, 192, 256}) {
            uint64_t tiles = 0;
            for (int i : c.members) {
                int tx;
                uint64_t t;
                tile_grid(c, items[i].img.height, items[i].img.width, rows, &tx, &t);
                tiles += t;
            }
            const uint64_t cost = ((tiles + slots - 1) / slots) * (uint64_t)(rows + c.window - 1);
            if (best_cost == 0 || cost < best_cost) {
                best_cost = cost;
                c.strip_rows = rows;
            }
        }
    }

    // per-class tile tables, largest image first
    std::vector<BatchItem> table;
    uint64_t flag_slots = 0, pixels = 0, tiles_all = 0;
    for (BatchClass& c : classes) {
        std::vector<std::pair<uint64_t, int>> order;
        for (int i : c.members) {
            int tx;
            uint64_t t;
            tile_grid(c, items[i].img.height, items[i].img.width, c.strip_rows, &tx, &t);
            order.push_back({t, i});
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const std::pair<uint64_t, int>& a, const std::pair<uint64_t, int>& b) {
                             return a.first > b.first;
                         });
        c.table_off = table.size();
        c.pixels = 0;
        c.tiles = 0;
        c.members.clear();
        for (const auto& o : order) {
            const vf_image& im = items[o.second].img;
            BatchItem b{};
            b.src = (const unsigned char*)im.src;
            b.dst = (unsigned char*)im.dst;
            b.src_pitch = im.src_pitch;
            b.dst_pitch = im.dst_pitch;
            b.H = im.height;
            b.W = im.width;
            b.u16 = im.dtype == VF_U16;
            uint64_t t;
            tile_grid(c, im.height, im.width, c.strip_rows, &b.tiles_x, &t);
            b.first_tile = (uint32_t)c.tiles;
            b.first_pixel = (uint32_t)c.pixels;
            b.index = (int32_t)(table.size() - c.table_off);
            table.push_back(b);
            c.members.push_back(o.second);
            c.tiles += t;
            c.pixels += (uint64_t)im.height * (uint64_t)im.width;
        }
        if (c.tiles >= (1ull << 32) || c.pixels >= (1ull << 32))
            return set_error(VF_EUNSUPPORTED, "a batch class of 2^32 or more pixels is not supported");
        c.flag_off = flag_slots;
        c.flag_cap = flag_capacity(c);
        flag_slots += c.flag_cap;
        pixels += c.pixels;
        tiles_all += c.tiles;
    }
    // cost order: the heaviest classes first (pairs per window x pixels), each
    // to the branch with the least work so far
    auto cost = [](const BatchClass& c) { return (double)c.pixels * c.window * c.window * c.window * c.window; };
    std::stable_sort(classes.begin(), classes.end(),
                     [&](const BatchClass& a, const BatchClass& b) { return cost(a) > cost(b); });
    const int nb = branch_count((int)classes.size());
    {
        double load[kMaxBranches] = {};
        for (BatchClass& c : classes) {
            int best = 0;
            for (int b = 1; b < nb; ++b)
                if (load[b] < load[best]) best = b;
            c.branch = best;
            load[best] += cost(c);
        }
    }

    // workspace: [table][counters][flag pixels][flag items][candidate masks]
    const int nc = (int)classes.size();
    const size_t off_cnt = align_up(table.size() * sizeof(BatchItem), 256);
    const size_t off_flag = align_up(off_cnt + 2 * (size_t)nc * sizeof(uint32_t), 256);
    const size_t off_item = align_up(off_flag + flag_slots * sizeof(uint32_t), 256);
    const size_t off_mask = align_up(off_item + flag_slots * sizeof(uint32_t), 256);
    const size_t bytes = align_up(off_mask + flag_slots * sizeof(uint64_t), 256);
    hipError_t e;
    if (g->ws_bytes < bytes) {
        if (g->ws) (void)hipFree(g->ws);
        g->ws = nullptr;
        g->ws_bytes = 0;
        if ((e = hipMalloc(&g->ws, bytes)) != hipSuccess) {
            g->ws = nullptr;
            return set_error(VF_ENOMEM, "cannot allocate the batch workspace");
        }
        g->ws_bytes = bytes;
    }
    char* ws = (char*)g->ws;
    if (!table.empty() &&
        (e = hipMemcpy(ws, table.data(), table.size() * sizeof(BatchItem), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy (batch table)");
    g->counters = (uint32_t*)(ws + off_cnt);
    g->nclasses = nc;

    if (!g->capture && (e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking)) != hipSuccess) {
        g->capture = nullptr;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    g->forks[0] = g->capture;
    for (int b = 1; b < nb; ++b)
        if (!g->forks[b] && (e = hipStreamCreateWithFlags(&g->forks[b], hipStreamNonBlocking)) != hipSuccess) {
            g->forks[b] = nullptr;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
    if (!g->fork_ev && (e = hipEventCreateWithFlags(&g->fork_ev, hipEventDisableTiming)) != hipSuccess) {
        g->fork_ev = nullptr;
        return hip_fail(e, "hipEventCreateWithFlags");
    }
    for (int b = 1; b < nb; ++b)
        if (!g->join_ev[b] && (e = hipEventCreateWithFlags(&g->join_ev[b], hipEventDisableTiming)) != hipSuccess) {
            g->join_ev[b] = nullptr;
            return hip_fail(e, "hipEventCreateWithFlags");
        }
    if ((e = hipStreamBeginCapture(g->capture, hipStreamCaptureModeRelaxed)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    int rc = launch_fill_u32(g->counters, (uint32_t)(2 * nc), 0u, g->capture);
    // fork: every branch starts after the fill kernel
    int forked = 1;
    if (rc == 0 && nb > 1) {
        rc = (int)hipEventRecord(g->fork_ev, g->capture);
        for (int b = 1; b < nb && rc == 0; ++b) {
            rc = (int)hipStreamWaitEvent(g->forks[b], g->fork_ev, 0);
            if (rc == 0) forked = b + 1;
        }
    }
    for (int ci = 0; ci < nc && rc == 0; ++ci) {
        const BatchClass& c = classes[ci];
        hipStream_t s = g->forks[c.branch];
        BatchParams bp{};
        vf_image first = items[c.members[0]].img;
        fill_kparams(&first, c.P, &bp.base);
        bp.base.strip_rows = c.strip_rows;
        bp.base.recheck = c.recheck ? 1 : 0;
        bp.base.flag_list = c.recheck ? (uint32_t*)(ws + off_flag) + c.flag_off : nullptr;
        bp.base.flag_item = c.recheck ? (uint32_t*)(ws + off_item) + c.flag_off : nullptr;
        const bool masks = c.recheck && writes_masks(c.filter, c.window, c.mode, c.streaming);
        bp.base.flag_mask = masks ? (uint64_t*)(ws + off_mask) + c.flag_off : nullptr;
        bp.base.flag_count = g->counters + 2 * ci + 1;
        bp.base.next_count = nullptr;
        bp.base.flag_cap = (uint32_t)c.flag_cap;
        bp.items = (const BatchItem*)ws + c.table_off;
        bp.nitems = (int32_t)c.members.size();
        bp.total = (uint32_t)c.tiles;
        bp.counter = g->counters + 2 * ci;
        rc = inject_hip_error("batch") ? (int)hipErrorLaunchFailure : class_launch(c, bp, ctx->num_cus, s, false);
        if (rc == 0 && c.recheck) {
            const uint64_t want = c.pixels / 64;
            const int blocks = (int)(want < 1 ? 1 : (want > 16384 ? 16384 : want));
            rc = launch_recheck_batch(c.filter, c.mode, c.window, bp, blocks, s);
        }
        if (rc == 0 && c.recheck && c.flag_cap < c.pixels) {
            // a few waves per CU: the pass is idle unless the list overflowed
            const uint64_t want = (uint64_t)(ctx->num_cus > 0 ? ctx->num_cus : 1) * 16u;
            const int blocks = (int)(want < c.pixels ? want : c.pixels);
            rc = launch_overflow_batch(c.filter, c.mode, c.window, bp, (uint32_t)c.pixels, blocks, s);
        }
    }
    // join: the capture stream waits for every branch that was forked (also
    // after a failed launch, so that the capture can end)
    for (int b = 1; b < forked; ++b) {
        const hipError_t j1 = hipEventRecord(g->join_ev[b], g->forks[b]);
        const hipError_t j2 = j1 == hipSuccess ? hipStreamWaitEvent(g->capture, g->join_ev[b], 0) : j1;
        if (rc == 0 && j2 != hipSuccess) rc = (int)j2;
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g->capture, &graph);
    if (rc != 0) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail((hipError_t)rc, "batch kernel launch (capture)");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    g->graph = graph;
    g->exec = exec;
    g->items.assign(items, items + n);
    g->strip_rows = ctx->strip_rows;
    g->tune_gen = ctx->tune_gen;
    g->cap_env = env_count("VF_BATCH_FLAG_CAP");
    g->streams_env = env_count("VF_BATCH_STREAMS");
    g->pixels = pixels;
    g->tiles = tiles_all;
    g->any_recheck = false;
    g->any_streaming = false;
    for (const BatchClass& c : classes) {
        g->any_recheck = g->any_recheck || c.recheck;
        g->any_streaming = g->any_streaming || c.streaming;
    }
    return VF_OK;
}

}  // namespace

vf_status run_batch(vf_context* ctx, const vf_batch_item* items, int32_t n, void* stream) {
    if (!ctx) return set_error(VF_EINVAL, "context is null");
    if (n < 0 || (n > 0 && !items)) return set_error(VF_EINVAL, "bad item list");
    if (ctx->pending)
        return set_error(VF_EINVAL, "a deferred re-check is pending: call vf_recheck_pending first");
    for (int32_t i = 0; i < n; ++i) {
        vf_status st = validate_image(&items[i].img);
        if (st != VF_OK) return st;
        if (items[i].approx.flags & VF_DEFER_RECHECK)
            return set_error(VF_EINVAL, "VF_DEFER_RECHECK is not accepted in a batch");
    }
    vf_status st = check_overlaps(items, n);
    if (st != VF_OK) return st;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return set_error(VF_EHIP, "hipSetDevice failed");
    ctx->last_batch = true;
    ctx->last_recheck = false;
    ctx->last_windows = 0;
    ctx->last_blocks = 0;
    if (n == 0) {
        if (ctx->batch) ctx->batch->nclasses = 0;
        return VF_OK;
    }
    if (!ctx->batch) ctx->batch = new BatchGraph();
    BatchGraph* g = ctx->batch;
    if (!g->exec || g->strip_rows != ctx->strip_rows || g->tune_gen != ctx->tune_gen ||
        g->cap_env != env_count("VF_BATCH_FLAG_CAP") || g->streams_env != env_count("VF_BATCH_STREAMS") ||
        !same_items(g->items, items, n)) {
        // the cached graph and its tables may still be in use
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        destroy_graph(g);
        g->nclasses = 0;
        if ((st = build_graph(ctx, items, n)) != VF_OK) {
            destroy_graph(g);
            g->nclasses = 0;
            return st;
        }
    }
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    ctx->last_windows = g->pixels;
    ctx->last_blocks = g->tiles;
    ctx->last_recheck = g->any_recheck;
    ctx->last_streaming = g->any_streaming;
    ctx->last_tile_w = 0;
    ctx->last_tile_h = 0;
    return VF_OK;
}

vf_status batch_flagged(vf_context* ctx, uint64_t* flagged) {
    *flagged = 0;
    BatchGraph* g = ctx->batch;
    if (!g || g->nclasses == 0) return VF_OK;
    std::vector<uint32_t> c(2 * (size_t)g->nclasses);
    hipError_t e = hipMemcpy(c.data(), g->counters, c.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    for (int i = 0; i < g->nclasses; ++i) *flagged += c[2 * i + 1];
    return VF_OK;
}

void batch_release(vf_context* ctx) {
    BatchGraph* g = ctx->batch;
    if (!g) return;
    destroy_graph(g);
    if (g->capture) (void)hipStreamDestroy(g->capture);
    for (int b = 1; b < kMaxBranches; ++b) {
        if (g->forks[b]) (void)hipStreamDestroy(g->forks[b]);
        if (g->join_ev[b]) (void)hipEventDestroy(g->join_ev[b]);
    }
    if (g->fork_ev) (void)hipEventDestroy(g->fork_ev);
    if (g->ws) (void)hipFree(g->ws);
    delete g;
    ctx->batch = nullptr;
}

}  // namespace vf
