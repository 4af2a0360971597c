// Autotuner: for one filter family (filter, window, dtype, evaluation kind),
// time every candidate configuration on a sample image and keep the fastest
// whose approximant meets the caller's function-error target.
//
// Candidates: polynomial degree (every degree the evaluation kind accepts, or
// the one given), evaluation scheme (Horner, Estrin), precision (FP32, packed
// FP16) where the kernels implement them, and the kernel: the streaming kernel
// with strips of 16 .. 256 output rows (the tile height; every lane produces
// one pixel per row of its strip) or of the height sized from its occupancy,
// or the per-window kernel. Each candidate is
// a real filter call, re-check included, timed with HIP events on the caller's
// stream (one warm-up, the median of five); a later candidate replaces the
// best so far only when more than 1% faster.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "context.h"

namespace vf {

namespace {

std::vector<int> degrees_for(int filter, int eval) {
    const bool angle = filter == VF_FILTER_VDF || filter == VF_FILTER_DDF;
    switch (eval) {
    case VF_EVAL_EXACT: return {0};
    case VF_EVAL_PAPER: return angle ? std::vector<int>{4} : (is_amnf(filter) ? std::vector<int>{2, 3, 4}
                                                                                        : std::vector<int>{4});
    case VF_EVAL_SPLIT: return {3, 5, 7, 9};
    case VF_EVAL_CHORD: return {7, 9, 11, 13};
    case VF_EVAL_MINIMAX: return {2, 3, 4, 5, 6, 7, 8, 9};
    case VF_EVAL_RATIONAL: return {4};
    case VF_EVAL_RATFIT: return {1, 2, 3, 4};
    }
    return {};
}

TuneEntry* find_entry(std::vector<TuneEntry>& t, int filter, int window, int dtype, int eval) {
    for (TuneEntry& e : t)
        if (e.filter == filter && e.window == window && e.dtype == dtype && e.eval == eval) return &e;
    return nullptr;
}

}  // namespace

bool apply_tuned(const vf_context* ctx, int filter, int window, int dtype, vf_approx* ap, int* strip_rows,
                 bool batch) {
    for (const TuneEntry& e : ctx->tuned) {
        if (e.filter != filter || e.window != window || e.dtype != dtype || e.eval != ap->eval) continue;
        ap->degree = e.degree;
        ap->scheme = batch ? VF_SCHEME_HORNER : e.scheme;
        ap->precision = batch ? VF_PREC_FP32 : e.precision;
        ap->flags = (ap->flags & ~VF_DIRECT) | (e.direct ? VF_DIRECT : 0u);
        // a batch class sizes its strips over all its images (a height tuned
        // on one sample image measured slower there)
        if (strip_rows && e.strip_rows > 0 && !batch) *strip_rows = e.strip_rows;
        return true;
    }
    return false;
}

}  // namespace vf

using namespace vf;

extern "C" {

vf_status vf_autotune(vf_context* ctx, int32_t filter, int32_t window, double param, const vf_approx* approx,
                      const vf_image* sample, double max_func_err, vf_tune_result* out, void* hip_stream) {
    if (!ctx || !approx || !sample || !out) return set_error(VF_EINVAL, "null argument");
    vf_status st = validate_image(sample);
    if (st != VF_OK) return st;
    if (filter < VF_FILTER_VDF || filter > VF_FILTER_EVMF) return set_error(VF_EINVAL, "unknown filter");
    std::vector<int> degrees = approx->degree > 0 ? std::vector<int>{approx->degree}
                                                  : degrees_for(filter, approx->eval);
    if (degrees.empty()) return set_error(VF_EINVAL, "unknown evaluation kind");
    const bool angle = filter == VF_FILTER_VDF || filter == VF_FILTER_DDF;
    const bool chord = angle && approx->eval == VF_EVAL_CHORD;
    const bool fe_minimax = !angle && approx->eval == VF_EVAL_MINIMAX;

    struct Cand {
        int degree, scheme, precision, direct, strip;
        double err;
    };
    std::vector<Cand> cands;
    for (int d : degrees) {
        for (int prec : {VF_PREC_FP32, VF_PREC_FP16X2}) {
            if (prec == VF_PREC_FP16X2 && !chord && !fe_minimax) continue;
            for (int sch : {VF_SCHEME_HORNER, VF_SCHEME_ESTRIN}) {
                if (sch == VF_SCHEME_ESTRIN && (!chord || prec != VF_PREC_FP32)) continue;
                vf_approx a = *approx;
                a.degree = d;
                a.scheme = sch;
                a.precision = prec;
                Prepared P;
                if (prepare(filter, window, param, &a, &P) != VF_OK) continue;
                if (max_func_err > 0.0 && P.eps > max_func_err) continue;
                // every filter has streaming kernels; the per-window ones evaluate
                // Horner in FP32 only
                // (strip 0: the height sized from the kernel's occupancy per call)
                for (int strip : {0, 16, 32, 64, 128, 256}) cands.push_back({d, sch, prec, 0, strip, P.eps});
                if (P.variant == 0) cands.push_back({d, sch, prec, 1, 0, P.eps});
            }
        }
    }
    if (cands.empty()) return set_error(VF_EUNSUPPORTED, "no approximant meets the error target");

    DeviceGuard dg(ctx->device);
    if (!dg.ok) return set_error(VF_EHIP, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he;
    if ((he = hipEventCreate(&e0)) != hipSuccess || (he = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    int best = -1;
    double best_ms = 0.0;
    int tried = 0;
    for (size_t ci = 0; ci < cands.size() && st == VF_OK; ++ci) {
        const Cand& c = cands[ci];
        vf_approx a = *approx;
        a.degree = c.degree;
        a.scheme = c.scheme;
        a.precision = c.precision;
        a.flags = (approx->flags & ~(VF_DIRECT | VF_DEFER_RECHECK | VF_TUNED)) | (c.direct ? VF_DIRECT : 0u);
        std::vector<float> ms;
        for (int rep = 0; rep < 6 && st == VF_OK; ++rep) {
            if ((he = hipEventRecord(e0, s)) != hipSuccess) { st = hip_fail(he, "hipEventRecord"); break; }
            st = run_filter(ctx, sample, filter, window, param, &a, hip_stream, c.strip);
            if (st != VF_OK) break;
            if ((he = hipEventRecord(e1, s)) != hipSuccess) { st = hip_fail(he, "hipEventRecord"); break; }
            if ((he = hipEventSynchronize(e1)) != hipSuccess) { st = hip_fail(he, "hipEventSynchronize"); break; }
            float t = 0.0f;
            if ((he = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) { st = hip_fail(he, "hipEventElapsedTime"); break; }
            if (rep > 0) ms.push_back(t);
        }
        if (st == VF_EUNSUPPORTED) {   // this combination has no kernel: skip it
            st = VF_OK;
            continue;
        }
        if (st != VF_OK) break;
        ++tried;
        std::sort(ms.begin(), ms.end());
        const double med = ms[ms.size() / 2];
        // a later candidate must win by more than 1% (timing noise), so ties go
        // to the earlier, simpler configuration: lower degree, Horner, FP32,
        // the occupancy-sized strips
        if (best < 0 || med < 0.99 * best_ms) {
            best = (int)ci;
            best_ms = med;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != VF_OK) return st;
    if (best < 0) return set_error(VF_EUNSUPPORTED, "no candidate configuration could run");
    const Cand& c = cands[best];
    TuneEntry e{filter, window, sample->dtype, approx->eval, c.direct, c.strip, c.degree, c.scheme, c.precision,
                best_ms, c.err};
    if (TuneEntry* old = find_entry(ctx->tuned, filter, window, sample->dtype, approx->eval)) *old = e;
    else ctx->tuned.push_back(e);
    ++ctx->tune_gen;
    std::memset(out, 0, sizeof(*out));
    out->direct = c.direct;
    out->strip_rows = c.strip;
    out->degree = c.degree;
    out->scheme = c.scheme;
    out->precision = c.precision;
    out->ms = best_ms;
    out->func_err = c.err;
    out->candidates = tried;
    return VF_OK;
}

vf_status vf_tune_save(vf_context* ctx, const char* path) {
    if (!ctx || !path) return set_error(VF_EINVAL, "null argument");
    FILE* f = std::fopen(path, "w");
    if (!f) return set_error(VF_EINVAL, "cannot open the file for writing");
    std::fprintf(f, "# vf tune v1: filter window dtype eval direct strip_rows degree scheme precision ms func_err\n");
    for (const TuneEntry& e : ctx->tuned)
        std::fprintf(f, "%d %d %d %d %d %d %d %d %d %.6g %.6g\n", e.filter, e.window, e.dtype, e.eval, e.direct,
                     e.strip_rows, e.degree, e.scheme, e.precision, e.ms, e.func_err);
    const bool ok = std::fclose(f) == 0;
    return ok ? VF_OK : set_error(VF_EINVAL, "write failed");
}

vf_status vf_tune_load(vf_context* ctx, const char* path) {
    if (!ctx || !path) return set_error(VF_EINVAL, "null argument");
    FILE* f = std::fopen(path, "r");
    if (!f) return set_error(VF_EINVAL, "cannot open the file");
    std::vector<TuneEntry> got;
    char line[512];
    vf_status st = VF_OK;
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        TuneEntry e{};
        if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d %lf %lf", &e.filter, &e.window, &e.dtype, &e.eval,
                        &e.direct, &e.strip_rows, &e.degree, &e.scheme, &e.precision, &e.ms, &e.func_err) != 11) {
            st = set_error(VF_EINVAL, "malformed tune file");
            break;
        }
        // the entry must describe a valid approximant and tile height
        vf_approx a{};
        a.eval = e.eval;
        a.degree = e.degree;
        a.scheme = e.scheme;
        a.precision = e.precision;
        Prepared P;
        // (a parameter the entry's approximant accepts: the EVMF rational needs T >= 0.05)
        const double param = e.filter == VF_FILTER_DDF
                                 ? 0.5
                                 : (is_amnf(e.filter) ? 0.33 : (e.eval == VF_EVAL_PAPER ? 0.05 : 0.0));
        if (prepare(e.filter, e.window, param, &a, &P) != VF_OK || P.variant == 3 ||
            (e.dtype != VF_U8 && e.dtype != VF_U16) ||
            e.strip_rows < 0 || e.strip_rows > 4096 || (e.direct != 0 && e.direct != 1)) {
            st = set_error(VF_EINVAL, "tune file entry out of range");
            break;
        }
        got.push_back(e);
    }
    std::fclose(f);
    if (st != VF_OK) return st;
    for (const TuneEntry& e : got) {
        if (TuneEntry* old = find_entry(ctx->tuned, e.filter, e.window, e.dtype, e.eval)) *old = e;
        else ctx->tuned.push_back(e);
    }
    ++ctx->tune_gen;
    return VF_OK;
}

vf_status vf_tune_clear(vf_context* ctx) {
    if (!ctx) return set_error(VF_EINVAL, "null argument");
    ctx->tuned.clear();
    ++ctx->tune_gen;
    return VF_OK;
}

}  // extern "C"
