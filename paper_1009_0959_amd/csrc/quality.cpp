// vf_quality: the quality criteria of Section 4 (MAE, MSE, NCD) of a filtered
// image against its original, on the GPU (kern_quality.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>

#include "context.h"

using namespace vf;

extern "C" vf_status vf_quality(vf_context* ctx, const vf_image* img, vf_quality_result* out, void* hip_stream) {
    if (!ctx) return set_error(VF_EINVAL, "context is null");
    if (!img || !out) return set_error(VF_EINVAL, "null image or result");
    if (!img->src || !img->dst) return set_error(VF_EINVAL, "null original (src) or filtered image (dst)");
    if (img->dtype != VF_U8 && img->dtype != VF_U16) return set_error(VF_EINVAL, "dtype must be VF_U8 or VF_U16");
    if (img->height < 1 || img->width < 1) return set_error(VF_EINVAL, "height and width must be >= 1");
    const bool u16 = img->dtype == VF_U16;
    const uint64_t pixels = (uint64_t)img->height * (uint64_t)img->width;
    // the squared-difference sum stays below 2^64: 3 * 65535^2 per 16-bit pixel
    if (pixels >= (u16 ? (1ull << 30) : (1ull << 32)))
        return set_error(VF_EUNSUPPORTED, "images of 2^32 (8-bit) or 2^30 (16-bit) pixels or more are not supported");
    const int64_t row = 3 * (int64_t)img->width * (u16 ? 2 : 1);
    if (img->src_pitch < row || img->dst_pitch < row) return set_error(VF_EINVAL, "pitch smaller than a row");
    if (u16 && ((img->src_pitch | img->dst_pitch) & 1)) return set_error(VF_EINVAL, "uint16 pitches must be even");
    if (ctx->pending)
        return set_error(VF_EINVAL, "a deferred re-check is pending: call vf_recheck_pending first");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return set_error(VF_EHIP, "hipSetDevice failed");
    hipError_t e;
    if (!ctx->qual_ws && (e = hipMalloc(&ctx->qual_ws, (kQualMaxBlocks + 1) * sizeof(QualPartial))) != hipSuccess) {
        ctx->qual_ws = nullptr;
        return set_error(VF_ENOMEM, "cannot allocate the quality-criteria partials");
    }
    const uint64_t want = (pixels + 255) / 256;
    const uint64_t cap = std::min<uint64_t>((uint64_t)(ctx->num_cus > 0 ? ctx->num_cus : 1) * 8u, kQualMaxBlocks);
    const int blocks = (int)(want < cap ? want : cap);
    const int rc = launch_quality((const unsigned char*)img->src, img->src_pitch, (const unsigned char*)img->dst,
                                  img->dst_pitch, img->height, img->width, u16, blocks, ctx->qual_ws, hip_stream);
    if (rc != 0) return hip_fail((hipError_t)rc, "quality kernel launch");
    QualPartial r;
    if ((e = hipMemcpyAsync(&r, static_cast<QualPartial*>(ctx->qual_ws) + blocks, sizeof(r), hipMemcpyDeviceToHost,
                            (hipStream_t)hip_stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync (quality result)");
    if ((e = hipStreamSynchronize((hipStream_t)hip_stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    out->pixels = pixels;
    out->l1_sum = r.l1;
    out->l2sq_sum = r.l2sq;
    out->lab_diff_sum = r.lab_diff;
    out->lab_ref_sum = r.lab_ref;
    const double n3 = 3.0 * (double)pixels;
    out->mae = (double)r.l1 / n3;
    out->mse = (double)r.l2sq / n3;
    if (r.lab_ref > 0.0) out->ncd = r.lab_diff / r.lab_ref;
    else out->ncd = r.lab_diff == 0.0 ? 0.0 : std::numeric_limits<double>::infinity();
    return VF_OK;
}
