// vf_filter_vdf_noalloc: the vector directional filter without any device
// allocation, for callers that cannot allocate (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc). The re-check workspace that
// vf_filter_vdf takes from its context lives here in a file-scope device
// array: each GPU holds its own copy from the time the library's code is
// loaded on it until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "context.h"

namespace vf {
namespace {

// Layout: two counters (this call's flagged windows; a spare slot the re-check
// kernel clears), padded to 256 bytes, then the re-check list of up to
// kNoAllocPixels pixel indices, then their candidate masks. The list must hold
// one entry per pixel of the image (every window may be flagged), which
// bounds the image size: 2^20 pixels, 12 MiB of scratch in all.
constexpr uint32_t kNoAllocPixels = 1u << 20;
constexpr size_t kNoAllocCounterBytes = 256;
constexpr size_t kNoAllocListBytes = (size_t)kNoAllocPixels * sizeof(uint32_t);
constexpr size_t kNoAllocBytes = kNoAllocCounterBytes + kNoAllocListBytes + (size_t)kNoAllocPixels * sizeof(uint64_t);

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// In host code `scratch` names a host-side stand-in, not device memory: every
// use goes through the device address found once per device.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices];

// The scratch address on `device`, which must be current.
vf_status scratch_on(int device, unsigned char** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the no-allocation scratch");
        if (!ptr) return set_error(VF_EHIP, "hipGetSymbolAddress returned a null scratch address");
        g_scratch[device] = (unsigned char*)ptr;
    }
    *out = g_scratch[device];
    return VF_OK;
}

}  // namespace
}  // namespace vf

using namespace vf;

extern "C" vf_status vf_filter_vdf_noalloc(int32_t device, const vf_image* img, int32_t window,
                                           const vf_approx* approx, void* hip_stream) {
    vf_status st = validate_image(img);
    if (st != VF_OK) return st;
    if (!approx) return set_error(VF_EINVAL, "approx is null");
    if (approx->flags & (VF_DEFER_RECHECK | VF_TUNED))
        return set_error(VF_EINVAL, "VF_DEFER_RECHECK and VF_TUNED need a context (use vf_filter_vdf)");
    const uint64_t pixels = (uint64_t)img->height * (uint64_t)img->width;
    if (pixels > kNoAllocPixels)
        return set_error(VF_EINVAL, "image larger than the no-allocation scratch: at most 1048576 pixels");
    Prepared P;
    if ((st = prepare(VF_FILTER_VDF, window, 0.0, approx, &P)) != VF_OK) return st;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count || device >= kMaxDevices) return set_error(VF_EINVAL, "no such device");
    DeviceGuard dg(device);
    if (!dg.ok) return set_error(VF_EHIP, "hipSetDevice failed");
    unsigned char* base = nullptr;
    if ((st = scratch_on(device, &base)) != VF_OK) return st;
    KParams k;
    fill_kparams(img, P, &k);
    if (P.variant == 3) {   // every window in FP64: no scratch needed
        const int blocks = (int)(pixels < 65536 ? pixels : 65536);
        const int rc = launch_fp64(VF_FILTER_VDF, P.eval, window, k, blocks, hip_stream);
        return rc != 0 ? hip_fail((hipError_t)rc, "FP64 window kernel launch") : VF_OK;
    }
    int num_cus = 1;
    if (hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || num_cus < 1)
        num_cus = 1;
    const bool recheck = !(approx->flags & VF_NO_RECHECK);
    uint32_t* counters = reinterpret_cast<uint32_t*>(base);
    k.recheck = recheck ? 1 : 0;
    k.flag_list = reinterpret_cast<uint32_t*>(base + kNoAllocCounterBytes);
    k.flag_count = counters;
    k.next_count = counters + 1;
    k.flag_cap = (uint32_t)(recheck ? pixels : 0);
    uint64_t* masks = reinterpret_cast<uint64_t*>(base + kNoAllocCounterBytes + kNoAllocListBytes);
    if (recheck) {
        // the previous call on this GPU left its count behind: clear it (a fill
        // kernel, not a memset, so that the call can be captured in a graph)
        const int rc = launch_fill_u32(counters, 2u, 0u, hip_stream);
        if (rc != 0) return hip_fail((hipError_t)rc, "counter fill kernel launch");
    }
    WindowLaunch wl;
    if ((st = launch_window_kernels(img, VF_FILTER_VDF, window, P, approx->flags, 0, num_cus, masks, k, hip_stream,
                                    &wl)) != VF_OK)
        return st;
    if (recheck) {
        const uint64_t want = pixels / 64;
        const int rblocks = (int)(want < 1 ? 1 : (want > 16384 ? 16384 : want));
        const int rc = launch_recheck(VF_FILTER_VDF, wl.mode, window, k, rblocks, hip_stream);
        if (rc != 0) return hip_fail((hipError_t)rc, "re-check kernel launch");
    }
    return VF_OK;
}
