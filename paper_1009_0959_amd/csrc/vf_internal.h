// Internal declarations of the vf library (host and device). Not part of the ABI.
#pragma once

#include <stdint.h>

#include "../../include/vf.h"

namespace vf {

// Output tile of the window kernels: 64 columns (one wavefront) x 4 rows.
constexpr int kTileX = 64;
constexpr int kTileY = 4;
constexpr int kThreads = kTileX * kTileY;
constexpr int kMaxCoef = 16;

// Evaluation modes as the kernels see them (one per vf_eval value).
enum : int { EV_EXACT = 0, EV_PAPER = 1, EV_SPLIT = 2, EV_CHORD = 3, EV_MINIMAX = 4 };

// The two kernel functions of the AMNF equation share every code path.
constexpr bool is_amnf(int filter) { return filter == VF_FILTER_AMNFE || filter == VF_FILTER_AMNFG; }

// Kernel mode of an AMNFE / AMNFG evaluation: exact expf, a rational (EV_PAPER:
// Table 3 or a fitted R^d_d), or a polynomial (EV_MINIMAX: the Table 2 ones and
// the minimax fits).
constexpr int amnfe_mode(int eval) {
    return eval == EV_EXACT ? EV_EXACT
                            : ((eval == VF_EVAL_RATIONAL || eval == VF_EVAL_RATFIT) ? EV_PAPER : EV_MINIMAX);
}

// The streaming VDF kernels for 3x3 and 5x5 windows with approximated angles
// run their step loop unrolled by the window height.
constexpr bool stream_unrolled_cfg(int filter, int window, int mode) {
    return filter == VF_FILTER_VDF && window <= 5 && mode != EV_EXACT;
}

// Whether a window kernel lists, with each flagged window, the mask of its
// members that may still be the minimum. The angle filters do for 5x5 and
// larger windows, except the unrolled streaming kernels, which sit at their
// register limit, and the exact-acosf 5x5 kernels, which flag about one
// window in eighty: most waves would form masks at most steps, which costs
// more than the smaller re-check saves. 3x3 windows are re-checked whole:
// nine members fit in one pass of the wave, and the masks' LDS would cost the
// 3x3 DDF kernel a workgroup per CU. Host code gives a kernel the mask array
// exactly when this holds, so the re-check never reads masks that the kernel
// did not write.
constexpr bool writes_masks(int filter, int window, int mode, bool streaming) {
    return (filter == VF_FILTER_VDF || filter == VF_FILTER_DDF) && window >= 5 &&
           !(window == 5 && mode == EV_EXACT) && !(streaming && stream_unrolled_cfg(filter, window, mode));
}

// Everything a window kernel needs, passed by value (lives in the kernarg
// segment; coefficients are read into scalar registers).
struct KParams {
    const unsigned char* src;
    unsigned char* dst;
    int64_t src_pitch;
    int64_t dst_pitch;
    int32_t H, W;
    int32_t tiles_x;       // tiles (or column strips) per row of the image
    int32_t strip_rows;    // streaming kernels: output rows per strip
    int32_t u16;           // 1 for uint16 channels
    float lo[kMaxCoef];    // FP32 coefficients: angle lower piece / exp / ENT numerator / ln1p
    float hi[kMaxCoef];    // angle upper piece / ENT denominator
    int32_t n_lo, n_hi;
    float eta;             // absolute part of the FP32 error bound of one pair criterion (angle filters)
    float kscale;          // AMNFE: n^(kappa/3); DDF: p
    float cutoff;          // exp: T = 10 (0 above); ENT rational: T = 0.05 (0 below)
    float rho;             // angle filters: relative per-pair error bound (per-pair bound eta + rho * angle);
                           // AMNFE FP32 approximants: relative bound of every weight; packed FP16
                           // AMNFE / EVMF: absolute bound of the FP16 correction term
    uint32_t lo16[kMaxCoef];   // packed FP16 AMNFE / EVMF: lo16[k - 1] = the FP16 pair {c_k, c_k} of lo
    float wbound;          // AMNFE / AMNFG: relative FP32 error of a weight, in units of 2^-24
                           // (reciprocal, cube, EXP argument and evaluation; see approx.cpp)
    float zband;           // AMNFE / AMNFG: members whose EXP argument lies within zband of the
                           // cutoff flag the window (0: the argument stays below the cutoff)
    int32_t recheck;       // list near-tie windows for the FP64 re-check
    double param64;        // DDF p, AMNFE kappa (FP64 re-check)
    double scale64;        // AMNFE n^(-kappa/3), computed on the host
    double cutoff64;
    uint32_t* flag_list;   // flagged pixels y * W + x (each workgroup reserves its slots at once)
    uint32_t* flag_count;  // this call's counter slot
    uint32_t* next_count;  // the next call's counter slot (cleared by the re-check kernel)
    uint32_t flag_cap;
    uint32_t* flag_item;   // batch: item index of each listed pixel (null for one image)
    uint64_t* flag_mask;   // per listed pixel: members that may be the minimum (bit i = member i;
                           // all ones = re-check the whole window); null: whole windows
    int32_t item;          // batch: this image's index
};

// One image of a batch class, as the persistent kernels read it (device table).
struct BatchItem {
    const unsigned char* src;
    unsigned char* dst;
    int64_t src_pitch;
    int64_t dst_pitch;
    int32_t H, W;
    int32_t u16;
    int32_t tiles_x;
    uint32_t first_tile;   // prefix over the (sorted) items
    int32_t index;         // position in the class's item table
    uint32_t first_pixel;  // pixel prefix over the (sorted) items
};

// A batch class: images sharing filter, window and approximant, run by one
// persistent kernel (batch.h).
struct BatchParams {
    KParams base;              // class constants; flag list and counters of the class
    const BatchItem* items;    // sorted by tile count, largest first
    int32_t nitems;
    uint32_t total;            // tiles over all items
    uint32_t* counter;         // next tile to hand out (zeroed before the launch)
};

// Re-check counters: a ring of per-call slots, so no kernel has to clear the
// slot it counts into (the re-check of call k clears the slot of call k + 1).
constexpr int kCounterSlots = 64;

// Host-side description of a prepared approximant.
struct Prepared {
    int filter, window, eval, degree;
    double param;
    float lo[kMaxCoef], hi[kMaxCoef];
    int n_lo, n_hi;
    double eps;            // minimax error of the approximant (0 for exact)
    float eta;             // per-pair FP32 bound used for flagging
    float cutoff;
    double cutoff64;       // the same cutoff in FP64 (the re-check's)
    float kscale;
    int variant;           // evaluation: 0 Horner FP32, 1 Estrin FP32, 2 packed FP16 correction,
                           // 3 every window in FP64 (VF_PREC_FP64)
    float wbound, zband;   // AMNF weight error bound and cutoff band (see KParams)
    double rho;            // angle filters: relative per-pair bound (eta + rho * angle); 0 for exact;
                           // AMNFE FP32 approximants: relative bound of every weight;
                           // packed FP16 exp / ln1p: absolute bound of the FP16 correction
};

vf_status set_error(vf_status st, const char* msg);
vf_status minimax_coeffs(int func, double a, double b, int degree, int basis, double* out, double* err);
vf_status minimax_rational(int func, double a, double b, int n, int m, double* num, double* den, double* err);
vf_status prepare(int filter, int window, double param, const vf_approx* ap, Prepared* out);

// Host, per thread: non-null while run_filter asks a streaming launcher for
// the resident workgroups per CU of the kernel it would launch.
int*& occupancy_query();

// Kernel launchers (one per translation unit family); return hipError_t as int.
// The AMNFE launchers and the re-check take the kernel mode amnfe_mode(eval).
int launch_angle(int filter, int window, int eval, int n_lo, int n_hi, const KParams& p,
                 int blocks, void* stream);
int launch_angle_stream(int window, int filter, int eval, int n_lo, int n_hi, const KParams& p,
                        int blocks, void* stream);
int launch_angle_stream_var(int window, int filter, int eval, int n_lo, int n_hi, int variant,
                            const KParams& p, int blocks, void* stream);
int launch_amnfe(int filter, int window, int eval, const KParams& p, int blocks, void* stream);
int launch_amnfe_stream(int filter, int window, int eval, const KParams& p, int blocks, void* stream);
int launch_evmf_stream(int window, int eval, const KParams& p, int blocks, void* stream);
int launch_fe_stream_f16(int filter, int window, int eval, const KParams& p, int blocks, void* stream);
int launch_evmf(int window, int eval, const KParams& p, int blocks, void* stream);
int launch_recheck(int filter, int eval, int window, const KParams& p, int blocks, void* stream);
// Every window of the image in FP64 (VF_PREC_FP64), grid-stride over the pixels.
int launch_fp64(int filter, int eval, int window, const KParams& p, int blocks, void* stream);
int launch_eval_function(int filter, int eval, int n_lo, int n_hi, int variant, const KParams& p,
                         const float* in, float* out, int64_t count, void* stream);
int launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, void* stream);

// Batch launchers (persistent kernels over a class's tile table, batch.h).
// With `probe` set they launch nothing and return 0 if a kernel exists.
int launch_angle_batch_w3(int filter, int eval, int n_lo, int n_hi, bool streaming, const BatchParams& bp,
                          int num_cus, void* stream, bool probe);
int launch_angle_batch_w5(int filter, int eval, int n_lo, int n_hi, bool streaming, const BatchParams& bp,
                          int num_cus, void* stream, bool probe);
int launch_angle_batch_w7(int filter, int eval, int n_lo, int n_hi, bool streaming, const BatchParams& bp,
                          int num_cus, void* stream, bool probe);
int launch_amnfe_batch(int filter, int window, int eval, const BatchParams& bp, int num_cus, void* stream,
                       bool probe);
int launch_amnfe_stream_batch(int filter, int window, int eval, const BatchParams& bp, int num_cus, void* stream,
                              bool probe);
int launch_evmf_stream_batch(int window, int eval, const BatchParams& bp, int num_cus, void* stream, bool probe);
int launch_evmf_batch(int window, int eval, const BatchParams& bp, int num_cus, void* stream, bool probe);
int launch_recheck_batch(int filter, int eval, int window, const BatchParams& bp, int blocks, void* stream);
// Quality criteria (kern_quality.hip): one workgroup's sums, and the launch of
// the partial kernel over `blocks` workgroups (<= kQualMaxBlocks) and the
// final fold; parts holds blocks + 1 partials, the last one the result.
struct QualPartial {
    unsigned long long l1, l2sq;   // sums of |x - y| and (x - y)^2 over pixels and channels
    double lab_diff, lab_ref;      // sums of |x^Lab - y^Lab|_2 and |x^Lab|_2
};
constexpr int kQualMaxBlocks = 4096;
int launch_quality(const unsigned char* x, int64_t x_pitch, const unsigned char* y, int64_t y_pitch, int H, int W,
                   bool u16, int blocks, void* parts, void* stream);

// The class's FP64 pass over all of its `pixels` windows, which does work only
// when the class flagged more windows than its re-check list holds.
int launch_overflow_batch(int filter, int eval, int window, const BatchParams& bp, uint32_t pixels, int blocks,
                          void* stream);

}  // namespace vf
