/*
 * vf.h -- C ABI of the MI355X (gfx950) sliding-window vector order-statistics
 * filters of Celebi, Kingravi, Lukac and Celiker, "Cost-Effective Implementation
 * of Order-Statistics Based Vector Filters Using Minimax Approximations".
 *
 * Every call takes plain pointers and sizes. Image buffers are DEVICE pointers
 * owned by the caller (the library never frees or retains them); the library
 * owns only its context workspace. Filter calls are asynchronous and ordered
 * on the HIP stream passed in (NULL = the default stream); argument validation
 * finishes before any device work, so a call that returns an error has written
 * nothing. Launch failures return VF_EHIP; faults during execution surface at
 * the caller's next synchronisation. One context may be used from one host
 * thread at a time, and calls on one context must be ordered (same stream or
 * externally synchronised) because they share the context's workspace.
 */
#ifndef VF_H
#define VF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VF_OK = 0,
    VF_EINVAL = -1,        /* bad argument (null pointer, bad size, overlap, ...) */
    VF_EDOMAIN = -2,       /* interval outside the function's domain */
    VF_ENOCONV = -3,       /* Remez exchange did not converge */
    VF_EHIP = -4,          /* HIP runtime error */
    VF_ENOMEM = -5,        /* workspace allocation failed */
    VF_EUNSUPPORTED = -6   /* valid but unsupported combination (e.g. window 9) */
} vf_status;

typedef enum { VF_U8 = 1, VF_U16 = 2 } vf_dtype;

typedef enum {
    VF_FILTER_VDF = 0,     /* basic vector directional filter (Section 3.1, BVDF equation) */
    VF_FILTER_DDF = 1,     /* directional-distance filter (named in Section 3.1) */
    VF_FILTER_AMNFE = 2,   /* adaptive multichannel non-parametric filter, exp kernel (Section 3.2) */
    VF_FILTER_EVMF = 3,    /* entropy vector median filter (Section 3.3) */
    VF_FILTER_AMNFG = 4    /* adaptive multichannel non-parametric filter, Gaussian kernel (Section 3.2) */
} vf_filter;

/* Kernel function K of the AMNF equation (vf_filter_fuzzy_exp). */
typedef enum {
    VF_KERNEL_EXP = 0,     /* K(x) = exp(-|x|_1): AMNFE */
    VF_KERNEL_GAUSS = 1    /* K(x) = exp(-0.5 |x|_2^2): AMNFG */
} vf_kernel;

/* Elementary functions known to vf_minimax_coeffs. */
typedef enum {
    VF_F_ACOS = 1,         /* acos(z), domain [-1, 1] (Table 1, ARCCOS row on [0, 0.5]) */
    VF_F_ASIN = 2,         /* asin(z), domain [-1, 1] */
    VF_F_ASIN2_TAU = 3,    /* 2 asin(tau / sqrt 2), domain [-sqrt 2, sqrt 2] (Table 1, ARCSIN row) */
    VF_F_CHORD = 4,        /* 2 asin(s / 2): angle subtended by a unit-sphere chord s, domain [-2, 2] */
    VF_F_EXPNEG = 5,       /* exp(-z) (Table 2) */
    VF_F_LN1P = 6,         /* ln(1 + t), domain t > -1 */
    VF_F_XLNX = 7          /* z ln z, domain z >= 0 (the ENT function of Section 3.3) */
} vf_func;

typedef enum {
    VF_BASIS_FULL = 0,     /* a_0 + a_1 z + ... + a_d z^d (the P_n of Section 2) */
    VF_BASIS_ODD = 1       /* a_1 z + a_3 z^3 + ... + a_d z^d, symmetric interval, d odd */
} vf_basis;

/* How a filter evaluates its elementary function. */
typedef enum {
    VF_EVAL_EXACT = 0,     /* HIP device math in FP32: acosf / expf / logf */
    VF_EVAL_PAPER = 1,     /* the paper's printed approximants: Table 1 two-piece arccos
                              (degree 4), Table 2 exp polynomial (degree 2, 3 or 4, on
                              [0, 10] with the T = 10 cutoff), Table 4 ENT rational with
                              the T = 0.05 cutoff */
    VF_EVAL_SPLIT = 2,     /* angle: odd minimax split covering z in [-1, 1]; degree odd, 3..9:
                              |z| < 1/2 -> pi/2 - asin fit; z >= 1/2 -> chord fit of
                              s = sqrt(2(1 - z)) */
    VF_EVAL_CHORD = 3,     /* angle: one odd minimax polynomial in the chord s over z in
                              [0, 1] (the range of non-negative RGB); degree 7, 9, 11 or 13 */
    VF_EVAL_MINIMAX = 4,   /* exp: minimax of exp(-z) on [0, min(b, T)], degree 2..9, with
                              b = n^(kappa/3) (AMNFE) or 0.5 n^(2 kappa/3) (AMNFG) the
                              largest argument the kernel reaches and T = 10 the cutoff;
                              ENT: z (e ln 2 + q(m - 1)) with z = m 2^e and q the minimax
                              of ln(1 + t) on [0, 1], degree 2..9. A degree whose minimax
                              error is below 2^-24 of the function's largest value is
                              refused (VF_EUNSUPPORTED; no gain in FP32): at kappa = 0.33
                              exp accepts up to degree 6 (AMNFE) or 5 (AMNFG), ENT up to 7 */
    VF_EVAL_RATIONAL = 5,  /* exp (AMNFE, AMNFG): the paper's Table 3 rational R^4_4 of
                              exp(-z) on [0, 10] with the T = 10 cutoff, evaluated in FP32
                              (numerator and denominator by Horner, one divide); degree
                              4 or 0. EVMF's rational (Table 4) is VF_EVAL_PAPER */
    VF_EVAL_RATFIT = 6     /* exp (AMNFE, AMNFG): the best rational R^d_d of exp(-z) on
                              [0, min(b, T)] (b as for VF_EVAL_MINIMAX) from this library's
                              rational Remez exchange (vf_minimax_rational), evaluated like
                              VF_EVAL_RATIONAL; degree d 1..4, refused below FP32
                              resolution as for VF_EVAL_MINIMAX (kappa = 0.33: d <= 2) */
} vf_eval;

/* Arithmetic of the elementary-function evaluation (sums always accumulate in
 * FP32). VF_PREC_FP16X2 (streaming kernels only): for VF_EVAL_CHORD angle
 * filters, angle = s (c_0 + t) with the correction t = s^2 q(s^2) evaluated
 * for two pairs at once with packed FP16 multiply-adds and c_1.. rounded to
 * FP16, c_0 s in FP32; for VF_EVAL_MINIMAX AMNFE, AMNFG and EVMF, p(x) = c_0 + t(x)
 * with t(x) = sum_{k>=1} c_k x^k evaluated the same way for two window
 * members at once (exp: x = z; ENT: x = the reduced mantissa), c_1.. rounded
 * to FP16. Its larger error bound flags more windows for the FP64 re-check
 * (see vf_get_stats), which evaluates the same rounded polynomial in FP64. */
/* VF_PREC_FP64: every window evaluated in FP64 on the GPU from its
 * definition (the BVDF, DDF, AMNF and EVF equations of Section 3), with the
 * elementary function of approx->eval (exact: the FP64 acos / exp / log;
 * approximants: the same FP32 constants widened exactly to FP64), summed in
 * member order with one rounding per operation, as the FP64 re-check does for
 * near-tie windows. One wavefront per window: the correctness anchor, not a
 * fast path. No re-check list is used (VF_NO_RECHECK / VF_DEFER_RECHECK /
 * VF_DIRECT have no effect); Horner's scheme only; not accepted by
 * vf_filter_batch, vf_eval_function or vf_autotune. */
typedef enum { VF_PREC_FP32 = 0, VF_PREC_FP16X2 = 1, VF_PREC_FP64 = 2 } vf_precision;
/* Polynomial evaluation order (VF_SCHEME_ESTRIN: VF_EVAL_CHORD angle filters,
 * streaming kernels, FP32 only). Results differ from Horner only by rounding. */
typedef enum { VF_SCHEME_HORNER = 0, VF_SCHEME_ESTRIN = 1 } vf_scheme;

/* flags */
#define VF_NO_RECHECK 0x1u   /* skip the FP64 re-check of near-tie / near-rounding windows */
#define VF_DIRECT 0x2u       /* score every window's pairs separately (per-window kernel)
                                instead of streaming each pixel pair once (same results) */
#define VF_DEFER_RECHECK 0x4u /* list the near-tie windows but do not re-check them yet:
                                 vf_recheck_pending() runs that call's re-check later */
#define VF_TUNED 0x8u        /* use the context's autotuned configuration for this filter,
                                window, dtype and eval (vf_autotune): its degree, scheme,
                                precision, kernel and tile height replace the request's;
                                without an entry the request is used as given */

typedef struct {
    int32_t eval;        /* vf_eval */
    int32_t degree;      /* polynomial degree where the mode takes one */
    int32_t precision;   /* vf_precision */
    int32_t scheme;      /* vf_scheme */
    uint32_t flags;      /* VF_NO_RECHECK | VF_DIRECT | VF_DEFER_RECHECK */
} vf_approx;

/* An interleaved RGB image (H x W pixels, 3 channels of uint8 or uint16,
 * channel order as stored). src and dst are device pointers; pitches are bytes
 * between row starts and must be at least 3 * width * element size. src and
 * dst must not overlap. */
typedef struct {
    const void* src;
    void* dst;
    int32_t height;
    int32_t width;
    int64_t src_pitch;
    int64_t dst_pitch;
    int32_t dtype;       /* vf_dtype */
} vf_image;

typedef struct vf_context vf_context;

/*
 * Create a context on a HIP device. Its workspace is allocated lazily and
 * grown as needed: for calls with the re-check, 12 bytes per pixel of the
 * largest image so far (the re-check list: pixel index and candidate mask).
 * The streaming kernels' strip height (output rows per wave) is sized per
 * call from the kernel's residency on the device; the environment variable
 * VF_STRIP_ROWS (1 .. 4096), read here, fixes it for the context instead.
 */
vf_status vf_create(int32_t device, vf_context** out);
/* Destroy a context; waits for its outstanding work. NULL is accepted. */
vf_status vf_destroy(vf_context* ctx);

/*
 * Vector directional filter (Section 3.1, BVDF equation):
 *   y(r,c) = argmin_{x_i in W(r,c)} sum_j A(x_i, x_j),
 *   A(x_i, x_j) = arccos(x_i . x_j / (|x_i|_2 |x_j|_2)).
 * window: 3, 5 or 7 (the sqrt(n) of Section 3). Borders replicate the edge
 * pixel. Ties: the centre wins if it is among the minimisers, else the lowest
 * row-major window index. Identical or collinear vectors have angle 0; a zero
 * vector against a non-zero one has angle pi/2.
 * approx->eval: VF_EVAL_EXACT, VF_EVAL_PAPER, VF_EVAL_SPLIT or VF_EVAL_CHORD.
 * Unless VF_NO_RECHECK is set, windows whose two best sums (over distinct
 * vectors) are closer than the FP32 error bound are recomputed in FP64 with
 * the same approximant.
 */
vf_status vf_filter_vdf(vf_context* ctx, const vf_image* img, int32_t window,
                        const vf_approx* approx, void* hip_stream);

/*
 * vf_filter_vdf without any device allocation and without a context, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. The results equal
 * vf_filter_vdf's. The re-check workspace (two counters, a list of up to
 * 2^20 flagged pixels and their candidate masks: 12 MiB) is a file-scope
 * device array of the library that every GPU it runs on holds from the time
 * the library's code is loaded there until the process ends; device is the
 * HIP device the image lives on, made current for the call. Limits: at most
 * 2^20 = 1048576 pixels per image (VF_EINVAL beyond, nothing launched);
 * VF_DEFER_RECHECK and VF_TUNED are refused (VF_EINVAL: they keep state in a
 * context); the streaming strip height is sized per call. Every call on one
 * GPU shares that GPU's scratch, which keeps the last call's contents (each
 * call clears its counters first, with a fill kernel): calls that overlap on
 * one GPU (different streams without ordering) race and must not be issued.
 * Host-side approximant preparation may still allocate host memory (the
 * Remez cache). Other errors as vf_filter_vdf.
 */
vf_status vf_filter_vdf_noalloc(int32_t device, const vf_image* img, int32_t window,
                                const vf_approx* approx, void* hip_stream);

/*
 * Directional-distance filter (cited in Section 3.1): argmin of
 *   (sum_j |x_i - x_j|_2)^(1 - p) * (sum_j A(x_i, x_j))^p,  0 <= p <= 1
 * (p = 0.5 is the usual choice). Other conventions as vf_filter_vdf.
 */
vf_status vf_filter_ddf(vf_context* ctx, const vf_image* img, int32_t window, double p,
                        const vf_approx* approx, void* hip_stream);

/*
 * Adaptive multichannel non-parametric filters (Section 3.2, AMNF equation):
 *   y = sum_i x_i w_i / sum_j w_j,  w_i = h_i^-3 K((x_C - x_i) / h_i),
 *   h_i = n^(-kappa/3) sum_j |x_i - x_j|_1,
 * kernel VF_KERNEL_EXP (AMNFE): K(x) = exp(-|x|_1);
 * kernel VF_KERNEL_GAUSS (AMNFG): K(x) = exp(-0.5 |x|_2^2).
 * The EXP argument is 0 (K = 0) above the cutoff T = 10 of Section 3.2.
 * kappa > 0 (0.33 in the paper). The mean is rounded per channel with
 * floor(v + 0.5); a uniform window returns its centre. approx->eval:
 * VF_EVAL_EXACT, VF_EVAL_PAPER (Table 2, degree 2..4), VF_EVAL_MINIMAX
 * (degree 2..9) or VF_EVAL_RATIONAL (Table 3). Windows whose rounded mean
 * lies within the FP32 error bound of a rounding boundary, or with an EXP
 * argument within its FP32 error of T, are recomputed in FP64 (unless
 * VF_NO_RECHECK). VF_EINVAL for another kernel value.
 */
vf_status vf_filter_fuzzy_exp(vf_context* ctx, const vf_image* img, int32_t window,
                              double kappa, int32_t kernel, const vf_approx* approx,
                              void* hip_stream);

/*
 * Entropy vector median filter (Section 3.3, EVF equation): the vector
 * median argmin_i sum_j |x_i - x_j|_2 when P_C > beta_C, else the centre.
 * The test is evaluated as P_C * H > -ENT(P_C), H = -sum_j ENT(P_j),
 * ENT(z) = z ln z. The cutoff T of Section 3.3 applies in every mode:
 * ENT(z) = 0 for z < T (T = 0: no cutoff). approx->eval: VF_EVAL_EXACT,
 * VF_EVAL_PAPER (Table 4 rational, which holds on [0.05, 1]: T >= 0.05, the
 * paper's T = 0.05) or VF_EVAL_MINIMAX (range-reduced ln, degree 2..9). A
 * P_j within the FP32 error band of T is decided in FP64. Errors: VF_EINVAL
 * (T outside [0, 1], and as vf_filter_vdf), VF_EDOMAIN (VF_EVAL_PAPER with
 * T < 0.05).
 */
vf_status vf_filter_log(vf_context* ctx, const vf_image* img, int32_t window, double cutoff,
                        const vf_approx* approx, void* hip_stream);

/*
 * Run the FP64 re-check of the context's last filter call made with
 * VF_DEFER_RECHECK, on hip_stream (which must be ordered after that call).
 * While a re-check is pending, every other filter or batch call on the
 * context returns VF_EINVAL and does nothing (it would share the pending
 * call's re-check list). VF_OK and no work if nothing is pending.
 */
vf_status vf_recheck_pending(vf_context* ctx, void* hip_stream);

/* One image of a batch. filter: vf_filter; param: p (DDF), kappa (AMNFE, AMNFG)
 * or the ENT cutoff T (EVMF). */
typedef struct {
    vf_image img;
    int32_t filter;
    int32_t window;
    double param;
    vf_approx approx;
} vf_batch_item;

/*
 * Filter many images of uneven size, each with its own filter, window and
 * approximant, as one stream-ordered submission: images are grouped into
 * classes (filter, window, parameter, approximant, flags, tile height); each
 * class is one persistent kernel whose workgroups pull tiles from a table
 * sorted largest image first, followed by its FP64 re-check; the classes run
 * as up to four concurrent chains (VF_BATCH_STREAMS = 1 .. 4 in the
 * environment sets the number), so that one class's tail overlaps the next
 * one's start; the whole submission is captured once as a HIP graph and
 * relaunched while the item list stays the same. Results equal those of the
 * individual filter calls. Items with VF_TUNED take the tuned degree and
 * kernel (Horner, FP32; the class sizes its strips over all its images).
 * Re-check lists are capped per class at an eighth of its windows (half for
 * exact evaluation), at least 65536 and at most all of them
 * (VF_BATCH_FLAG_CAP in the environment replaces the cap); a class that
 * flags more windows than its cap evaluates every one of its windows in FP64
 * instead, with the same results, more slowly. Errors: as the filter calls;
 * VF_EINVAL also when a destination overlaps any source or another
 * destination, or an item sets VF_DEFER_RECHECK; VF_EUNSUPPORTED for the
 * Estrin or FP16 variants. Device memory: 16 bytes per re-check slot plus the
 * tables (at most 2 bytes per pixel of an approximant class, 8 per pixel of
 * an exact class), kept by the context until a different list is submitted.
 */
vf_status vf_filter_batch(vf_context* ctx, const vf_batch_item* items, int32_t count,
                          void* hip_stream);

/*
 * Minimax polynomial of f on [a, b] by the Remez exchange algorithm
 * (Section 2; eps = max |f - P| over [a, b]). Host only, thread-safe, needs
 * no GPU. basis VF_BASIS_FULL: coeffs_out[0..degree] are a_0..a_degree of
 * the monomial form in z. VF_BASIS_ODD (a == -b, degree odd):
 * coeffs_out[0..(degree-1)/2] are a_1, a_3, ..., a_degree. *err_out receives
 * the levelled error |E|; on return max|f - P| on [a, b] is within 1e-12 of it.
 * Errors: VF_EINVAL (a >= b, degree out of [0, 16], odd basis with even degree
 * or asymmetric interval, null pointers), VF_EDOMAIN ([a, b] leaves f's
 * domain), VF_ENOCONV (no convergence within the iteration cap).
 */
vf_status vf_minimax_coeffs(int32_t func, double a, double b, int32_t degree, int32_t basis,
                            double* coeffs_out, double* err_out);

/*
 * Best rational approximation p / q of f on [a, b] from the class R^n_m
 * (Section 2: p in P_n, q in P_m, minimising max |f - p / q|; Tables 3 and 4
 * are R^4_4 of exp(-z) on [0, 10] and z ln z on [0.05, 1]) by the rational
 * Remez exchange. Host only, thread-safe, needs no GPU. num_out[0..n] and
 * den_out[0..m] are the monomial coefficients in z, scaled so that
 * den_out[0] = 1; *err_out receives the levelled error |E| (max |f - p/q| on
 * [a, b] is within 1e-12, and within 1e-10 relative, of it). Errors:
 * VF_EINVAL (a >= b, n or m out of [0, 8], null pointers), VF_EDOMAIN,
 * VF_ENOCONV (no convergence, or a denominator with a zero on [a, b]).
 */
vf_status vf_minimax_rational(int32_t func, double a, double b, int32_t n, int32_t m,
                              double* num_out, double* den_out, double* err_out);

/*
 * The FP32 constants a filter call with these arguments evaluates, and the
 * approximant's minimax error. lo/hi receive up to 16 values each (the two
 * pieces of an angle approximant; exp and ENT polynomials use lo only, the
 * rationals (Table 3 exp, fitted R^d_d exp, Table 4 ENT) use lo = numerator,
 * hi = denominator).
 * Host only.
 */
vf_status vf_get_approximant(int32_t filter, int32_t window, double param,
                             const vf_approx* approx, float* lo, int32_t* n_lo,
                             float* hi, int32_t* n_hi, double* eps_out);

/*
 * Evaluate a filter's elementary function on a device array exactly as the
 * filter kernels do (FP32, or the packed-FP16 correction where the approximant
 * asks for it for AMNFE / EVMF), for error measurements:
 *   VDF/DDF: in[i] = squared chord s^2 = 2(1 - z) of two unit vectors, out = angle;
 *   AMNFE, AMNFG: in[i] = z >= 0, out = K = exp(-z) approximant (0 above the cutoff);
 *   EVMF:    in[i] = P in [0, 1], out = ENT(P).
 */
vf_status vf_eval_function(vf_context* ctx, int32_t filter, int32_t window, double param,
                           const vf_approx* approx, const float* in, float* out,
                           int64_t count, void* hip_stream);

typedef struct {
    uint64_t windows;      /* windows filtered by the last call */
    uint64_t flagged;      /* windows flagged for the FP64 re-check by the last call */
    int32_t tile_w;        /* output tile (or column strip) of the last call's main kernel */
    int32_t tile_h;        /* its height (rows per strip for the streaming kernels) */
    int32_t workgroups;    /* workgroups the last call's main kernel launched */
    int32_t streaming;     /* 1 if the last call used a streaming (pair-sharing) kernel */
} vf_stats;

/* Result of vf_autotune: the fastest configuration found. */
typedef struct {
    int32_t direct;        /* 1: per-window kernel; 0: streaming kernel */
    int32_t strip_rows;    /* streaming: output rows per strip (tile height); 0: sized per call
                              from the kernel's occupancy, or the per-window kernel */
    int32_t degree;        /* polynomial degree (0 for exact evaluation) */
    int32_t scheme;        /* vf_scheme */
    int32_t precision;     /* vf_precision */
    int32_t candidates;    /* configurations timed */
    double ms;             /* median time of one filter call on the sample, re-check included */
    double func_err;       /* max |f - P| of the chosen approximant (0 for exact) */
} vf_tune_result;

/*
 * Autotune one filter family (the batch's "autotuned tile shape and degree"):
 * times, on `sample` (src and dst device images; dst is overwritten) and on
 * hip_stream, every configuration of the filter with approx->eval whose
 * approximant error |f - P| is at most max_func_err (<= 0: no limit):
 * every degree the evaluation accepts (or approx->degree if > 0), Horner and
 * Estrin schemes and FP32 / packed FP16 where implemented, and the streaming
 * kernel with 16, 32, 64, 128 and 256-row strips or strips sized from its
 * occupancy (the default of untuned calls), or the per-window kernel.
 * Each timing is a whole filter call including its FP64 re-check (median of
 * 5 after one warm-up). The fastest is stored in the context under (filter,
 * window, sample dtype, approx->eval), used by calls with VF_TUNED, and
 * returned in *out. Synchronises hip_stream. Errors: VF_EINVAL (null or
 * invalid arguments), VF_EUNSUPPORTED (no configuration meets the target),
 * VF_EHIP.
 */
vf_status vf_autotune(vf_context* ctx, int32_t filter, int32_t window, double param,
                      const vf_approx* approx, const vf_image* sample, double max_func_err,
                      vf_tune_result* out, void* hip_stream);
/* Write the context's tuned configurations to a text file (one line each). */
vf_status vf_tune_save(vf_context* ctx, const char* path);
/* Read configurations written by vf_tune_save into the context (replacing
 * entries of the same key). VF_EINVAL for an unreadable, malformed or
 * out-of-range file; then the context is unchanged. */
vf_status vf_tune_load(vf_context* ctx, const char* path);
/* Forget every tuned configuration of the context. */
vf_status vf_tune_clear(vf_context* ctx);

/* Quality criteria of a filtered image against its original (Section 4). */
typedef struct {
    uint64_t pixels;
    uint64_t l1_sum;        /* sum over pixels and channels of |x - y| (exact) */
    uint64_t l2sq_sum;      /* sum over pixels and channels of (x - y)^2 (exact) */
    double lab_diff_sum;    /* sum over pixels of |x^Lab - y^Lab|_2 */
    double lab_ref_sum;     /* sum over pixels of |x^Lab|_2 */
    double mae;             /* l1_sum / (3 pixels), in the image's units */
    double mse;             /* l2sq_sum / (3 pixels) */
    double ncd;             /* lab_diff_sum / lab_ref_sum (0 when both are 0, +inf when only the first is) */
} vf_quality_result;

/*
 * The quality criteria of Section 4: MAE, MSE and the normalized colour
 * difference NCD in CIE L*a*b* of the filtered image img->dst (Y) against the
 * original img->src (X); both are only read and may be the same buffer.
 * CIELAB reading: values are sRGB scaled to [0, 1] by the type's maximum,
 * decoded with the sRGB transfer function, taken to XYZ by the sRGB
 * primaries' matrix (four-digit form), relative to the white that matrix
 * gives the RGB white (white is L* = 100, a* = b* = 0). The L1 and squared
 * sums are exact integers; the two FP64 CIELAB sums are folded in a fixed
 * order (the same image on the same device gives the same bits). Runs on
 * hip_stream and waits for it. Errors: VF_EINVAL (null pointers, bad dtype,
 * size or pitch, a deferred re-check pending), VF_EUNSUPPORTED (2^32 8-bit
 * or 2^30 16-bit pixels or more), VF_ENOMEM, VF_EHIP.
 */
vf_status vf_quality(vf_context* ctx, const vf_image* img, vf_quality_result* out, void* hip_stream);

/* Statistics of the context's last filter call (waits for that call). */
vf_status vf_get_stats(vf_context* ctx, vf_stats* out);

const char* vf_status_string(int32_t status);
/* Detail of the calling thread's last error ("" if none). A call that fails
 * with VF_EHIP after its window kernel was issued leaves its outputs
 * unspecified; the context stays usable (the next call re-zeroes the
 * re-check counters first). For tests of that path, the environment
 * variable VF_INJECT_HIP_ERROR=window|recheck|batch makes the named launch
 * report hipErrorLaunchFailure without launching. */
const char* vf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VF_H */
