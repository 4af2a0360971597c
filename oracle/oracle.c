/*
 * oracle.c -- plain FP64 CPU reference of the sliding-window vector filters.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. It shares no code, header or
 * constant with the GPU library; every convention below is restated from the
 * paper (and, where the paper is silent, from the documented readings).
 *
 * Image model (paper, Section 3 opening paragraph): an M x N RGB image of
 * 3-component vectors, a sqrt(n) x sqrt(n) window W(r,c) centred on each pixel,
 * sliding in raster order, output M x N. The window's members are re-indexed
 * x_1..x_n with the centre x_C = x_{(n+1)/2}.
 *   Readings: pixels outside the image replicate the nearest edge pixel;
 *   members are numbered row-major inside the window (0-based index
 *   i = (dy + r) * w + (dx + r), centre (n - 1) / 2).
 *
 * Filters:
 *   VDF   (Section 3.1, BVDF equation): y = argmin_i sum_j A(x_i, x_j),
 *         A = arccos(x_i . x_j / (|x_i|_2 |x_j|_2)).
 *   DDF   (cited in Section 3.1; reading): argmin_i (sum_j |x_i - x_j|_2)^(1-p)
 *         * (sum_j A(x_i, x_j))^p.
 *   AMNFE (Section 3.2, AMNF equation with the exponential kernel):
 *         y = sum_i x_i w_i / sum_j w_j,  w_i = h_i^-3 K((x_C - x_i)/h_i),
 *         h_i = n^(-kappa/3) sum_j |x_i - x_j|_1,  K(x) = exp(-|x|_1).
 *   AMNFG (Section 3.2, the same equation with the Gaussian kernel):
 *         K(x) = exp(-0.5 |x|_2^2), the same h_i.
 *   EVMF  (Section 3.3, EVF equation): if P_C > beta_C output the vector
 *         median argmin_i sum_j |x_i - x_j|_2, else x(r,c); P_i and beta_i as
 *         in that equation with the mean vector x_bar.
 *
 * Conventions (readings of what the paper leaves open):
 *   - argmin ties: the centre wins if it is among the minimisers, otherwise the
 *     lowest window index.
 *   - cosine of two vectors: identical or collinear vectors (integer cross
 *     product zero, both non-zero, or both zero) have z = 1; one zero vector
 *     against a non-zero one has z = 0; otherwise z = dot / (|x_i| |x_j|),
 *     clamped to [-1, 1].
 *   - AMNFE: a window with some h_i = 0 (uniform window) outputs x_C; the
 *     weighted mean is rounded per channel with floor(v + 0.5).
 *   - EVMF: a window with sum_j |x_j - x_bar| = 0 outputs x_C; the switching
 *     test P_C > beta_C is evaluated multiplied through by the (non-negative)
 *     denominator of beta_C:  P_C * H > -ENT(P_C),  H = -sum_j ENT(P_j).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math), so that
 * every product and sum is a separately rounded IEEE double operation.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXN 49
#define ORC_MAXC 16

/* ---- elementary-function evaluators ------------------------------------ */

/* Angle evaluator kinds. */
enum { ORC_ACOS_EXACT = 0,   /* acos(z) */
       ORC_ACOS_PAPER2 = 1,  /* Table 1 form: z < 0.5 -> P_lo(z) (full basis);
                                z >= 0.5 -> P_hi(tau), tau = sqrt(1 - z) */
       ORC_ACOS_SPLIT = 2,   /* odd split over [-1, 1]:
                                |z| < 0.5  -> pi/2 - z * L(z^2)          (L: odd asin fit)
                                z >= 0.5   -> s * U(s^2), s = sqrt(2(1 - z))   (U: odd chord fit)
                                z <= -0.5  -> pi - s * U(s^2), s = sqrt(2(1 + z)) */
       ORC_ACOS_CHORD = 3 }; /* one odd chord fit U over z in [0, 1]:
                                z >= 0 -> s * U(s^2), s = sqrt(2(1 - z));
                                z < 0  -> pi - s * U(s^2), s = sqrt(2(1 + z)) */

typedef struct {
    int kind;
    int n_lo, n_hi;
    double lo[ORC_MAXC];
    double hi[ORC_MAXC];
} orc_acos_t;

/* exp(-z) evaluator kinds. */
enum { ORC_EXP_EXACT = 0,
       ORC_EXP_POLY = 1,      /* c(z) */
       ORC_EXP_RATIONAL = 2 };/* c(z) / q(z) (Table 3 form) */
typedef struct {
    int kind;
    int n;
    double c[ORC_MAXC];
    double cutoff;   /* arguments above the cutoff give 0 (Section 3.2) */
    int n_q;
    double q[ORC_MAXC];
} orc_exp_t;

/* z ln z evaluator kinds. */
enum { ORC_ENT_EXACT = 0,     /* z log z, 0 at z = 0 */
       ORC_ENT_RATIONAL = 1,  /* p(z) / q(z) (Table 4 form) */
       ORC_ENT_RANGERED = 2 };/* z = m 2^e, m in [1,2): z * (e ln2 + Q(m - 1)) */
typedef struct {
    int kind;
    int n_p, n_q;
    double p[ORC_MAXC];
    double q[ORC_MAXC];
    double cutoff;   /* T: arguments below it give 0 in every kind (Section 3.3) */
} orc_ent_t;

static double horner(const double* c, int n, double z) {
    double acc = c[n - 1];
    for (int k = n - 2; k >= 0; --k) acc = acc * z + c[k];
    return acc;
}

static double eval_angle(const orc_acos_t* ap, double z) {
    switch (ap->kind) {
    case ORC_ACOS_EXACT:
        return acos(z);
    case ORC_ACOS_PAPER2:
        if (z < 0.5) return horner(ap->lo, ap->n_lo, z);
        return horner(ap->hi, ap->n_hi, sqrt(1.0 - z));
    case ORC_ACOS_SPLIT:
        if (z >= 0.5) {
            double s = sqrt(2.0 * (1.0 - z));
            return s * horner(ap->hi, ap->n_hi, s * s);
        }
        if (z <= -0.5) {
            double s = sqrt(2.0 * (1.0 + z));
            return M_PI - s * horner(ap->hi, ap->n_hi, s * s);
        }
        return M_PI / 2.0 - z * horner(ap->lo, ap->n_lo, z * z);
    case ORC_ACOS_CHORD:
        if (z >= 0.0) {
            double s = sqrt(2.0 * (1.0 - z));
            return s * horner(ap->hi, ap->n_hi, s * s);
        } else {
            double s = sqrt(2.0 * (1.0 + z));
            return M_PI - s * horner(ap->hi, ap->n_hi, s * s);
        }
    }
    return NAN;
}

static double eval_expneg(const orc_exp_t* ep, double z) {
    if (z > ep->cutoff) return 0.0;
    if (ep->kind == ORC_EXP_EXACT) return exp(-z);
    if (ep->kind == ORC_EXP_RATIONAL) return horner(ep->c, ep->n, z) / horner(ep->q, ep->n_q, z);
    return horner(ep->c, ep->n, z);
}

/* ENT(z) = z ln z (Section 3.3), 0 at 0 and below the cutoff T in every kind */
static double eval_ent(const orc_ent_t* en, double z) {
    if (z <= 0.0 || z < en->cutoff) return 0.0;
    switch (en->kind) {
    case ORC_ENT_EXACT:
        return z * log(z);
    case ORC_ENT_RATIONAL:
        return horner(en->p, en->n_p, z) / horner(en->q, en->n_q, z);
    case ORC_ENT_RANGERED: {
        int e;
        double m = frexp(z, &e);     /* z = m 2^e, m in [0.5, 1) */
        m *= 2.0;
        e -= 1;                      /* m in [1, 2) */
        return z * ((double)e * M_LN2 + horner(en->p, en->n_p, m - 1.0));
    }
    }
    return NAN;
}

/* ---- window gathering ---------------------------------------------------- */

typedef struct {
    const void* src;
    int height, width;
    int bytes_per_channel;   /* 1 (uint8) or 2 (uint16) */
    int64_t pitch;           /* row pitch in channels (elements) */
} orc_img_t;

static void pixel_at(const orc_img_t* im, int y, int x, int64_t out[3]) {
    if (y < 0) y = 0;
    if (y >= im->height) y = im->height - 1;
    if (x < 0) x = 0;
    if (x >= im->width) x = im->width - 1;
    int64_t off = (int64_t)y * im->pitch + (int64_t)x * 3;
    for (int k = 0; k < 3; ++k) {
        if (im->bytes_per_channel == 1) out[k] = ((const uint8_t*)im->src)[off + k];
        else out[k] = ((const uint16_t*)im->src)[off + k];
    }
}

static int gather(const orc_img_t* im, int y, int x, int w, int64_t v[][3]) {
    int r = (w - 1) / 2;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx)
            pixel_at(im, y + dy, x + dx, v[(dy + r) * w + (dx + r)]);
    return w * w;
}

/* ---- per-pair criteria --------------------------------------------------- */

/* Cosine of the angle between two non-negative integer vectors, with the
 * documented conventions for identical, collinear and zero vectors. */
static double cosine(const int64_t* a, const int64_t* b) {
    int64_t na = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    int64_t nb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    if (na == 0 && nb == 0) return 1.0;
    if (na == 0 || nb == 0) return 0.0;
    int64_t c0 = a[1] * b[2] - a[2] * b[1];
    int64_t c1 = a[2] * b[0] - a[0] * b[2];
    int64_t c2 = a[0] * b[1] - a[1] * b[0];
    if (c0 == 0 && c1 == 0 && c2 == 0) return 1.0;  /* collinear (same direction: components >= 0) */
    double dot = (double)(a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
    double z = dot / (sqrt((double)na) * sqrt((double)nb));
    if (z > 1.0) z = 1.0;
    if (z < -1.0) z = -1.0;
    return z;
}

static double dist_l2(const int64_t* a, const int64_t* b) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        double d = (double)(a[k] - b[k]);
        s += d * d;
    }
    return sqrt(s);
}

static int64_t dist_l1(const int64_t* a, const int64_t* b) {
    int64_t s = 0;
    for (int k = 0; k < 3; ++k) s += llabs(a[k] - b[k]);
    return s;
}

/* argmin with the tie rule: the centre stays unless strictly beaten; among
 * the others the lowest index wins (strict < while scanning in order). */
static int argmin_tie(const double* s, int n) {
    int best = (n - 1) / 2;
    for (int i = 0; i < n; ++i)
        if (s[i] < s[best]) best = i;
    return best;
}

/* ---- window-level filters (exported for per-pixel inspection) ------------- */

/* VDF: fills S[i] = sum_j A(x_i, x_j) over all ordered j (j = i included) and
 * returns the selected index. */
int orc_window_vdf(const int64_t v[][3], int n, const orc_acos_t* ap, double* S) {
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += eval_angle(ap, cosine(v[i], v[j]));
        S[i] = acc;
    }
    return argmin_tie(S, n);
}

/* DDF: SA[i] angle sums, SD[i] Euclidean sums, Psi[i] = SD^(1-p) SA^p. */
int orc_window_ddf(const int64_t v[][3], int n, double p, const orc_acos_t* ap,
                   double* SA, double* SD, double* Psi) {
    for (int i = 0; i < n; ++i) {
        double a = 0.0, d = 0.0;
        for (int j = 0; j < n; ++j) {
            a += eval_angle(ap, cosine(v[i], v[j]));
            d += dist_l2(v[i], v[j]);
        }
        SA[i] = a;
        SD[i] = d;
        Psi[i] = pow(d, 1.0 - p) * pow(a, p);
    }
    return argmin_tie(Psi, n);
}

/* AMNF (exponential kernel, gauss = 0: AMNFE; Gaussian kernel, gauss = 1:
 * AMNFG): writes the unrounded weighted mean to mean[3]; returns 1 when the
 * window is uniform (output x_C), else 0. The EXP argument of member i is
 * |x|_1 (AMNFE) or 0.5 |x|_2^2 (AMNFG) of x = (x_C - x_i) / h_i. */
static int window_amnf(const int64_t v[][3], int n, double kappa, const orc_exp_t* ep, int gauss,
                       double* mean) {
    int C = (n - 1) / 2;
    int64_t S1[ORC_MAXN];
    for (int i = 0; i < n; ++i) {
        int64_t acc = 0;
        for (int j = 0; j < n; ++j) acc += dist_l1(v[i], v[j]);
        S1[i] = acc;
    }
    for (int i = 0; i < n; ++i) {
        if (S1[i] == 0) {
            for (int k = 0; k < 3; ++k) mean[k] = (double)v[C][k];
            return 1;
        }
    }
    double scale = pow((double)n, -kappa / 3.0);
    double num[3] = {0.0, 0.0, 0.0}, den = 0.0;
    for (int i = 0; i < n; ++i) {
        double h = scale * (double)S1[i];
        double z;
        if (gauss) {
            double q = 0.0;
            for (int k = 0; k < 3; ++k) {
                double t = (double)(v[C][k] - v[i][k]) / h;
                q += t * t;
            }
            z = 0.5 * q;
        } else {
            z = (double)dist_l1(v[C], v[i]) / h;
        }
        double wgt = eval_expneg(ep, z) / (h * h * h);
        den += wgt;
        for (int k = 0; k < 3; ++k) num[k] += wgt * (double)v[i][k];
    }
    if (!(den > 0.0)) {
        for (int k = 0; k < 3; ++k) mean[k] = (double)v[C][k];
        return 1;
    }
    for (int k = 0; k < 3; ++k) mean[k] = num[k] / den;
    return 0;
}

int orc_window_amnfe(const int64_t v[][3], int n, double kappa, const orc_exp_t* ep, double* mean) {
    return window_amnf(v, n, kappa, ep, 0, mean);
}

int orc_window_amnfg(const int64_t v[][3], int n, double kappa, const orc_exp_t* ep, double* mean) {
    return window_amnf(v, n, kappa, ep, 1, mean);
}

/* EVMF: returns the selected index (C when not switched). info[0] = P_C,
 * info[1] = H, info[2] = ENT(P_C), info[3] = switched (0/1); S[] receives the
 * vector-median sums (filled in every case). */
int orc_window_evmf(const int64_t v[][3], int n, const orc_ent_t* en, double* info, double* S) {
    int C = (n - 1) / 2;
    double mean[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) mean[k] += (double)v[i][k];
    for (int k = 0; k < 3; ++k) mean[k] /= (double)n;
    double d[ORC_MAXN], D = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) {
            double t = (double)v[i][k] - mean[k];
            s += t * t;
        }
        d[i] = sqrt(s);
        D += d[i];
    }
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += dist_l2(v[i], v[j]);
        S[i] = acc;
    }
    info[0] = info[1] = info[2] = info[3] = 0.0;
    if (D == 0.0) return C;
    double H = 0.0;
    for (int j = 0; j < n; ++j) H -= eval_ent(en, d[j] / D);
    double PC = d[C] / D;
    double entC = eval_ent(en, PC);
    info[0] = PC;
    info[1] = H;
    info[2] = entC;
    if (!(PC * H > -entC)) return C;
    info[3] = 1.0;
    return argmin_tie(S, n);
}

/* ---- whole-image filters ------------------------------------------------- */

static void put_px(void* dst, int bpc, int64_t pitch, int y, int x, const int64_t* v) {
    int64_t off = (int64_t)y * pitch + (int64_t)x * 3;
    for (int k = 0; k < 3; ++k) {
        if (bpc == 1) ((uint8_t*)dst)[off + k] = (uint8_t)v[k];
        else ((uint16_t*)dst)[off + k] = (uint16_t)v[k];
    }
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Filter ids: 0 VDF, 1 DDF, 2 AMNFE, 3 EVMF, 4 AMNFG. rows/cols restrict the work to a
 * list of pixels when npix > 0 (outputs written to dst at those pixels only). */
typedef struct {
    int filter;
    int window;
    double param;            /* DDF: p; AMNFE, AMNFG: kappa */
    orc_acos_t acos_ap;
    orc_exp_t exp_ap;
    orc_ent_t ent_ap;
} orc_cfg_t;

static void filter_pixel(const orc_img_t* im, const orc_cfg_t* cfg, int y, int x,
                         void* dst, int64_t dst_pitch) {
    int64_t v[ORC_MAXN][3];
    double S[ORC_MAXN], S2[ORC_MAXN], S3[ORC_MAXN], info[4];
    int n = gather(im, y, x, cfg->window, v);
    int sel = (n - 1) / 2;
    int64_t out[3];
    switch (cfg->filter) {
    case 0:
        sel = orc_window_vdf((const int64_t(*)[3])v, n, &cfg->acos_ap, S);
        break;
    case 1:
        sel = orc_window_ddf((const int64_t(*)[3])v, n, cfg->param, &cfg->acos_ap, S, S2, S3);
        break;
    case 2:
    case 4: {
        double mean[3];
        window_amnf((const int64_t(*)[3])v, n, cfg->param, &cfg->exp_ap, cfg->filter == 4, mean);
        int64_t maxv = im->bytes_per_channel == 1 ? 255 : 65535;
        for (int k = 0; k < 3; ++k) {
            double r = floor(mean[k] + 0.5);
            if (r < 0) r = 0;
            if (r > (double)maxv) r = (double)maxv;
            out[k] = (int64_t)r;
        }
        put_px(dst, im->bytes_per_channel, dst_pitch, y, x, out);
        return;
    }
    case 3:
        sel = orc_window_evmf((const int64_t(*)[3])v, n, &cfg->ent_ap, info, S);
        break;
    }
    put_px(dst, im->bytes_per_channel, dst_pitch, y, x, v[sel]);
}

/* Filter the whole image (npix == 0) or only the listed pixels. Returns 0. */
int orc_filter(const void* src, int height, int width, int bytes_per_channel,
               int64_t src_pitch, void* dst, int64_t dst_pitch, const orc_cfg_t* cfg,
               const int32_t* ys, const int32_t* xs, int64_t npix, int nthreads) {
    orc_img_t im = {src, height, width, bytes_per_channel, src_pitch};
    set_threads(nthreads);
    if (npix <= 0) {
        #pragma omp parallel for schedule(dynamic, 1)
        for (int y = 0; y < height; ++y)
            for (int x = 0; x < width; ++x) filter_pixel(&im, cfg, y, x, dst, dst_pitch);
    } else {
        #pragma omp parallel for schedule(dynamic, 64)
        for (int64_t t = 0; t < npix; ++t) filter_pixel(&im, cfg, ys[t], xs[t], dst, dst_pitch);
    }
    return 0;
}

/* Per-pixel inspection: gathers the window at (y, x) and fills out[] with the
 * filter's internal quantities. Layout of out (n = window^2):
 *   VDF:   out[0..n)   angle sums;                 returns selected index
 *   DDF:   out[0..n) SA, out[n..2n) SD, out[2n..3n) Psi;  returns selected index
 *   AMNFE, AMNFG: out[0..3) unrounded mean;        returns 1 if uniform
 *   EVMF:  out[0..4) P_C, H, ENT(P_C), switched; out[4..4+n) VMF sums; returns index */
int orc_inspect(const void* src, int height, int width, int bytes_per_channel,
                int64_t src_pitch, const orc_cfg_t* cfg, int y, int x, double* out) {
    orc_img_t im = {src, height, width, bytes_per_channel, src_pitch};
    int64_t v[ORC_MAXN][3];
    int n = gather(&im, y, x, cfg->window, v);
    switch (cfg->filter) {
    case 0: return orc_window_vdf((const int64_t(*)[3])v, n, &cfg->acos_ap, out);
    case 1: return orc_window_ddf((const int64_t(*)[3])v, n, cfg->param, &cfg->acos_ap,
                                  out, out + n, out + 2 * n);
    case 2: return orc_window_amnfe((const int64_t(*)[3])v, n, cfg->param, &cfg->exp_ap, out);
    case 3: return orc_window_evmf((const int64_t(*)[3])v, n, &cfg->ent_ap, out, out + 4);
    case 4: return orc_window_amnfg((const int64_t(*)[3])v, n, cfg->param, &cfg->exp_ap, out);
    }
    return -1;
}

/* Scalar evaluators, exported so the tests can pin them one by one. */
double orc_eval_angle(const orc_acos_t* ap, double z) { return eval_angle(ap, z); }
double orc_eval_expneg(const orc_exp_t* ep, double z) { return eval_expneg(ep, z); }
double orc_eval_ent(const orc_ent_t* en, double z) { return eval_ent(en, z); }
double orc_cosine(const int64_t* a, const int64_t* b) { return cosine(a, b); }
