// Approximant preparation (host): turns (filter, window, parameter, vf_approx)
// into the FP32 constants the kernels evaluate, with a process-wide cache of
// Remez results.
//
// The paper's printed approximants (Tables 1, 2 and 4) are typed in here as
// printed; minimax ones come from this library's Remez exchange:
//   angle SPLIT d : odd asin fit on [-1/2, 1/2] (lo) and odd chord fit of
//                   2 asin(s/2) on [-1, 1] (hi), s = sqrt(2 (1 - z));
//   angle CHORD d : odd chord fit on [-sqrt 2, sqrt 2] (covers z in [0, 1]);
//   exp MINIMAX d : exp(-z) on [0, min(b, T)], b the largest EXP argument the
//                   AMNF kernel reaches (|x_C - x_i|_2 <= |x_C - x_i|_1 <=
//                   sum_j |x_i - x_j|_1): n^(kappa/3) for the exponential
//                   kernel, 0.5 n^(2 kappa/3) for the Gaussian one; K is 0
//                   above the cutoff T;
//   ENT MINIMAX d : ln(1 + t) on [0, 1] for the reduced mantissa.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "vf_internal.h"

namespace vf {
namespace {

// Table 1 (Section 3.1), monomial coefficients a_0..a_4.
const double kT1Arccos[5] = {1.570786, -9.990285e-01, -1.429899e-02, -9.481335e-02, -1.381942e-01};
const double kT1Arcsin[5] = {2.097797e-05, 1.412840, 1.429881e-02, 6.704361e-02, 6.909677e-02};
const double kT1Eps = 2.097814e-05;
// Table 2 (Section 3.2): exp(-z) on [0, 10].
const double kT2P2[3] = {8.214528e-01, -3.186948e-01, 2.544088e-02};
const double kT2P3[4] = {9.174126e-01, -5.631179e-01, 1.015041e-01, -5.519183e-03};
const double kT2P4[5] = {9.666313e-01, -7.620584e-01, 2.145386e-01, -2.509526e-02, 1.032877e-03};
const double kT2Eps[5] = {0, 0, 1.785517e-01, 8.259345e-02, 3.337085e-02};
// Table 3 (Section 3.2): exp(-z) on [0, 10], numerator / denominator.
const double kT3Num[5] = {3.206619e-02, -1.195191e-02, 1.756974e-03, -1.199261e-04, 3.182685e-06};
const double kT3Den[5] = {3.206627e-02, 2.011147e-02, 5.853684e-03, 9.780143e-04, 1.251598e-04};
const double kT3Eps = 2.227050e-06;
// Table 4 (Section 3.3): z ln z on [0.05, 1], numerator / denominator.
const double kT4Num[5] = {-1.519742e-04, -6.835769e-02, -8.856923e-01, -5.369609e-01, 1.491165};
const double kT4Den[5] = {1.532270e-02, 3.987796e-01, 1.461793, 6.827004e-01, -4.469776e-02};
const double kT4Eps = 7.342477e-07;
const double kExpCutoff = 10.0;   // Section 3.2: 0 for arguments above T = 10
const double kEntCutoff = 0.05;   // Section 3.3: 0 for arguments below T = 0.05

// Per-pair FP32 error bound of a polynomial angle evaluation, |computed -
// polynomial in exact arithmetic| <= eta + rho * angle:
//  * unit vectors rounded to FP32 (2^-24 per component), their difference and
//    the FMA sum of squares move the chord s by at most 2^-23 + 4.5 2^-24 s,
//    and d(angle)/ds <= sqrt 2: at most 1.7e-7 + 3.8e-7 angle;
//  * Horner in FP32 with m <= 7 coefficients: relative 2m 2^-24 of
//    sum |c_k| x^k (within 1% of p for these fits), the scaling by s and the
//    square root 2^-24 each: at most 9.5e-7 angle (the split form's pi/2 -
//    z L(z^2) piece is below that relative to its angles >= pi/3).
// Rounded up: eta = 2e-7, rho = 1.4e-6. Sums over the window's n - 1 pairs
// then give (n - 1) eta + rho S_i, added to the summation bound.
const float kAngleEta = 2.0e-7f;
const double kAngleRho = 1.4e-6;
// The packed FP16 variant adds FP16 subnormal rounding of the correction
// (at most 7 x 2^-25 s <= 2.1e-7 angle) to rho, plus its own FP16 term.
const double kAngleRhoF16Sub = 2.1e-7;

// Minimax exp and ENT fits whose levelled error lies below the FP32 unit
// roundoff of the function's largest value are refused: evaluated in FP32
// they are no more accurate than the fit of the degree below, and their
// highest monomial coefficients (of order 1e-5 and less) are not determined
// by an FP64 Remez exchange to the precision of their FP32 rounding (two
// correct FP64 implementations round them differently).
const double kFitFloor = 5.9604644775390625e-08;   // 2^-24
const char* const kFitFloorMsg =
    "minimax error of this degree is below the FP32 resolution of the function: take a lower degree";

struct Fit {
    std::vector<double> c;
    double err;
};

std::mutex g_mu;
std::map<std::tuple<int, double, double, int, int>, Fit> g_cache;

vf_status fit(int func, double a, double b, int degree, int basis, Fit* out) {
    auto key = std::make_tuple(func, a, b, degree, basis);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            *out = it->second;
            return VF_OK;
        }
    }
    Fit f;
    f.c.assign(kMaxCoef, 0.0);
    vf_status st = minimax_coeffs(func, a, b, degree, basis, f.c.data(), &f.err);
    if (st != VF_OK) return st;
    f.c.resize(basis == VF_BASIS_ODD ? (degree + 1) / 2 : degree + 1);
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = f;
    *out = f;
    return VF_OK;
}

// Fitted R^d_d rationals, cached like the polynomial fits.
std::map<std::tuple<int, double, double, int>, std::vector<double>> g_rcache;

vf_status rational_fit(int func, double a, double b, int d, double* num, double* den, double* err) {
    auto key = std::make_tuple(func, a, b, d);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_rcache.find(key);
        if (it != g_rcache.end()) {
            for (int i = 0; i <= d; ++i) num[i] = it->second[i];
            for (int i = 0; i <= d; ++i) den[i] = it->second[d + 1 + i];
            *err = it->second[2 * d + 2];
            return VF_OK;
        }
    }
    vf_status st = minimax_rational(func, a, b, d, d, num, den, err);
    if (st != VF_OK) return st;
    std::vector<double> v(2 * d + 3);
    for (int i = 0; i <= d; ++i) v[i] = num[i];
    for (int i = 0; i <= d; ++i) v[d + 1 + i] = den[i];
    v[2 * d + 2] = *err;
    std::lock_guard<std::mutex> lk(g_mu);
    g_rcache[key] = v;
    return VF_OK;
}

void put(float* dst, int* n, const double* src, int count) {
    for (int i = 0; i < count; ++i) dst[i] = (float)src[i];   // round to nearest FP32
    *n = count;
}

}  // namespace

// Relative error bound rho of the packed-FP16 chord evaluation (per pair,
// |angle_computed - angle_poly| <= eta + rho * angle): x = s^2 is rounded to FP16
// (relative 2^-11), the correction t = x q(x) takes m - 2 FMAs and one multiply
// in FP16, each rounding once (relative 2^-11 of a sum of non-negative terms
// bounded by sum_k |c_k| x^k), so |dt| <= (m + 1) 2^-11 sum_{k>=1} |c_k| x^k and
// the angle error is s |dt|. rho is the maximum over s in (0, sqrt 2] of that
// over the angle itself (evaluated on a fine grid, plus 10%). FP16
// subnormals add at most (m + 1) 2^-25 s absolute, which eta covers.
static double f16_relative_bound(const float* c, int m) {
    const double u16 = std::ldexp(1.0, -11);
    double worst = 0.0;
    for (int i = 1; i <= 4096; ++i) {
        const double s = std::sqrt(2.0) * i / 4096.0;
        const double x = s * s;
        double t = 0.0, a = 0.0, xp = x;
        for (int k = 1; k < m; ++k, xp *= x) a += std::fabs((double)c[k]) * xp;
        xp = 1.0;
        for (int k = 0; k < m; ++k, xp *= x) t += (double)c[k] * xp;
        const double angle = s * t;
        worst = std::max(worst, (m + 1) * u16 * s * a / angle);
    }
    return worst * 1.1;
}

// Absolute error bound of the packed-FP16 correction t(x) = sum_{k>=1} c_k x^k
// over x in [0, xmax] (exp: x = z; ln1p: x = the reduced mantissa t), the
// part of p(x) = c_0 + t(x) that the AMNFE / EVMF FP16 variants evaluate in
// FP16 (c_0 is added in FP32): x rounded to FP16 moves t by at most
// max|t'| (2^-11 x + 2^-25); Horner's m - 2 FMAs and the final multiply round
// m - 1 times, |error| <= gamma_{m-1} sum_{k>=1} |c_k| x^k with u = 2^-11
// (Higham's FMA-Horner bound); FP16 subnormals add at most 2^-25 per rounding,
// carried through later steps by at most max(1, xmax)^k. The maximum over a
// 4097-point grid, plus 10% for the grid.
static double f16_correction_bound(const float* c, int m, double xmax) {
    const double u = std::ldexp(1.0, -11), sub = std::ldexp(1.0, -25);
    const double gam = (m - 1) * u / (1.0 - (m - 1) * u);
    double dmax = 0.0;   // max |t'| on the interval
    for (int i = 0; i <= 4096; ++i) {
        const double x = xmax * i / 4096.0;
        double d = 0.0, xp = 1.0;
        for (int k = 1; k < m; ++k, xp *= x) d += k * (double)c[k] * xp;
        dmax = std::max(dmax, std::fabs(d));
    }
    const double big = std::max(1.0, xmax);
    double carry = 0.0, bp = 1.0;
    for (int k = 0; k < m; ++k, bp *= big) carry += bp;
    double worst = 0.0;
    for (int i = 0; i <= 4096; ++i) {
        const double x = xmax * i / 4096.0;
        double a = 0.0, xp = x;
        for (int k = 1; k < m; ++k, xp *= x) a += std::fabs((double)c[k]) * xp;
        worst = std::max(worst, dmax * (u * x + sub) + gam * a + (m - 1) * sub * carry);
    }
    return worst * 1.1;
}

// Absolute error bound of the FP32 Horner evaluation of the polynomial c(x)
// on [0, xmax] at a given FP32 argument (coefficients already FP32): the
// kernels' Horner rounds once per FMA, m - 1 times, so gamma_{m-1} sum |c_k| x^k
// with 2^-24 units. Maximum over a 4097-point grid with 10% margin.
static double horner_bound(const float* c, int m, double xmax) {
    const double u = std::ldexp(1.0, -24);
    const double g = (m - 1) * u / (1.0 - (m - 1) * u);
    double worst = 0.0;
    for (int i = 0; i <= 4096; ++i) {
        const double x = xmax * i / 4096.0;
        double s = 0.0, xp = 1.0;
        for (int k = 0; k < m; ++k, xp *= x) s += std::fabs((double)c[k]) * xp;
        worst = std::max(worst, g * s);
    }
    return worst * 1.1;
}

// Absolute error bound of the FP32 evaluation of the rational a(x) / b(x) on
// [0, xmax] at a given FP32 argument (coefficients already FP32): Horner with
// FMA keeps each of a and b within gamma_{m-1} sum |c_k| x^k (2^-24 units),
// and the correctly rounded divide adds 2^-24 of the quotient:
// |computed - a/b| <= (Ea + |a/b| Eb) / (b - Eb) + 2^-24 |a/b|. Maximum over a
// 4097-point grid with 10% margin (b > 0 and smooth on the interval).
static double rational_bound(const float* a, int na, const float* b, int nb, double xmax) {
    const double u = std::ldexp(1.0, -24);
    const double ga = (na - 1) * u / (1.0 - (na - 1) * u);
    const double gb = (nb - 1) * u / (1.0 - (nb - 1) * u);
    double worst = 0.0;
    for (int i = 0; i <= 4096; ++i) {
        const double x = xmax * i / 4096.0;
        double va = 0.0, vb = 0.0, sa = 0.0, sb = 0.0, xp = 1.0;
        for (int k = 0; k < std::max(na, nb); ++k, xp *= x) {
            if (k < na) { va += (double)a[k] * xp; sa += std::fabs((double)a[k]) * xp; }
            if (k < nb) { vb += (double)b[k] * xp; sb += std::fabs((double)b[k]) * xp; }
        }
        const double q = std::fabs(va / vb), ea = ga * sa, eb = gb * sb;
        worst = std::max(worst, (ea + q * eb) / (vb - eb) + u * q);
    }
    return worst * 1.1;
}

// Relative bound of each AMNFE weight K(z) h^-3 from an absolute bound rho of
// the evaluated K: rho / K_min with K_min the least value of the approximant
// a(x) (or a(x) / b(x)) on [0, xmax] (4097-point grid, 1% margin; these
// approximants decrease, the minimum sits at xmax). Perturbing every weight by
// a relative r moves the mean y = x_C + sum w d / sum w by at most
// r (sum w |d| / sum w + |y - x_C|) / (1 - r); returned as r / (1 - r), or
// 1e30 when K_min <= rho: then the kernels flag every window (weights may be
// zero or negative, e.g. a low-degree fit over [0, T] near T, and no FP32
// bound of the mean holds).
static double weight_rel_bound(double rho, const float* a, int na, const float* b, int nb, double xmax) {
    double kmin = 1e300;
    for (int i = 0; i <= 4096; ++i) {
        const double x = xmax * i / 4096.0;
        double va = 0.0, vb = 0.0, xp = 1.0;
        for (int k = 0; k < std::max(na, nb); ++k, xp *= x) {
            if (k < na) va += (double)a[k] * xp;
            if (k < nb) vb += (double)b[k] * xp;
        }
        kmin = std::min(kmin, nb > 0 ? va / vb : va);
    }
    kmin *= 0.99;
    if (!(kmin > rho)) return 1e30;
    const double r = rho / kmin;
    return r / (1.0 - r);
}

// Round c_1 .. c_{m-1} to FP16 (round to nearest even); c_0 stays FP32.
static void round_f16_tail(float* c, int m) {
    for (int k = 1; k < m; ++k) c[k] = (float)(_Float16)c[k];
}

// max |f(x) - p(x)| over x in [0, xmax] on a 65537-point grid, f = exp(-x) or
// ln(1 + x) (the error of a minimax polynomial once its coefficients are
// rounded).
static double poly_error(const float* c, int m, double xmax, int func) {
    double worst = 0.0;
    for (int i = 0; i <= 65536; ++i) {
        const double x = xmax * i / 65536.0;
        double acc = 0.0;
        for (int k = m - 1; k >= 0; --k) acc = acc * x + (double)c[k];
        const double f = func == VF_F_EXPNEG ? std::exp(-x) : std::log1p(x);
        worst = std::max(worst, std::fabs(f - acc));
    }
    return worst;
}

// max |2 asin(s/2) - s p(s^2)| over s in [0, sqrt 2] on a 65537-point grid
// (the error of the chord polynomial once its coefficients are rounded).
static double chord_error(const float* c, int m) {
    double worst = 0.0;
    for (int i = 0; i <= 65536; ++i) {
        const double s = std::sqrt(2.0) * i / 65536.0;
        const double x = s * s;
        double acc = 0.0;
        for (int k = m - 1; k >= 0; --k) acc = acc * x + (double)c[k];
        worst = std::max(worst, std::fabs(2.0 * std::asin(0.5 * s) - s * acc));
    }
    return worst;
}

vf_status prepare(int filter, int window, double param, const vf_approx* ap, Prepared* out) {
    if (!ap) return set_error(VF_EINVAL, "approx is null");
    if (window != 3 && window != 5 && window != 7)
        return set_error(window > 0 && window % 2 == 1 ? VF_EUNSUPPORTED : VF_EINVAL,
                         "window must be 3, 5 or 7");
    if (ap->precision != VF_PREC_FP32 && ap->precision != VF_PREC_FP16X2 && ap->precision != VF_PREC_FP64)
        return set_error(VF_EINVAL, "unknown precision");
    if (ap->precision == VF_PREC_FP64 && ap->scheme != VF_SCHEME_HORNER)
        return set_error(VF_EUNSUPPORTED, "FP64 evaluation uses Horner's scheme");
    if (ap->scheme != VF_SCHEME_HORNER && ap->scheme != VF_SCHEME_ESTRIN)
        return set_error(VF_EINVAL, "unknown evaluation scheme");
    const bool chord_angle = (filter == VF_FILTER_VDF || filter == VF_FILTER_DDF) && ap->eval == VF_EVAL_CHORD;
    const bool fe_minimax = (is_amnf(filter) || filter == VF_FILTER_EVMF) && ap->eval == VF_EVAL_MINIMAX;
    if (ap->precision == VF_PREC_FP16X2 && !chord_angle && !fe_minimax)
        return set_error(VF_EUNSUPPORTED,
                         "packed FP16 is implemented for the chord angle and the minimax exp / ln approximants");
    if (ap->scheme == VF_SCHEME_ESTRIN && !chord_angle)
        return set_error(VF_EUNSUPPORTED, "Estrin evaluation is implemented for the chord angle approximant only");
    if (ap->scheme == VF_SCHEME_ESTRIN && ap->precision == VF_PREC_FP16X2)
        return set_error(VF_EUNSUPPORTED, "packed FP16 evaluation uses Horner's scheme");
    Prepared P;
    std::memset(&P, 0, sizeof(P));
    P.filter = filter;
    P.window = window;
    P.eval = ap->eval;
    P.degree = ap->degree;
    P.param = param;
    const int n = window * window;
    Fit f, g;
    vf_status st;
    switch (filter) {
    case VF_FILTER_VDF:
    case VF_FILTER_DDF:
        if (filter == VF_FILTER_DDF && !(param >= 0.0 && param <= 1.0))
            return set_error(VF_EINVAL, "DDF exponent p must lie in [0, 1]");
        P.kscale = (float)param;
        switch (ap->eval) {
        case VF_EVAL_EXACT:
            break;
        case VF_EVAL_PAPER:
            if (ap->degree != 4 && ap->degree != 0)
                return set_error(VF_EUNSUPPORTED, "the paper's arccos approximant has degree 4");
            P.degree = 4;
            put(P.lo, &P.n_lo, kT1Arccos, 5);
            put(P.hi, &P.n_hi, kT1Arcsin, 5);
            P.eps = kT1Eps;
            P.eta = kAngleEta;
            P.rho = kAngleRho;
            break;
        case VF_EVAL_SPLIT:
            if (ap->degree < 3 || ap->degree > 9 || ap->degree % 2 == 0)
                return set_error(VF_EUNSUPPORTED, "split angle degree must be 3, 5, 7 or 9");
            if ((st = fit(VF_F_ASIN, -0.5, 0.5, ap->degree, VF_BASIS_ODD, &f)) != VF_OK) return st;
            if ((st = fit(VF_F_CHORD, -1.0, 1.0, ap->degree, VF_BASIS_ODD, &g)) != VF_OK) return st;
            put(P.lo, &P.n_lo, f.c.data(), (int)f.c.size());
            put(P.hi, &P.n_hi, g.c.data(), (int)g.c.size());
            P.eps = f.err > g.err ? f.err : g.err;
            P.eta = kAngleEta;
            P.rho = kAngleRho;
            break;
        case VF_EVAL_CHORD:
            if (ap->degree < 7 || ap->degree > 13 || ap->degree % 2 == 0)
                return set_error(VF_EUNSUPPORTED, "chord angle degree must be 7, 9, 11 or 13");
            if ((st = fit(VF_F_CHORD, -std::sqrt(2.0), std::sqrt(2.0), ap->degree, VF_BASIS_ODD,
                          &g)) != VF_OK)
                return st;
            put(P.hi, &P.n_hi, g.c.data(), (int)g.c.size());
            P.n_lo = 0;
            P.eps = g.err;
            P.eta = kAngleEta;
            P.rho = kAngleRho;   // Estrin: the same per-coefficient rounding count
            P.variant = ap->scheme == VF_SCHEME_ESTRIN ? 1 : 0;
            if (ap->precision == VF_PREC_FP16X2) {
                P.variant = 2;
                // c_1 .. c_{m-1} become FP16 constants (round to nearest even); c_0 stays FP32
                for (int k = 1; k < P.n_hi; ++k) P.hi[k] = (float)(_Float16)P.hi[k];
                P.rho = kAngleRho + kAngleRhoF16Sub + f16_relative_bound(P.hi, P.n_hi);
                P.eps = chord_error(P.hi, P.n_hi);
            }
            break;
        default:
            return set_error(VF_EUNSUPPORTED, "angle filters take EXACT, PAPER, SPLIT or CHORD");
        }
        break;
    case VF_FILTER_AMNFE:
    case VF_FILTER_AMNFG: {
        if (!(param > 0.0) || !std::isfinite(param)) return set_error(VF_EINVAL, "kappa must be > 0");
        const bool gauss = filter == VF_FILTER_AMNFG;
        const double ks = std::pow((double)n, param / 3.0);
        P.kscale = (float)ks;
        P.cutoff = (float)kExpCutoff;
        P.cutoff64 = kExpCutoff;
        // the argument stays in [0, b], b = n^(kappa/3) (exponential kernel) or
        // 0.5 n^(2 kappa/3) (Gaussian kernel), and K is 0 above T
        const double b = gauss ? 0.5 * ks * ks : ks;
        const double zr = std::min(b, kExpCutoff);
        // FP32 error of one weight K(z) S1^-3, relative, in units of 2^-24: the
        // reciprocal of S1 (one ulp, 2 units) cubed with two roundings (8), expf
        // (one ulp, 2) and the product (1), 3 spare; plus the argument's own
        // relative error (exponential: z = L1 rs k_s, 5 units with the rounding
        // of k_s; Gaussian: z = 0.5 q (rs k_s)^2, 13 units with q's three
        // roundings) times z <= zr, since |dK / K| = |dz|.
        const double zrel = gauss ? 13.0 : 5.0;
        P.wbound = (float)(16.0 + zrel * zr);
        // where the argument can reach the cutoff, K jumps there: a member
        // whose computed z lies within twice its error bound of T may sit on
        // the other side of T in exact arithmetic
        P.zband = b >= kExpCutoff * (1.0 - 1e-4) ? (float)(2.0 * zrel * std::ldexp(kExpCutoff, -24)) : 0.0f;
        switch (ap->eval) {
        case VF_EVAL_EXACT:
            break;
        case VF_EVAL_PAPER:
            if (ap->degree == 2) put(P.lo, &P.n_lo, kT2P2, 3);
            else if (ap->degree == 3) put(P.lo, &P.n_lo, kT2P3, 4);
            else if (ap->degree == 4) put(P.lo, &P.n_lo, kT2P4, 5);
            else return set_error(VF_EUNSUPPORTED, "the paper's exp polynomials have degree 2, 3 or 4");
            P.eps = kT2Eps[ap->degree];
            P.rho = weight_rel_bound(horner_bound(P.lo, P.n_lo, zr), P.lo, P.n_lo, nullptr, 0, zr);
            break;
        case VF_EVAL_MINIMAX:
            if (ap->degree < 2 || ap->degree > 9)
                return set_error(VF_EUNSUPPORTED, "exp minimax degree must be in [2, 9]");
            if ((st = fit(VF_F_EXPNEG, 0.0, zr, ap->degree, VF_BASIS_FULL, &f)) != VF_OK) return st;
            if (f.err < kFitFloor * 1.0)   // (max exp(-z) = 1 on [0, zr])
                return set_error(VF_EUNSUPPORTED, kFitFloorMsg);
            put(P.lo, &P.n_lo, f.c.data(), (int)f.c.size());
            P.eps = f.err;
            P.rho = weight_rel_bound(horner_bound(P.lo, P.n_lo, zr), P.lo, P.n_lo, nullptr, 0, zr);
            if (ap->precision == VF_PREC_FP16X2) {
                P.variant = 2;
                round_f16_tail(P.lo, P.n_lo);
                P.rho = f16_correction_bound(P.lo, P.n_lo, zr);
                P.eps = poly_error(P.lo, P.n_lo, zr, VF_F_EXPNEG);
            }
            break;
        case VF_EVAL_RATFIT: {
            if (ap->degree < 1 || ap->degree > 4)
                return set_error(VF_EUNSUPPORTED, "fitted exp rational degree must be in [1, 4]");
            if (ap->precision == VF_PREC_FP16X2)
                return set_error(VF_EUNSUPPORTED, "rational approximants evaluate in FP32");
            double num[9], den[9], err = 0.0;
            if ((st = rational_fit(VF_F_EXPNEG, 0.0, zr, ap->degree, num, den, &err)) != VF_OK) {
                // past a degree whose error is already under FP32 resolution the
                // exchange turns ill-conditioned (errors near FP64 noise): such a
                // degree is refused like the fits below FP32 resolution
                double e2 = 1.0;
                if (ap->degree > 1 && rational_fit(VF_F_EXPNEG, 0.0, zr, ap->degree - 1, num, den, &e2) == VF_OK &&
                    e2 < kFitFloor)
                    return set_error(VF_EUNSUPPORTED, kFitFloorMsg);
                return st;
            }
            if (err < kFitFloor * 1.0) return set_error(VF_EUNSUPPORTED, kFitFloorMsg);
            put(P.lo, &P.n_lo, num, ap->degree + 1);
            put(P.hi, &P.n_hi, den, ap->degree + 1);
            P.eps = err;
            P.rho = weight_rel_bound(rational_bound(P.lo, P.n_lo, P.hi, P.n_hi, zr), P.lo, P.n_lo, P.hi,
                                     P.n_hi, zr);
            break;
        }
        case VF_EVAL_RATIONAL:
            if (ap->degree != 4 && ap->degree != 0)
                return set_error(VF_EUNSUPPORTED, "the paper's exp rational has degree 4");
            P.degree = 4;
            put(P.lo, &P.n_lo, kT3Num, 5);
            put(P.hi, &P.n_hi, kT3Den, 5);
            P.eps = kT3Eps;
            P.rho = weight_rel_bound(rational_bound(P.lo, P.n_lo, P.hi, P.n_hi, zr), P.lo, P.n_lo, P.hi,
                                     P.n_hi, zr);
            break;
        default:
            return set_error(VF_EUNSUPPORTED, "AMNFE and AMNFG take EXACT, PAPER, MINIMAX, RATIONAL or RATFIT");
        }
        break;
    }
    case VF_FILTER_EVMF:
        // param: the cutoff T (Section 3.3), ENT(z) = 0 for z < T in every mode
        if (!(param >= 0.0 && param <= 1.0)) return set_error(VF_EINVAL, "the ENT cutoff T must be in [0, 1]");
        P.cutoff = (float)param;
        P.cutoff64 = param;
        switch (ap->eval) {
        case VF_EVAL_EXACT:
            break;
        case VF_EVAL_PAPER:
            if (param < kEntCutoff)
                return set_error(VF_EDOMAIN, "the Table 4 rational holds on [0.05, 1]: the cutoff T must be >= 0.05");
            put(P.lo, &P.n_lo, kT4Num, 5);
            put(P.hi, &P.n_hi, kT4Den, 5);
            P.eps = kT4Eps;
            P.degree = 4;
            break;
        case VF_EVAL_MINIMAX:
            if (ap->degree < 2 || ap->degree > 9)
                return set_error(VF_EUNSUPPORTED, "ENT minimax degree must be in [2, 9]");
            if ((st = fit(VF_F_LN1P, 0.0, 1.0, ap->degree, VF_BASIS_FULL, &f)) != VF_OK) return st;
            if (f.err < kFitFloor * std::log(2.0))   // (max ln(1 + t) = ln 2 on [0, 1])
                return set_error(VF_EUNSUPPORTED, kFitFloorMsg);
            put(P.lo, &P.n_lo, f.c.data(), (int)f.c.size());
            P.eps = f.err;
            if (ap->precision == VF_PREC_FP16X2) {
                P.variant = 2;
                round_f16_tail(P.lo, P.n_lo);
                P.rho = f16_correction_bound(P.lo, P.n_lo, 1.0);
                P.eps = poly_error(P.lo, P.n_lo, 1.0, VF_F_LN1P);
            }
            break;
        default:
            return set_error(VF_EUNSUPPORTED, "EVMF takes EXACT, PAPER or MINIMAX");
        }
        break;
    default:
        return set_error(VF_EINVAL, "unknown filter");
    }
    if (ap->precision == VF_PREC_FP64) P.variant = 3;   // the same constants, widened to FP64
    *out = P;
    return VF_OK;
}

}  // namespace vf
