// Minimax polynomial coefficients by the Remez exchange algorithm (paper,
// Section 2: minimise eps = max |f - P| over [a, b] for P in P_n; the paper
// uses Remez exchange and prints the results in Tables 1 and 2).
//
// Design: the iteration works in a Chebyshev basis of the scaled variable
// (T_k((z - mid)/half) for the full basis, T_{2k+1}(z/b) for the odd basis on
// [0, b]) so the levelled systems stay well conditioned up to degree 16; the
// levelled system is solved by Gaussian elimination with partial pivoting;
// error extrema are bracketed on a cosine-spaced grid and polished with
// successive parabolic interpolation; the exchange keeps one extremum per
// sign run and trims the weaker end. The result is re-expanded into monomials
// of z, the form the filters evaluate.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#include "vf_internal.h"

namespace vf {
namespace {

double fn_eval(int func, double z) {
    switch (func) {
    case VF_F_ACOS: return std::acos(z);
    case VF_F_ASIN: return std::asin(z);
    case VF_F_ASIN2_TAU: return 2.0 * std::asin(z / std::sqrt(2.0));
    case VF_F_CHORD: return 2.0 * std::asin(0.5 * z);
    case VF_F_EXPNEG: return std::exp(-z);
    case VF_F_LN1P: return std::log1p(z);
    case VF_F_XLNX: return z > 0.0 ? z * std::log(z) : 0.0;
    }
    return NAN;
}

bool in_domain(int func, double a, double b) {
    switch (func) {
    case VF_F_ACOS:
    case VF_F_ASIN: return a >= -1.0 && b <= 1.0;
    case VF_F_ASIN2_TAU: return a >= -std::sqrt(2.0) && b <= std::sqrt(2.0);
    case VF_F_CHORD: return a >= -2.0 && b <= 2.0;
    case VF_F_EXPNEG: return std::isfinite(a) && std::isfinite(b);
    case VF_F_LN1P: return a > -1.0 && std::isfinite(b);
    case VF_F_XLNX: return a >= 0.0 && std::isfinite(b);
    }
    return false;
}

// Chebyshev values T_0..T_{m-1} at t.
void cheb_all(double t, int m, double* out) {
    if (m > 0) out[0] = 1.0;
    if (m > 1) out[1] = t;
    for (int k = 2; k < m; ++k) out[k] = 2.0 * t * out[k - 1] - out[k - 2];
}

// Solve A x = r (n x n, row-major, destroyed) by Gaussian elimination with
// partial pivoting. Returns false on a singular matrix.
bool gauss_solve(std::vector<double>& A, std::vector<double>& r, int n) {
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int row = col + 1; row < n; ++row)
            if (std::fabs(A[row * n + col]) > std::fabs(A[piv * n + col])) piv = row;
        if (A[piv * n + col] == 0.0) return false;
        if (piv != col) {
            for (int k = 0; k < n; ++k) std::swap(A[piv * n + k], A[col * n + k]);
            std::swap(r[piv], r[col]);
        }
        for (int row = col + 1; row < n; ++row) {
            double f = A[row * n + col] / A[col * n + col];
            if (f == 0.0) continue;
            for (int k = col; k < n; ++k) A[row * n + k] -= f * A[col * n + k];
            r[row] -= f * r[col];
        }
    }
    for (int row = n - 1; row >= 0; --row) {
        double s = r[row];
        for (int k = row + 1; k < n; ++k) s -= A[row * n + k] * r[k];
        r[row] = s / A[row * n + row];
    }
    return true;
}

// The approximation problem in Chebyshev form over a variable x in [lo, hi].
struct Problem {
    int func;
    bool odd;          // odd basis on [0, b]: basis T_{2k+1}(x / b)
    double mid, half;  // full basis: t = (x - mid) / half
    double b;          // odd basis scale
    int m;             // number of basis functions
    double lo, hi;     // search interval of x

    void basis(double x, double* out) const {
        double tmp[40];
        if (!odd) {
            cheb_all((x - mid) / half, m, out);
        } else {
            cheb_all(x / b, 2 * m, tmp);
            for (int k = 0; k < m; ++k) out[k] = tmp[2 * k + 1];
        }
    }
    double approx(const std::vector<double>& c, double x) const {
        double phi[20];
        basis(x, phi);
        double s = 0.0;
        for (int k = m - 1; k >= 0; --k) s += c[k] * phi[k];
        return s;
    }
    double err(const std::vector<double>& c, double x) const { return fn_eval(func, x) - approx(c, x); }
};

// Successive parabolic interpolation for an extremum of g inside [l, r] with
// g(m0) >= g(l), g(r) (g is sign * error).
double polish(const std::function<double(double)>& g, double l, double m0, double r) {
    double gl = g(l), gm = g(m0), gr = g(r);
    for (int it = 0; it < 60; ++it) {
        double d1 = (m0 - l) * (gm - gr), d2 = (m0 - r) * (gm - gl);
        double den = 2.0 * (d1 - d2);
        double x;
        if (den == 0.0) break;
        x = m0 - ((m0 - l) * d1 - (m0 - r) * d2) / den;
        if (!(x > l && x < r) || std::fabs(x - m0) < 1e-17 * std::max(1.0, std::fabs(m0))) {
            // fall back to bisecting the larger side
            x = (m0 - l > r - m0) ? 0.5 * (l + m0) : 0.5 * (m0 + r);
        }
        double gx = g(x);
        if (gx >= gm) {
            if (x < m0) { r = m0; gr = gm; } else { l = m0; gl = gm; }
            m0 = x; gm = gx;
        } else {
            if (x < m0) { l = x; gl = gx; } else { r = x; gr = gx; }
        }
        if (r - l < 1e-16 * std::max(1.0, std::fabs(m0))) break;
    }
    return m0;
}

// Iteration cap: 100 exchanges, or the value of the environment variable
// VF_REMEZ_MAX_ITER (1 .. 100) when set: a way to force VF_ENOCONV in tests.
int remez_max_iter() {
    int cap = 100;
    if (const char* env = std::getenv("VF_REMEZ_MAX_ITER")) {
        const int v = std::atoi(env);
        if (v >= 1 && v <= 100) cap = v;
    }
    return cap;
}

vf_status run_remez(const Problem& P, std::vector<double>& coef, double& E_out) {
    const int max_iter = remez_max_iter();
    const int m = P.m;          // unknown coefficients
    const int npts = m + 1;     // reference points
    std::vector<double> ref(npts);
    if (!P.odd) {
        for (int i = 0; i < npts; ++i)
            ref[i] = P.mid - P.half * std::cos(M_PI * i / (double)(npts - 1));
    } else {
        // positive extrema of T_{2m+1}, ascending
        for (int i = 0; i < npts; ++i)
            ref[i] = P.b * std::cos(M_PI * (double)(npts - 1 - i) / (double)(2 * m + 1));
    }
    std::vector<double> sgn(npts);
    for (int i = 0; i < npts; ++i) sgn[i] = (i % 2 == 0) ? 1.0 : -1.0;

    // cosine-spaced scan grid (dense near the ends where extrema crowd)
    const int G = 3000 * npts;
    std::vector<double> grid(G + 1);
    for (int i = 0; i <= G; ++i) {
        double th = M_PI * (double)(G - i) / (double)G;
        grid[i] = 0.5 * (P.lo + P.hi) + 0.5 * (P.hi - P.lo) * std::cos(th);
    }
    grid[0] = P.lo;
    grid[G] = P.hi;

    std::vector<double> A(npts * npts), rhs(npts), phi(m);
    double E = 0.0;
    for (int iter = 0; iter < max_iter; ++iter) {
        for (int i = 0; i < npts; ++i) {
            P.basis(ref[i], phi.data());
            for (int k = 0; k < m; ++k) A[i * npts + k] = phi[k];
            A[i * npts + m] = sgn[i];
            rhs[i] = fn_eval(P.func, ref[i]);
        }
        if (!gauss_solve(A, rhs, npts)) return VF_ENOCONV;
        coef.assign(rhs.begin(), rhs.begin() + m);
        E = rhs[m];

        std::vector<double> eg(G + 1);
        for (int i = 0; i <= G; ++i) eg[i] = P.err(coef, grid[i]);
        std::vector<double> xs, es;
        auto push = [&](double x) {
            xs.push_back(x);
            es.push_back(P.err(coef, x));
        };
        if (!P.odd) push(P.lo);
        for (int i = 1; i < G; ++i) {
            bool mx = eg[i] >= eg[i - 1] && eg[i] > eg[i + 1];
            bool mn = eg[i] <= eg[i - 1] && eg[i] < eg[i + 1];
            if (!(mx || mn)) continue;
            double s = mx ? 1.0 : -1.0;
            auto g = [&](double x) { return s * P.err(coef, x); };
            push(polish(g, grid[i - 1], grid[i], grid[i + 1]));
        }
        push(P.hi);
        // one extremum per sign run
        std::vector<double> rx, re;
        for (size_t i = 0; i < xs.size(); ++i) {
            if (es[i] == 0.0) continue;
            if (!re.empty() && ((es[i] > 0) == (re.back() > 0))) {
                if (std::fabs(es[i]) > std::fabs(re.back())) {
                    rx.back() = xs[i];
                    re.back() = es[i];
                }
            } else {
                rx.push_back(xs[i]);
                re.push_back(es[i]);
            }
        }
        double emax = 0.0;
        for (double v : re) emax = std::max(emax, std::fabs(v));
        if ((int)rx.size() < npts) return VF_ENOCONV;
        while ((int)rx.size() > npts) {
            if (std::fabs(re.front()) < std::fabs(re.back())) {
                rx.erase(rx.begin());
                re.erase(re.begin());
            } else {
                rx.pop_back();
                re.pop_back();
            }
        }
        // converged when the error curve's extrema equal the levelled error:
        // within 1e-12, and within 1e-10 of |E| relative (FP64 rounding of the
        // error curve allows no less than about 1e-15), so that the
        // coefficients are settled well below their FP32 rounding
        const double tol = std::min(1e-12, std::max(1e-10 * std::fabs(E), 1e-15));
        if (emax - std::fabs(E) <= tol) {
            E_out = std::fabs(E);
            return VF_OK;
        }
        ref = rx;
        for (int i = 0; i < npts; ++i) sgn[i] = re[i] > 0 ? 1.0 : -1.0;
    }
    return VF_ENOCONV;
}

// Rational exchange for R^n_m (Section 2: the best p / q, p in P_n, q in P_m,
// on [lo, hi]), in the Chebyshev basis of t = (x - mid) / half with q's T_0
// coefficient fixed to 1. At each reference t_0 .. t_{n+m+1} the levelled
// equations p(t_i) = (f(t_i) - s_i E) q(t_i) are nonlinear only through the
// product E q; they are solved by fixing that E at its previous value and
// iterating the linear system (p_0..p_n, q_1..q_m, E) to a fixed point. The
// exchange is the polynomial one on the error f - p / q.
vf_status run_remez_rational(const Problem& P, int n, int m, std::vector<double>& pc, std::vector<double>& qc,
                             double& E_out) {
    const int max_iter = remez_max_iter();
    const int npts = n + m + 2;
    std::vector<double> ref(npts), sgn(npts);
    for (int i = 0; i < npts; ++i) {
        const double t = -std::cos(M_PI * i / (double)(npts - 1));
        ref[i] = P.mid + P.half * t;
        sgn[i] = (i % 2 == 0) ? 1.0 : -1.0;
    }
    const int G = 3000 * npts;
    std::vector<double> grid(G + 1);
    for (int i = 0; i <= G; ++i) {
        double th = M_PI * (double)(G - i) / (double)G;
        grid[i] = P.mid + P.half * std::cos(th);
    }
    grid[0] = P.lo;
    grid[G] = P.hi;
    auto cheb = [&](double x, int k, double* out) { cheb_all((x - P.mid) / P.half, k, out); };
    auto rat = [&](double x) {
        double tp[20], tq[20];
        cheb(x, n + 1, tp);
        cheb(x, m + 1, tq);
        double a = 0.0, b = 1.0;
        for (int j = n; j >= 0; --j) a += pc[j] * tp[j];
        for (int k = m; k >= 1; --k) b += qc[k] * tq[k];
        return a / b;
    };
    auto denom = [&](double x) {
        double tq[20];
        cheb(x, m + 1, tq);
        double b = 1.0;
        for (int k = m; k >= 1; --k) b += qc[k] * tq[k];
        return b;
    };
    pc.assign(n + 1, 0.0);
    qc.assign(m + 1, 0.0);
    double E = 0.0;
    std::vector<double> A(npts * npts), rhs(npts);
    for (int iter = 0; iter < max_iter; ++iter) {
        // levelled system at this reference: F_i = p(t_i) - (f_i - s_i E) q(t_i) = 0
        // in x = (p_0..p_n, q_1..q_m, E), bilinear through E q. A first solve
        // with the product's E fixed at its previous value, then Newton steps
        // on the full system (Jacobian columns T_j, -(f_i - s_i E) T_k, s_i q).
        std::vector<double> fi(npts), x(npts, 0.0);
        std::vector<std::vector<double>> tp(npts, std::vector<double>(n + 1)), tq(npts, std::vector<double>(m + 1));
        for (int i = 0; i < npts; ++i) {
            cheb(ref[i], n + 1, tp[i].data());
            cheb(ref[i], m + 1, tq[i].data());
            fi[i] = fn_eval(P.func, ref[i]);
        }
        bool solved = false;
        for (int it2 = 0; it2 < 40; ++it2) {
            const double Ecur = it2 == 0 ? E : x[n + m + 1];
            for (int i = 0; i < npts; ++i) {
                double qv = 1.0, pv = 0.0;
                for (int k = 1; k <= m; ++k) qv += (it2 == 0 ? 0.0 : x[n + k]) * tq[i][k];
                for (int j = 0; j <= n; ++j) pv += (it2 == 0 ? 0.0 : x[j]) * tp[i][j];
                for (int j = 0; j <= n; ++j) A[i * npts + j] = tp[i][j];
                for (int k = 1; k <= m; ++k) A[i * npts + n + k] = -(fi[i] - sgn[i] * Ecur) * tq[i][k];
                if (it2 == 0) {
                    // linear in (p, q, E) with the product's E fixed
                    A[i * npts + n + m + 1] = sgn[i];
                    rhs[i] = fi[i];
                } else {
                    A[i * npts + n + m + 1] = sgn[i] * qv;
                    rhs[i] = -(pv - (fi[i] - sgn[i] * Ecur) * qv);   // -F_i
                }
            }
            if (!gauss_solve(A, rhs, npts)) return VF_ENOCONV;
            double step = 0.0, size = 0.0;
            if (it2 == 0) {
                x = rhs;
            } else {
                for (int k = 0; k < npts; ++k) {
                    x[k] += rhs[k];
                    step = std::max(step, std::fabs(rhs[k]));
                    size = std::max(size, std::fabs(x[k]));
                }
                // (rounding of the solve leaves steps of a few ulps of x)
                if (step <= 1e-13 * size || (it2 == 39 && step <= 1e-8 * size)) {
                    solved = true;
                    break;
                }
            }
        }
        if (!solved) return VF_ENOCONV;
        for (int j = 0; j <= n; ++j) pc[j] = x[j];
        for (int k = 1; k <= m; ++k) qc[k] = x[n + k];
        E = x[n + m + 1];
        // the denominator must keep one sign (no pole) on the interval
        const double q0 = denom(grid[0]);
        for (int i = 0; i <= G; i += 7)
            if (!(denom(grid[i]) * q0 > 0.0)) return VF_ENOCONV;
        std::vector<double> eg(G + 1);
        for (int i = 0; i <= G; ++i) eg[i] = fn_eval(P.func, grid[i]) - rat(grid[i]);
        std::vector<double> xs, es;
        auto push = [&](double x) {
            xs.push_back(x);
            es.push_back(fn_eval(P.func, x) - rat(x));
        };
        push(P.lo);
        for (int i = 1; i < G; ++i) {
            const bool mx = eg[i] >= eg[i - 1] && eg[i] > eg[i + 1];
            const bool mn = eg[i] <= eg[i - 1] && eg[i] < eg[i + 1];
            if (!(mx || mn)) continue;
            const double s = mx ? 1.0 : -1.0;
            auto g = [&](double x) { return s * (fn_eval(P.func, x) - rat(x)); };
            push(polish(g, grid[i - 1], grid[i], grid[i + 1]));
        }
        push(P.hi);
        std::vector<double> rx, re;
        for (size_t i = 0; i < xs.size(); ++i) {
            if (es[i] == 0.0) continue;
            if (!re.empty() && ((es[i] > 0) == (re.back() > 0))) {
                if (std::fabs(es[i]) > std::fabs(re.back())) {
                    rx.back() = xs[i];
                    re.back() = es[i];
                }
            } else {
                rx.push_back(xs[i]);
                re.push_back(es[i]);
            }
        }
        double emax = 0.0;
        for (double v : re) emax = std::max(emax, std::fabs(v));
        // the quotient's FP64 evaluation leaves the error curve about 1e-14 of noise
        const double tol = std::min(1e-12, std::max(1e-10 * std::fabs(E), 1e-14));
        if (emax - std::fabs(E) <= tol) {
            E_out = std::fabs(E);
            return VF_OK;
        }
        if ((int)rx.size() < npts) return VF_ENOCONV;
        while ((int)rx.size() > npts) {
            if (std::fabs(re.front()) < std::fabs(re.back())) {
                rx.erase(rx.begin());
                re.erase(re.begin());
            } else {
                rx.pop_back();
                re.pop_back();
            }
        }
        ref = rx;
        for (int i = 0; i < npts; ++i) sgn[i] = re[i] > 0 ? 1.0 : -1.0;
    }
    return VF_ENOCONV;
}

// Monomial coefficients of T_0..T_{n-1}: mono[k][j] multiplies t^j in T_k.
std::vector<std::vector<double>> cheb_monomials(int n) {
    std::vector<std::vector<double>> T(n, std::vector<double>(n, 0.0));
    if (n > 0) T[0][0] = 1.0;
    if (n > 1) T[1][1] = 1.0;
    for (int k = 2; k < n; ++k) {
        for (int j = 0; j < n; ++j) {
            double v = -T[k - 2][j];
            if (j > 0) v += 2.0 * T[k - 1][j - 1];
            T[k][j] = v;
        }
    }
    return T;
}

// Chebyshev coefficients in t = (z - mid) / half -> monomial coefficients in z.
std::vector<double> cheb_to_z(const std::vector<double>& c, double mid, double half) {
    const int m = (int)c.size();
    auto T = cheb_monomials(m);
    std::vector<double> ct(m, 0.0);   // monomials in t
    for (int k = 0; k < m; ++k)
        for (int j = 0; j <= k; ++j) ct[j] += c[k] * T[k][j];
    std::vector<double> cz(m, 0.0);
    for (int j = 0; j < m; ++j) {
        double scale = ct[j] / std::pow(half, j);
        double binom = 1.0;
        for (int i = 0; i <= j; ++i) {   // (z - mid)^j = sum_i C(j,i) z^i (-mid)^(j-i)
            cz[i] += scale * binom * std::pow(-mid, j - i);
            binom = binom * (double)(j - i) / (double)(i + 1);
        }
    }
    return cz;
}

}  // namespace

vf_status minimax_rational(int func, double a, double b, int n, int m, double* num, double* den,
                           double* err) {
    if (!num || !den || !err) return set_error(VF_EINVAL, "null output pointer");
    if (!(a < b)) return set_error(VF_EINVAL, "interval must satisfy a < b");
    if (n < 0 || m < 0 || n > 8 || m > 8) return set_error(VF_EINVAL, "degrees must be in [0, 8]");
    if (func < VF_F_ACOS || func > VF_F_XLNX) return set_error(VF_EINVAL, "unknown function");
    if (!in_domain(func, a, b)) return set_error(VF_EDOMAIN, "interval leaves the function's domain");
    Problem P{};
    P.func = func;
    P.odd = false;
    P.mid = 0.5 * (a + b);
    P.half = 0.5 * (b - a);
    P.lo = a;
    P.hi = b;
    std::vector<double> pc, qc;
    double E = 0.0;
    vf_status st = run_remez_rational(P, n, m, pc, qc, E);
    if (st != VF_OK) return set_error(st, "rational Remez exchange did not converge");
    qc[0] = 1.0;
    std::vector<double> pz = cheb_to_z(pc, P.mid, P.half), qz = cheb_to_z(qc, P.mid, P.half);
    const double s = qz[0];
    if (!(s != 0.0) || !std::isfinite(s)) return set_error(VF_ENOCONV, "denominator vanishes at z = 0");
    for (int j = 0; j <= n; ++j) num[j] = pz[j] / s;
    for (int k = 0; k <= m; ++k) den[k] = qz[k] / s;
    *err = E;
    return VF_OK;
}

vf_status minimax_coeffs(int func, double a, double b, int degree, int basis, double* out,
                         double* err) {
    if (!out || !err) return set_error(VF_EINVAL, "null output pointer");
    if (!(a < b)) return set_error(VF_EINVAL, "interval must satisfy a < b");
    if (degree < 0 || degree > 16) return set_error(VF_EINVAL, "degree must be in [0, 16]");
    if (func < VF_F_ACOS || func > VF_F_XLNX) return set_error(VF_EINVAL, "unknown function");
    if (!in_domain(func, a, b)) return set_error(VF_EDOMAIN, "interval leaves the function's domain");
    Problem P{};
    P.func = func;
    std::vector<double> c;
    double E = 0.0;
    if (basis == VF_BASIS_FULL) {
        P.odd = false;
        P.mid = 0.5 * (a + b);
        P.half = 0.5 * (b - a);
        P.m = degree + 1;
        P.lo = a;
        P.hi = b;
        vf_status st = run_remez(P, c, E);
        if (st != VF_OK) return set_error(st, "Remez exchange did not converge");
        auto T = cheb_monomials(P.m);
        std::vector<double> ct(P.m, 0.0);   // monomials in t
        for (int k = 0; k < P.m; ++k)
            for (int j = 0; j <= k; ++j) ct[j] += c[k] * T[k][j];
        // t = (z - mid) / half  ->  monomials in z
        std::vector<double> cz(P.m, 0.0);
        for (int j = 0; j < P.m; ++j) {
            double scale = ct[j] / std::pow(P.half, j);
            double binom = 1.0;
            for (int i = 0; i <= j; ++i) {   // (z - mid)^j = sum_i C(j,i) z^i (-mid)^(j-i)
                cz[i] += scale * binom * std::pow(-P.mid, j - i);
                binom = binom * (double)(j - i) / (double)(i + 1);
            }
        }
        for (int j = 0; j < P.m; ++j) out[j] = cz[j];
    } else if (basis == VF_BASIS_ODD) {
        if (degree % 2 != 1) return set_error(VF_EINVAL, "odd basis needs an odd degree");
        if (a != -b) return set_error(VF_EINVAL, "odd basis needs a symmetric interval");
        P.odd = true;
        P.b = b;
        P.m = (degree + 1) / 2;
        P.lo = 0.0;
        P.hi = b;
        vf_status st = run_remez(P, c, E);
        if (st != VF_OK) return set_error(st, "Remez exchange did not converge");
        auto T = cheb_monomials(2 * P.m);
        for (int k = 0; k < P.m; ++k) out[k] = 0.0;
        for (int k = 0; k < P.m; ++k)         // T_{2k+1}(z / b) has only odd powers
            for (int j = 0; j < P.m; ++j)
                out[j] += c[k] * T[2 * k + 1][2 * j + 1] / std::pow(b, 2 * j + 1);
    } else {
        return set_error(VF_EINVAL, "unknown basis");
    }
    *err = E;
    return VF_OK;
}

}  // namespace vf
