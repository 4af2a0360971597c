// Host-code driver for the AddressSanitizer / UndefinedBehaviorSanitizer build
// of the library's host C++ (approximant preparation and both Remez
// exchanges). Runs every filter / window / evaluation / degree / precision /
// scheme combination through prepare(), valid or not, every elementary
// function through the polynomial Remez at all degrees and both bases, and
// the rational Remez at small degrees; exits 0 when nothing aborted. Built
// and run by tests/test_sanitizers.py with the ROCm host compiler.
#include <cmath>
#include <cstdio>
#include <initializer_list>

#include "vf_internal.h"

namespace vf {
// the library's error reporter lives in the HIP part; a silent stand-in here
vf_status set_error(vf_status st, const char*) { return st; }
}  // namespace vf

int main() {
    long ok = 0, refused = 0;
    const double params[] = {0.0, 0.05, 0.33, 0.5, 1.0, 4.0, -1.0, NAN};
    for (int filter = -1; filter <= 5; ++filter)
        for (int window : {1, 3, 4, 5, 7, 9})
            for (int eval = -1; eval <= 7; ++eval)
                for (int degree : {-1, 0, 1, 2, 3, 4, 5, 6, 7, 9, 11, 13, 16, 17})
                    for (int prec = -1; prec <= 3; ++prec)
                        for (int scheme = 0; scheme <= 2; ++scheme)
                            for (double param : params) {
                                vf_approx a{};
                                a.eval = eval;
                                a.degree = degree;
                                a.precision = prec;
                                a.scheme = scheme;
                                vf::Prepared P;
                                if (vf::prepare(filter, window, param, &a, &P) == VF_OK) {
                                    ++ok;
                                    if (!(P.n_lo >= 0 && P.n_lo <= vf::kMaxCoef && P.n_hi >= 0 &&
                                          P.n_hi <= vf::kMaxCoef)) {
                                        std::fprintf(stderr, "coefficient count out of range\n");
                                        return 2;
                                    }
                                } else {
                                    ++refused;
                                }
                            }
    if (vf::prepare(VF_FILTER_VDF, 3, 0.0, nullptr, nullptr) == VF_OK) return 3;
    double c[24], err;
    for (int func = 0; func <= 8; ++func)
        for (int basis = 0; basis <= 1; ++basis)
            for (int d = -1; d <= 17; ++d) {
                const double a = func == VF_F_XLNX ? 0.05 : (basis == 1 ? -0.5 : 0.0);
                (void)vf::minimax_coeffs(func, a, 1.0, d, basis, c, &err);
                (void)vf::minimax_coeffs(func, 1.0, 0.0, d, basis, c, &err);   // empty interval
            }
    double num[12], den[12];
    for (int n = -1; n <= 4; ++n)
        for (int m = -1; m <= 3; ++m) {
            (void)vf::minimax_rational(VF_F_EXPNEG, 0.0, 1.5, n, m, num, den, &err);
            (void)vf::minimax_rational(VF_F_XLNX, 0.05, 1.0, n, m, num, den, &err);
        }
    std::printf("prepare: %ld accepted, %ld refused\n", ok, refused);
    return 0;
}
