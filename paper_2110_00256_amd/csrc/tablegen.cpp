// Lookup-table generation for the BW and QS processes (paper Sec. 3.1, 3.2),
// from the Bessel-function integrals of Sec. 2.1 and Sec. 2.2.  Host code,
// FP64, one thread per chi row.
//
// Quadrature design (independent of any other implementation in this
// repository):
//  * e^x K_nu(x) and e^x IK_nu(x), IK_nu(x) = int_x^inf K_nu, from the even
//    integrands exp(-2 x sinh^2(t/2)) cosh(nu t) [/ cosh t] (integral
//    representation DLMF 10.32.9, integrated once for IK) by the trapezoidal
//    rule on the half line, which converges geometrically for even analytic
//    integrands; the step shrinks as 1/sqrt(x) where the integrand becomes a
//    narrow Gaussian in t.
//  * The xi integrals by adaptive tanh-sinh quadrature (the paper also uses
//    tanh-sinh, Sec. 3) on each table interval, evaluated with the distance
//    to the nearer end point so that 1 - xi carries full precision.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "constants.hpp"
#include "tablegen.hpp"

namespace qedmi {
namespace {

// ---------------------------------------------------------------- Bessel
struct BesselPair {
    double ek;   // e^x K_{nu_k}(x)
    double eik;  // e^x int_x^inf K_{nu_ik}(s) ds
};

BesselPair bessel_scaled(double x, double nu_k, double nu_ik) {
    const double h = std::min(0.25, 0.5 / std::sqrt(x));
    const double grow = std::max(nu_k, nu_ik);
    // t = 0 term has weight 1/2 (even integrand on the half line)
    double sk = 0.5, sik = 0.5;
    for (int j = 1; j < 1000000; ++j) {
        const double t = j * h;
        const double s = std::sinh(0.5 * t);
        const double expo = -2.0 * x * s * s;
        const double e = std::exp(expo);
        const double ck = std::cosh(nu_k * t);
        const double cik = std::cosh(nu_ik * t) / std::cosh(t);
        sk += e * ck;
        sik += e * cik;
        // past the maximum of exp(expo + grow t) and 40 e-folds below the sum
        if (expo + grow * t < -40.0 && 2.0 * x * std::sinh(t) > grow &&
            e * ck < 1e-18 * sk && e * cik < 1e-18 * sik)
            break;
    }
    return {sk * h, sik * h};
}

// ---------------------------------------------------------------- tanh-sinh
// Integrand signature: f(x, distance to the lower end A, distance to the
// upper end B) of the ORIGINAL interval; [a, b] is a sub-interval with
// a - A = ea and B - b = eb.
template <class F>
double tanh_sinh_level(const F& f, double a, double b, double ea, double eb, int level,
                       bool odd_only) {
    const double h = std::ldexp(1.0, -level);
    const double d = 0.5 * (b - a);
    double s = 0.0;
    const int jmax = static_cast<int>(std::ceil(3.6 / h));
    for (int j = odd_only ? 1 : 0; j <= jmax; j += odd_only ? 2 : 1) {
        const double t = j * h;
        const double u = 0.5 * kPi * std::sinh(t);
        const double e = std::exp(-2.0 * u);                 // e^{-2u}
        const double off = 2.0 * d * e / (1.0 + e);          // distance from the end point
        const double w = d * 0.5 * kPi * std::cosh(t) * 4.0 * e / ((1.0 + e) * (1.0 + e));
        if (off <= 0.0 || w == 0.0) break;
        if (j == 0) {
            s += w * f(a + d, d + ea, d + eb);
        } else {
            s += w * (f(b - off, (b - a - off) + ea, off + eb) + f(a + off, off + ea, (b - a - off) + eb));
        }
    }
    return s * h;
}

// Non-adaptive estimate at a fixed level (used to size the absolute tolerance).
template <class F>
double tanh_sinh_fixed(const F& f, double a, double b, int level) {
    double s = tanh_sinh_level(f, a, b, 0.0, 0.0, 0, false);
    for (int l = 1; l <= level; ++l) s = 0.5 * s + tanh_sinh_level(f, a, b, 0.0, 0.0, l, true);
    return s;
}

// Adaptive: halve the step until two levels agree to 1e-15 relative or to
// abs_tol (set from the whole integral, so that negligible pieces stop
// early), else bisect the interval (at most 12 times).
template <class F>
double tanh_sinh(const F& f, double a, double b, double abs_tol, double ea = 0.0, double eb = 0.0,
                 int depth = 0) {
    double prev = tanh_sinh_level(f, a, b, ea, eb, 0, false);
    prev = 0.5 * prev + tanh_sinh_level(f, a, b, ea, eb, 1, true);
    prev = 0.5 * prev + tanh_sinh_level(f, a, b, ea, eb, 2, true);
    double cur = prev;
    for (int level = 3; level <= 7; ++level) {
        cur = 0.5 * cur + tanh_sinh_level(f, a, b, ea, eb, level, true);
        if (std::fabs(cur - prev) <= 1e-15 * std::fabs(cur) + abs_tol) return cur;
        prev = cur;
    }
    if (depth >= 12) return cur;
    const double m = 0.5 * (a + b);
    return tanh_sinh(f, a, m, 0.5 * abs_tol, ea, eb + (b - m), depth + 1) +
           tanh_sinh(f, m, b, 0.5 * abs_tol, ea + (m - a), eb, depth + 1);
}

// ---------------------------------------------------------------- integrands
// BW (Sec. 2.1) with u = chi_gamma xi and w = (2/3) s^{3/2}:
//   B(xi) = IK_{1/3}(z) + (1/(xi(1-xi)) - 2) K_{2/3}(z),  z = 2/(3 chi xi (1-xi)),
// T(chi) = int_0^1 B / (pi sqrt3 chi).  Returned scaled by e^{z0}, z0 = 8/(3 chi).
struct BwIntegrand {
    double chi;
    double operator()(double xi, double /*da*/, double db_half) const {
        // db_half is the distance to xi = 1/2 (the right end of every interval
        // is <= 1/2); 1 - xi = 1/2 + (1/2 - xi) is exact enough.
        (void)db_half;
        const double om = 1.0 - xi;
        const double q = xi * om;
        if (!(q > 0.0)) return 0.0;
        const double d = (2.0 / (3.0 * chi)) * (om - xi) * (om - xi) / q;
        if (d > 740.0) return 0.0;
        const BesselPair bp = bessel_scaled(2.0 / (3.0 * chi * q), 2.0 / 3.0, 1.0 / 3.0);
        return std::exp(-d) * (bp.eik + (1.0 / q - 2.0) * bp.ek);
    }
};

// QS (Sec. 2.2): S/xi = (sqrt3/(2 pi)) [IK_{5/3}(Y) + xi^2/(1-xi) K_{2/3}(Y)],
// Y = 2 xi / (3 chi (1 - xi)).  one_minus is 1 - xi to full precision.
inline double qs_bracket(double chi, double xi, double one_minus) {
    if (!(one_minus > 0.0)) return 0.0;
    const double y = 2.0 * xi / (3.0 * chi * one_minus);
    if (y > 740.0) return 0.0;
    if (!(y > 0.0)) return 0.0;
    const BesselPair bp = bessel_scaled(y, 2.0 / 3.0, 5.0 / 3.0);
    return std::exp(-y) * (bp.eik + xi * xi / one_minus * bp.ek);
}

// ---------------------------------------------------------------- rows
void bw_row(double chi, int n_frac, double* ln_t, double* cdf) {
    std::vector<double> cum(n_frac, 0.0);
    const BwIntegrand f{chi};
    double est = 0.0;
    for (int m = 1; m < n_frac; ++m)
        est += tanh_sinh_fixed(f, 0.5 * (m - 1) / (n_frac - 1), 0.5 * m / (n_frac - 1), 4);
    const double abs_tol = 1e-17 * est;
    double s = 0.0;
    for (int m = 1; m < n_frac; ++m) {
        const double a = 0.5 * (m - 1) / (n_frac - 1);
        const double b = 0.5 * m / (n_frac - 1);
        s += tanh_sinh(f, a, b, abs_tol);
        cum[m] = s;
    }
    const double total = 2.0 * s;  // integrand symmetric under xi -> 1 - xi
    const double z0 = 8.0 / (3.0 * chi);
    *ln_t = std::log(total) - z0 - std::log(kPi * std::sqrt(3.0) * chi);
    for (int m = 0; m < n_frac; ++m) cdf[m] = cum[m] / total;
    cdf[0] = 0.0;
    cdf[n_frac - 1] = 0.5;
}

void qs_row(double chi, int n_frac, double frac_min, double* ln_g, double* cdf) {
    std::vector<double> cum(n_frac, 0.0);
    // [0, xi_min]: xi = xi_min s^3 removes the xi^{-2/3} end-point growth
    auto f0 = [&](double sv, double /*da*/, double /*db*/) {
        const double xi = frac_min * sv * sv * sv;
        return qs_bracket(chi, xi, 1.0 - xi) * 3.0 * frac_min * sv * sv;
    };
    const double lmin = std::log(frac_min);
    auto knot = [&](int m) {
        return (m == n_frac - 1) ? 1.0 : std::exp(lmin * (1.0 - double(m) / (n_frac - 1)));
    };
    // the distance to the upper end is 1 - xi exactly on the last interval
    auto f = [&](double xi, double /*da*/, double db) { return qs_bracket(chi, xi, 1.0 - xi); };
    auto flast = [&](double xi, double /*da*/, double db) { return qs_bracket(chi, xi, db); };
    double est = tanh_sinh_fixed(f0, 0.0, 1.0, 4);
    for (int m = 1; m < n_frac - 1; ++m) est += tanh_sinh_fixed(f, knot(m - 1), knot(m), 4);
    est += tanh_sinh_fixed(flast, knot(n_frac - 2), 1.0, 4);
    const double abs_tol = 1e-17 * est;
    double s = tanh_sinh(f0, 0.0, 1.0, abs_tol);
    cum[0] = s;
    for (int m = 1; m < n_frac; ++m) {
        s += (m == n_frac - 1) ? tanh_sinh(flast, knot(m - 1), knot(m), abs_tol)
                               : tanh_sinh(f, knot(m - 1), knot(m), abs_tol);
        cum[m] = s;
    }
    const double total = s;
    *ln_g = std::log(std::sqrt(3.0) / (2.0 * kPi) * total);
    for (int m = 0; m < n_frac; ++m) cdf[m] = std::log(cum[m] / total);
    cdf[n_frac - 1] = 0.0;
}

}  // namespace

double grid_chi(double chi_min, double chi_max, int n_chi, int n) {
    const double l0 = std::log(chi_min), l1 = std::log(chi_max);
    return std::exp(l0 + n * (l1 - l0) / (n_chi - 1));
}

void generate_tables(int process, double chi_min, double chi_max, int n_chi, int n_frac,
                     double frac_min, int n_threads, double* ln_rate, double* cdf) {
    int nt = n_threads > 0 ? n_threads : static_cast<int>(std::thread::hardware_concurrency());
    nt = std::max(1, std::min(nt, n_chi));
    std::atomic<int> next{0};
    auto work = [&]() {
        for (int n = next.fetch_add(1); n < n_chi; n = next.fetch_add(1)) {
            const double chi = grid_chi(chi_min, chi_max, n_chi, n);
            double* row = cdf + static_cast<size_t>(n) * n_frac;
            if (process == 0)
                bw_row(chi, n_frac, &ln_rate[n], row);
            else
                qs_row(chi, n_frac, frac_min, &ln_rate[n], row);
        }
    };
    std::vector<std::thread> pool;
    for (int i = 1; i < nt; ++i) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
}

double bessel_k_scaled(double nu, double x) { return bessel_scaled(x, nu, nu).ek; }
double bessel_ik_scaled(double nu, double x) { return bessel_scaled(x, nu, nu).eik; }

}  // namespace qedmi
