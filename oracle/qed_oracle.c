/*
 * qed_oracle.c -- CPU reference ("oracle") for the strong-field QED Monte
 * Carlo step of PICSAR-QED (Fedeli et al., arXiv:2110.00256).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is plain, slow, FP64 C that follows
 * the paper's definitions step by step.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, constant or table with the HIP library; the only thing the
 * two sides have in common is the seeded input arrays.
 *
 * Contents, with the passage each part follows:
 *   - CODATA constants, Schwinger field E_s (paper Sec. 2, definition of E_s).
 *   - Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), used for every
 *     runtime draw.  The paper leaves the generator to the caller
 *     (Sec. 3.3, "Avoid dependencies on specific pseudo-random number
 *     generators"); the counter layout (seed; id, step, species, block) is
 *     this library's choice.
 *   - K_nu(x) and its tail integral IK_nu(x) = int_x^inf K_nu(s) ds from the
 *     integral representation K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt
 *     (DLMF 10.32.9), integrated once in x for IK.
 *   - Lookup tables (Sec. 3.1, 3.2): ln T(chi) and the BW cumulative
 *     distribution P(chi, xi) on linear xi in [0, 1/2]; ln G(chi) and the QS
 *     cumulative distribution ln P(chi, xi) on log-spaced xi in [xi_min, 1].
 *     Integrands from Sec. 2.1 (T(chi_gamma), the BW differential rate after
 *     chi_+ = chi_gamma - chi_-) and Sec. 2.2 (G(chi) and S(chi, xi)).
 *   - chi for leptons and photons (Sec. 2, quantum parameter definitions).
 *   - Runtime rate interpolation, out-of-table rules, inverse-CDF sampling
 *     (Sec. 3.1 and 3.2), product kinematics (Sec. 2.1, 2.2), the optical
 *     depth update and event test (Sec. 3 introduction, Fig. 1 caption).
 *   - Sequential, parent-ordered product append.
 *
 * Readings of the paper taken where it is silent or inconsistent are listed
 * at each function.  The out-of-table rules for T below chi_min / above
 * chi_max and the QS extrapolation below the first CDF knot are this
 * library's reading; each is pinned against the exact integral it continues
 * (tests/test_oracle_statistics.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <quadmath.h>
#include <omp.h>

/* ------------------------------------------------------------------------ */
/* Constants (CODATA 2018), paper Sec. 2: E_s = m_e^2 c^3 / (q_e hbar).     */
/* ------------------------------------------------------------------------ */
static const double ORC_ME = 9.1093837015e-31;
static const double ORC_C = 299792458.0;
static const double ORC_QE = 1.602176634e-19;
static const double ORC_HBAR = 1.054571817e-34;
static const double ORC_ALPHA = 7.2973525693e-3;

double orc_schwinger_field(void) {
    return ORC_ME * ORC_ME * ORC_C * ORC_C * ORC_C / (ORC_QE * ORC_HBAR);
}
/* alpha m_e c^2 / hbar, the prefactor of both total rates (Sec. 2.1, 2.2). */
double orc_rate_prefactor(void) {
    return ORC_ALPHA * ORC_ME * ORC_C * ORC_C / ORC_HBAR;
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11).                                    */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1): u = (2 m + 1) 2^-53 with m the top 52 bits of the word.
 * Exactly representable, never 0 or 1, and 1 - u is exact. */
double orc_u01(uint64_t w) {
    return (double)(2 * (w >> 12) + 1) * 0x1.0p-53;
}

/* The draw block of particle `id` at `step`: key (seed, 0),
 * counter (id, step, species, block). */
void orc_draws(uint64_t seed, uint64_t id, uint64_t step, uint64_t species,
               uint64_t block, double u[4]) {
    uint64_t ctr[4] = {id, step, species, block}, key[2] = {seed, 0}, w[4];
    orc_philox4x64_10(ctr, key, w);
    for (int k = 0; k < 4; ++k) u[k] = orc_u01(w[k]);
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n.              */
/* ------------------------------------------------------------------------ */
#define ORC_GL_T 16      /* nodes per panel for the Bessel t-integrals   */
#define ORC_GL_X 20      /* nodes per panel for the xi-integrals         */
#define ORC_T_PANELS 24  /* equal panels on [0, t_max]                   */
static double gl_t_x[ORC_GL_T], gl_t_w[ORC_GL_T];
static double gl_x_x[ORC_GL_X], gl_x_w[ORC_GL_X];

static void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p2 = p1; p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute derivative at the converged node */
        double p0 = 1.0, p1 = 0.0;
        for (int j = 1; j <= n; ++j) {
            double p2 = p1; p1 = p0;
            p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

__attribute__((constructor)) static void orc_init_rules(void) {
    gauss_legendre(ORC_GL_T, gl_t_x, gl_t_w);
    gauss_legendre(ORC_GL_X, gl_x_x, gl_x_w);
}

/* ------------------------------------------------------------------------ */
/* Bessel functions from their integral representation (DLMF 10.32.9):      */
/*   e^x K_nu(x)  = int_0^inf exp(-2 x sinh^2(t/2)) cosh(nu t) dt           */
/*   e^x IK_nu(x) = int_0^inf exp(-2 x sinh^2(t/2)) cosh(nu t)/cosh(t) dt   */
/* where IK_nu(x) = int_x^inf K_nu(s) ds.  exp(-x cosh t) = e^-x            */
/* exp(-2 x sinh^2(t/2)) removes the cancellation in cosh t - 1.            */
/* The t range is cut where 2 x sinh^2(t/2) >= 60 + 2 t, beyond which the   */
/* integrand is below e^-60 of its value scale for all nu <= 2.             */
/* ------------------------------------------------------------------------ */
static double t_upper(double x) {
    double lo = 0.0, hi = 1.0;
    while (2.0 * x * pow(sinh(0.5 * hi), 2) < 60.0 + 2.0 * hi) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (2.0 * x * pow(sinh(0.5 * mid), 2) < 60.0 + 2.0 * mid) lo = mid; else hi = mid;
        if (hi - lo < 1e-12 * hi) break;
    }
    return hi;
}

/* Scaled pair: ek = e^x K_{nu_k}(x), eik = e^x IK_{nu_ik}(x). */
void orc_bessel_pair_scaled(double x, double nu_k, double nu_ik, double* ek, double* eik) {
    double tmax = t_upper(x), h = tmax / ORC_T_PANELS, sk = 0.0, sik = 0.0;
    for (int p = 0; p < ORC_T_PANELS; ++p) {
        double a = p * h, mid = a + 0.5 * h;
        for (int i = 0; i < ORC_GL_T; ++i) {
            double t = mid + 0.5 * h * gl_t_x[i], wt = 0.5 * h * gl_t_w[i];
            double sh = sinh(0.5 * t);
            double e = exp(-2.0 * x * sh * sh);
            sk += wt * e * cosh(nu_k * t);
            sik += wt * e * cosh(nu_ik * t) / cosh(t);
        }
    }
    *ek = sk;
    *eik = sik;
}

double orc_bessel_k(double nu, double x) {
    double ek, eik;
    orc_bessel_pair_scaled(x, nu, nu, &ek, &eik);
    return ek * exp(-x);
}

double orc_bessel_ik(double nu, double x) {
    double ek, eik;
    orc_bessel_pair_scaled(x, nu, nu, &ek, &eik);
    return eik * exp(-x);
}

/* ------------------------------------------------------------------------ */
/* Table integrands.                                                        */
/*                                                                          */
/* BW (Sec. 2.1).  With u = chi_gamma xi and the exact substitution         */
/* w = (2/3) s^{3/2} in int_X^inf sqrt(s) K_{1/3}((2/3) s^{3/2}) ds, the    */
/* bracket of T(chi_gamma) becomes                                          */
/*   B(xi) = IK_{1/3}(z) + (1/(xi(1-xi)) - 2) K_{2/3}(z),                   */
/*   z = 2 / (3 chi_gamma xi (1 - xi)),                                     */
/* so T(chi_gamma) = (1/(pi sqrt3 chi_gamma)) int_0^1 B(xi) dxi and the     */
/* pair CDF is int_0^xi B / int_0^1 B.  z >= z0 = 8/(3 chi_gamma); the      */
/* integrand is kept scaled by e^{z0}: Bs = e^{-(z - z0)} (e^z IK + ...),    */
/* with z - z0 = (2/(3 chi)) (1 - 2 xi)^2 / (xi (1 - xi)).                   */
/*                                                                          */
/* QS (Sec. 2.2).  G(chi) = int_0^1 S(chi, xi)/xi dxi with                  */
/*   S/xi = (sqrt3/(2 pi)) [IK_{5/3}(Y) + xi^2/(1-xi) K_{2/3}(Y)],          */
/*   Y = 2 xi / (3 chi (1 - xi)).                                           */
/* The photon CDF is taken number-weighted, int_0^xi S/u du / int_0^1 S/u du,*/
/* i.e. the normalised integral of the differential rate d2N/dt dchi_gamma. */
/* The printed CDF omits the 1/u; read as a slip because its denominator    */
/* would then differ from G(chi), which normalises that rate.               */
/* ------------------------------------------------------------------------ */
static double bw_integrand_scaled(double chi, double xi) {
    double q = xi * (1.0 - xi);
    if (q <= 0.0) return 0.0;
    double d = (2.0 / (3.0 * chi)) * (1.0 - 2.0 * xi) * (1.0 - 2.0 * xi) / q;
    if (d > 745.0) return 0.0;
    double z = 2.0 / (3.0 * chi * q), ek, eik;
    orc_bessel_pair_scaled(z, 2.0 / 3.0, 1.0 / 3.0, &ek, &eik);
    return exp(-d) * (eik + (1.0 / q - 2.0) * ek);
}

static double qs_integrand(double chi, double xi) {
    if (xi >= 1.0) return 0.0;
    double y = 2.0 * xi / (3.0 * chi * (1.0 - xi));
    if (y > 745.0) return 0.0;
    double ek, eik;
    orc_bessel_pair_scaled(y, 2.0 / 3.0, 5.0 / 3.0, &ek, &eik);
    return exp(-y) * (eik + xi * xi / (1.0 - xi) * ek);
}

/* Local length scale of each integrand in xi, used to size GL panels.
 * BW: the scaled integrand is exp(-g(xi)) times smooth factors, g as above;
 * near xi = 1/2 it is a Gaussian of width sigma = sqrt(3 chi)/8, further
 * out it falls on the scale 1/|g'|.  QS: exp(-Y) falls on 1/Y', and the
 * power-law behaviour near 0 and the 1/(1-xi) growth near 1 need panels
 * no wider than a fraction of the distance to the end point. */
static double bw_panel(double chi, double xi) {
    double sigma = sqrt(3.0 * chi) / 8.0;
    double gp = (2.0 / (3.0 * chi)) * fabs(1.0 - 2.0 * xi) / (xi * xi * (1.0 - xi) * (1.0 - xi));
    double h = 0.5 * xi;
    if (1.0 / 32.0 < h) h = 1.0 / 32.0;
    if (sigma < h) h = sigma;
    if (gp > 0.0 && 2.0 / gp < h) h = 2.0 / gp;
    return h;
}

static double qs_panel(double chi, double xi) {
    double yp = (2.0 / (3.0 * chi)) / ((1.0 - xi) * (1.0 - xi));
    double h = 0.5 * xi;
    if (0.5 * (1.0 - xi) < h) h = 0.5 * (1.0 - xi);
    if (2.0 / yp < h) h = 2.0 / yp;
    return h;
}

static double gl_panel(double (*f)(double, double), double chi, double a, double b) {
    double mid = 0.5 * (a + b), half = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < ORC_GL_X; ++i) s += gl_x_w[i] * f(chi, mid + half * gl_x_x[i]);
    return s * half;
}

/* int_a^b f over panels no wider than the local scale. */
static double integrate_walk(double (*f)(double, double), double (*scale)(double, double),
                             double chi, double a, double b) {
    double s = 0.0, x = a;
    while (x < b) {
        double h = scale(chi, x);
        double y = (x + h < b) ? x + h : b;
        if (y <= x) break;
        s += gl_panel(f, chi, x, y);
        x = y;
    }
    return s;
}

/* One BW row at chi: cumulative integrals at the knots xi_m = 0.5 m/(N-1)
 * (Sec. 3.1), returning int_0^1 Bs = 2 int_0^{1/2} Bs (symmetry of the
 * integrand under xi -> 1 - xi).  cum[m] = int_0^{xi_m} Bs. */
static double bw_row(double chi, int n_frac, double* cum) {
    /* below xi_lo, g(xi) > 745 and the scaled integrand is below e^-745. */
    double q_lo = 1.0 / (4.0 + 745.0 * 1.5 * chi);
    double xi_lo = 0.5 * (1.0 - sqrt(1.0 - 4.0 * q_lo));
    double s = 0.0;
    cum[0] = 0.0;
    for (int m = 1; m < n_frac; ++m) {
        double a = 0.5 * (double)(m - 1) / (double)(n_frac - 1);
        double b = 0.5 * (double)m / (double)(n_frac - 1);
        if (b > xi_lo) s += integrate_walk(bw_integrand_scaled, bw_panel, chi, a > xi_lo ? a : xi_lo, b);
        cum[m] = s;
    }
    return 2.0 * s;
}

/* One QS row at chi: knots ln xi_m = ln xi_min (1 - m/(N-1)) (Sec. 3.2).
 * cum[m] = int_0^{xi_m} of the bracket; returns int_0^1.  On [0, xi_min]
 * the integrand grows like xi^{-2/3}; xi = xi_min s^3 makes it smooth. */
static double qs_row(double chi, int n_frac, double frac_min, double* cum) {
    double s0 = 0.0;
    /* int_0^{xi_min} f(xi) dxi = int_0^1 f(xi_min s^3) 3 xi_min s^2 ds, two panels */
    for (int p = 0; p < 2; ++p) {
        double a = 0.5 * p, mid = a + 0.25, half = 0.25;
        for (int i = 0; i < ORC_GL_X; ++i) {
            double sv = mid + half * gl_x_x[i];
            double xi = frac_min * sv * sv * sv;
            s0 += gl_x_w[i] * half * qs_integrand(chi, xi) * 3.0 * frac_min * sv * sv;
        }
    }
    double s = s0;
    double lmin = log(frac_min);
    cum[0] = s;
    /* beyond xi_hi, Y > 745 and the integrand vanishes to double precision */
    double xi_hi = 745.0 * 1.5 * chi / (1.0 + 745.0 * 1.5 * chi);
    double prev = frac_min;
    for (int m = 1; m < n_frac; ++m) {
        double b = (m == n_frac - 1) ? 1.0 : exp(lmin * (1.0 - (double)m / (double)(n_frac - 1)));
        double a = prev;
        double bb = b < xi_hi ? b : xi_hi;
        if (bb > a) s += integrate_walk(qs_integrand, qs_panel, chi, a, bb);
        cum[m] = s;
        prev = b;
    }
    cum[n_frac - 1] = s;
    return s;
}

/* ------------------------------------------------------------------------ */
/* Table object.                                                            */
/* ------------------------------------------------------------------------ */
enum { ORC_BW = 0, ORC_QS = 1 };

typedef struct {
    int proc;             /* ORC_BW or ORC_QS */
    int n_chi, n_frac;
    double chi_min, chi_max, frac_min;
    double* ln_rate;      /* [n_chi]: ln T (BW) or ln G (QS) */
    double* cdf;          /* [n_chi][n_frac]: P (BW) or ln P (QS) */
} orc_table;

/* One row of both tables at an arbitrary chi (used for row checks). */
void orc_table_row(int proc, double chi, int n_frac, double frac_min,
                   double* ln_rate, double* cdf_row) {
    double* cum = (double*)malloc(sizeof(double) * n_frac);
    if (proc == ORC_BW) {
        double tot = bw_row(chi, n_frac, cum);
        double z0 = 8.0 / (3.0 * chi);
        /* ln T = ln(int Bs) - z0 - ln(pi sqrt3 chi) */
        *ln_rate = log(tot) - z0 - log(M_PI * sqrt(3.0) * chi);
        for (int m = 0; m < n_frac; ++m) cdf_row[m] = cum[m] / tot;
        cdf_row[n_frac - 1] = 0.5;
    } else {
        double tot = qs_row(chi, n_frac, frac_min, cum);
        *ln_rate = log(sqrt(3.0) / (2.0 * M_PI) * tot);
        for (int m = 0; m < n_frac; ++m) cdf_row[m] = log(cum[m] / tot);
        cdf_row[n_frac - 1] = 0.0;
    }
    free(cum);
}

/* chi grid: ln chi_n = ln chi_min + n (ln chi_max - ln chi_min)/(N-1). */
double orc_grid_chi(double chi_min, double chi_max, int n_chi, int n) {
    double l0 = log(chi_min), l1 = log(chi_max);
    return exp(l0 + (double)n * (l1 - l0) / (double)(n_chi - 1));
}

/* Fill ln_rate[n_chi] and cdf[n_chi * n_frac] (row-major in chi). */
void orc_table_generate(int proc, double chi_min, double chi_max, int n_chi, int n_frac,
                        double frac_min, double* ln_rate, double* cdf) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < n_chi; ++n) {
        double chi = orc_grid_chi(chi_min, chi_max, n_chi, n);
        orc_table_row(proc, chi, n_frac, frac_min, &ln_rate[n], &cdf[(size_t)n * n_frac]);
    }
}

/* Single-point values of T(chi) and G(chi) (for pins). */
double orc_bw_T(double chi) {
    double lr, row[3];
    orc_table_row(ORC_BW, chi, 3, 0.0, &lr, row);
    return exp(lr);
}
double orc_qs_G(double chi) {
    double lr, row[3];
    orc_table_row(ORC_QS, chi, 3, 1e-12, &lr, row);
    return exp(lr);
}
/* CDFs at an arbitrary xi (for pins): BW P(chi, xi) for xi in [0, 1/2]; QS P(chi, xi). */
double orc_bw_cdf_at(double chi, double xi) {
    double tot = 0.0, part;
    double row_cum[65];
    tot = bw_row(chi, 65, row_cum);
    part = 0.0;
    double q_lo = 1.0 / (4.0 + 745.0 * 1.5 * chi);
    double xi_lo = 0.5 * (1.0 - sqrt(1.0 - 4.0 * q_lo));
    if (xi > xi_lo) part = integrate_walk(bw_integrand_scaled, bw_panel, chi, xi_lo, xi);
    return part / tot;
}
double orc_qs_cdf_at(double chi, double xi) {
    double cum[65];
    double tot = qs_row(chi, 65, 1e-12, cum);
    double part = cum[0];
    double xi_hi = 745.0 * 1.5 * chi / (1.0 + 745.0 * 1.5 * chi);
    if (xi < 1e-12) return NAN;
    double b = xi < xi_hi ? xi : xi_hi;
    if (b > 1e-12) part += integrate_walk(qs_integrand, qs_panel, chi, 1e-12, b);
    return part / tot;
}

/* ------------------------------------------------------------------------ */
/* Quantum parameter (Sec. 2): chi = (gamma/E_s) sqrt((E + v x B)^2 -       */
/* (v.E/c)^2).  With u = p/(m_e c), v = c u/gamma, so gamma (E + v x B) =   */
/* gamma E + c u x B and gamma v.E/c = u.E.  Splitting E = E_par n + E_perp */
/* along n = u/|u| gives gamma E + c u x B = gamma E_par n + a with         */
/* a = gamma E_perp + c u x B perpendicular to n, hence                     */
/*   (chi E_s)^2 = |a|^2 + (gamma^2 - |u|^2) E_par^2,                       */
/* with gamma^2 - |u|^2 = 1 for leptons and 0 for photons (gamma = |u|).    */
/* This is the same quantity without subtracting two O(gamma^2 E^2) terms.  */
/* ------------------------------------------------------------------------ */
static double chi_common(const double u[3], const double e[3], const double b[3], int photon) {
    double es = orc_schwinger_field();
    double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double um = sqrt(u2);
    if (um == 0.0) {
        if (photon) return 0.0;
        return sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) / es;
    }
    double gamma = photon ? um : sqrt(1.0 + u2);
    double n[3] = {u[0] / um, u[1] / um, u[2] / um};
    double epar = e[0] * n[0] + e[1] * n[1] + e[2] * n[2];
    double uxb[3] = {u[1] * b[2] - u[2] * b[1], u[2] * b[0] - u[0] * b[2], u[0] * b[1] - u[1] * b[0]};
    double a[3];
    for (int k = 0; k < 3; ++k) a[k] = gamma * (e[k] - epar * n[k]) + ORC_C * uxb[k];
    double s = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    if (!photon) s += epar * epar;
    return sqrt(s) / es;
}

double orc_chi_lepton(double ux, double uy, double uz, double ex, double ey, double ez,
                      double bx, double by, double bz) {
    double u[3] = {ux, uy, uz}, e[3] = {ex, ey, ez}, b[3] = {bx, by, bz};
    return chi_common(u, e, b, 0);
}
double orc_chi_photon(double ux, double uy, double uz, double ex, double ey, double ez,
                      double bx, double by, double bz) {
    double u[3] = {ux, uy, uz}, e[3] = {ex, ey, ez}, b[3] = {bx, by, bz};
    return chi_common(u, e, b, 1);
}

/* The paper's formula taken literally, in binary128, for pins. */
double orc_chi_literal_q(double ux, double uy, double uz, double ex, double ey, double ez,
                         double bx, double by, double bz, int photon) {
    __float128 c = ORC_C, es = (__float128)ORC_ME * ORC_ME * c * c * c / ((__float128)ORC_QE * ORC_HBAR);
    __float128 u[3] = {ux, uy, uz}, e[3] = {ex, ey, ez}, b[3] = {bx, by, bz};
    __float128 u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    __float128 gamma = photon ? sqrtq(u2) : sqrtq(1 + u2);
    if (gamma == 0) return 0.0;
    __float128 v[3] = {c * u[0] / gamma, c * u[1] / gamma, c * u[2] / gamma};
    __float128 f[3] = {e[0] + v[1] * b[2] - v[2] * b[1], e[1] + v[2] * b[0] - v[0] * b[2],
                       e[2] + v[0] * b[1] - v[1] * b[0]};
    __float128 ve = (v[0] * e[0] + v[1] * e[1] + v[2] * e[2]) / c;
    __float128 s = f[0] * f[0] + f[1] * f[1] + f[2] * f[2] - ve * ve;
    if (s < 0) s = 0;
    return (double)(gamma / es * sqrtq(s));
}

/* ------------------------------------------------------------------------ */
/* Runtime: rates (Sec. 2.1 total BW rate, Sec. 2.2 total QS rate) with the */
/* table interpolation of Sec. 3.1 / 3.2: find chi_n <= chi < chi_{n+1} and */
/* interpolate ln T (ln G) linearly in ln chi.                              */
/* ------------------------------------------------------------------------ */
static double interp_ln(const orc_table* t, const double* y, double chi) {
    double l0 = log(t->chi_min), l1 = log(t->chi_max);
    double d = (l1 - l0) / (double)(t->n_chi - 1);
    double lc = log(chi);
    int n = (int)floor((lc - l0) / d);
    if (n < 0) n = 0;
    if (n > t->n_chi - 2) n = t->n_chi - 2;
    double ln_n = l0 + n * d, ln_n1 = l0 + (n + 1) * d;
    return y[n] + (lc - ln_n) * (y[n + 1] - y[n]) / (ln_n1 - ln_n);
}

/* BW: dN/dt = (alpha m c^2/hbar) (chi_gamma/gamma_gamma) T(chi_gamma).
 * Outside the table the paper uses the asymptotic forms of T; the printed
 * forms are garbled, so the asymptotes of the integral definition are used,
 * matched to the table edge: T ~ exp(-8/(3 chi)) below chi_min and
 * T ~ chi^{-1/3} above chi_max. */
double orc_rate_bw(const orc_table* t, double chi, double gamma_g) {
    if (!(chi > 0.0) || !(gamma_g > 0.0)) return 0.0;
    double lnT;
    if (chi < t->chi_min)
        lnT = t->ln_rate[0] - (8.0 / 3.0) * (1.0 / chi - 1.0 / t->chi_min);
    else if (chi > t->chi_max)
        lnT = t->ln_rate[t->n_chi - 1] - (1.0 / 3.0) * (log(chi) - log(t->chi_max));
    else
        lnT = interp_ln(t, t->ln_rate, chi);
    return orc_rate_prefactor() * (chi / gamma_g) * exp(lnT);
}

/* QS: dN/dt = (2/3)(alpha m c^2/hbar)(1/gamma) G(chi); outside the table the
 * first or last stored value is used (Sec. 3.2), including chi = 0. */
double orc_rate_qs(const orc_table* t, double chi, double gamma) {
    double lnG;
    if (!(chi >= t->chi_min)) lnG = t->ln_rate[0];
    else if (chi > t->chi_max) lnG = t->ln_rate[t->n_chi - 1];
    else lnG = interp_ln(t, t->ln_rate, chi);
    return (2.0 / 3.0) * orc_rate_prefactor() * exp(lnG) / gamma;
}

/* Row interpolation setup for the 2D tables: chi clamped to the table range
 * (Sec. 3.1, 3.2), then n and the weight (ln chi - ln chi_n)/(ln chi_{n+1} -
 * ln chi_n). */
static void row_weight(const orc_table* t, double chi, int* n_out, double* f_out) {
    double c = chi;
    if (!(c >= t->chi_min)) c = t->chi_min;
    if (c > t->chi_max) c = t->chi_max;
    double l0 = log(t->chi_min), l1 = log(t->chi_max);
    double d = (l1 - l0) / (double)(t->n_chi - 1);
    double lc = log(c);
    int n = (int)floor((lc - l0) / d);
    if (n < 0) n = 0;
    if (n > t->n_chi - 2) n = t->n_chi - 2;
    double ln_n = l0 + n * d, ln_n1 = l0 + (n + 1) * d;
    *n_out = n;
    *f_out = (lc - ln_n) / (ln_n1 - ln_n);
}

/* BW pair sampling (Sec. 3.1).  r <= 1/2: the sampled fraction belongs to
 * the electron; otherwise r -> 1 - r and it belongs to the positron.  The
 * interpolated column values are searched for the largest m with
 * P_m <= r (so P_m <= r < P_{m+1}); then xi is interpolated linearly.
 * Returns xi in [0, 1/2]; *electron_selected tells who gets it. */
double orc_sample_bw(const orc_table* t, double chi, double r, int* electron_selected) {
    int n; double f;
    row_weight(t, chi, &n, &f);
    *electron_selected = (r <= 0.5);
    if (r > 0.5) r = 1.0 - r;
    const double* p0 = t->cdf + (size_t)n * t->n_frac;
    const double* p1 = p0 + t->n_frac;
    int N = t->n_frac;
    double* P = (double*)malloc(sizeof(double) * N);
    for (int m = 0; m < N; ++m) P[m] = p0[m] + f * (p1[m] - p0[m]);
    int lo = 0, hi = N - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (P[mid] <= r) lo = mid; else hi = mid;
    }
    double xa = 0.5 * (double)lo / (double)(N - 1), xb = 0.5 * (double)(lo + 1) / (double)(N - 1);
    double xi = xa + (r - P[lo]) * (xb - xa) / (P[lo + 1] - P[lo]);
    free(P);
    return xi;
}

/* QS photon sampling (Sec. 3.2): interpolated ln P_m, search for
 * ln P_m <= ln r < ln P_{m+1}, log-log interpolation of xi.  Below the first
 * knot (ln r < ln P_0) the small-xi law P ~ xi^{1/3} of the spectrum is
 * continued: ln xi = ln xi_min + 3 (ln r - ln P_0).  Returns ln xi. */
double orc_sample_qs_lnxi(const orc_table* t, double chi, double r) {
    int n; double f;
    row_weight(t, chi, &n, &f);
    int N = t->n_frac;
    const double* p0 = t->cdf + (size_t)n * N;
    const double* p1 = p0 + N;
    double* L = (double*)malloc(sizeof(double) * N);
    for (int m = 0; m < N; ++m) L[m] = p0[m] + f * (p1[m] - p0[m]);
    double lr = log(r), lmin = log(t->frac_min), out;
    if (lr < L[0]) {
        out = lmin + 3.0 * (lr - L[0]);
    } else {
        int lo = 0, hi = N - 1;
        while (hi - lo > 1) {
            int mid = (lo + hi) / 2;
            if (L[mid] <= lr) lo = mid; else hi = mid;
        }
        double la = lmin * (1.0 - (double)lo / (double)(N - 1));
        double lb = lmin * (1.0 - (double)(lo + 1) / (double)(N - 1));
        out = la + (lr - L[lo]) * (lb - la) / (L[lo + 1] - L[lo]);
    }
    free(L);
    return out;
}

/* ------------------------------------------------------------------------ */
/* The per-timestep QED sub-step (Fig. 1 caption, Sec. 3 introduction):     */
/* tau <- tau - (dN/dt) dt; an event happens when tau becomes negative      */
/* (strictly); at most one event per particle per step; the parent's tau    */
/* is redrawn as -ln u without carrying the negative remainder.            */
/* Draw block 0 of (seed; id, step, species): u0 -> sampling, u1 -> new tau */
/* of the parent (QS) or of the electron (BW), u2 -> tau of the new photon  */
/* (QS) or of the positron (BW).                                            */
/*                                                                          */
/* Kinematics (Sec. 2.1, 2.2, ultra-relativistic: products collinear with   */
/* the parent).  QS: gamma_gamma = (gamma - 1) xi along n = u/|u|; the      */
/* parent momentum becomes u - gamma_gamma n (momentum conserved exactly).  */
/* BW: the selected product takes xi u_gamma and the other u_gamma - xi     */
/* u_gamma; the photon is marked dead with tau = +inf.  The paper's energy  */
/* form K = (gamma_gamma - 2) chi_pm/chi_gamma is not used: with massive    */
/* collinear products it cannot conserve momentum exactly.                  */
/* ------------------------------------------------------------------------ */
enum { ORC_ELECTRON = 0, ORC_POSITRON = 1, ORC_PHOTON = 2, ORC_ION = 3 };
#define ORC_INIT_STEP 0xFFFFFFFFFFFFFFFFULL

typedef struct {
    double *ux, *uy, *uz, *ex, *ey, *ez, *bx, *by, *bz, *tau, *w;
    int64_t n, id_base;
    int32_t species;
} orc_particles;

typedef struct {
    double *ux, *uy, *uz, *w, *tau;
    int64_t* parent;
    int64_t capacity;
    int64_t count;
} orc_append;

void orc_init_optical_depth(orc_particles* p, uint64_t seed) {
    for (int64_t i = 0; i < p->n; ++i) {
        double u[4];
        orc_draws(seed, (uint64_t)(p->id_base + i), ORC_INIT_STEP, (uint64_t)p->species, 0, u);
        p->tau[i] = -log(u[0]);
    }
}

static void put(orc_append* a, int64_t slot, double ux, double uy, double uz, double w, double tau,
                int64_t parent) {
    if (slot >= a->capacity) return;
    a->ux[slot] = ux; a->uy[slot] = uy; a->uz[slot] = uz;
    a->w[slot] = w; a->tau[slot] = tau; a->parent[slot] = parent;
}

typedef struct {
    int nprod;          /* 0, 1 (QS photon) or 2 (BW pair) */
    double pa[5], pb[5];  /* product records: ux uy uz w tau */
} orc_event_out;

/* Classical radiation below the QED threshold (Sec. 6: below a minimum
 * quantum parameter pair production is ignored and photon emission is
 * treated classically).  The classical model taken here is the radiation
 * drag of the ultra-relativistic Landau-Lifshitz force: the particle loses
 * the energy radiated classically, P = (2/3) (alpha m c^2/hbar) chi^2 m c^2,
 * along its direction of motion over dt; gamma' = max(1, gamma - dgamma),
 * u' = u sqrt(gamma'^2 - 1)/|u|. */
static void classical_drag(double u[3], double chi, double dt) {
    double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (!(u2 > 0.0)) return;
    double gamma = sqrt(1.0 + u2);
    double dg = (2.0 / 3.0) * orc_rate_prefactor() * chi * chi * dt;
    double gp = gamma - dg;
    double sc = gp > 1.0 ? sqrt((gp - 1.0) * (gp + 1.0)) / sqrt(u2) : 0.0;
    u[0] *= sc; u[1] *= sc; u[2] *= sc;
}

/* Evolve one particle; returns 1 on an event.  Products go to *ev.  With
 * chi_qed_min > 0, a particle whose chi is below it keeps its optical depth:
 * photons do nothing, leptons take the classical drag instead. */
static int step_one(const orc_table* bw, const orc_table* qs, orc_particles* p, int64_t i,
                    double dt, uint64_t seed, uint64_t step, double photon_min_energy,
                    double chi_qed_min, orc_event_out* ev) {
    int photon = (p->species == ORC_PHOTON);
    double u[3] = {p->ux[i], p->uy[i], p->uz[i]};
    double e[3] = {p->ex[i], p->ey[i], p->ez[i]};
    double b[3] = {p->bx[i], p->by[i], p->bz[i]};
    double chi = chi_common(u, e, b, photon);
    double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double um = sqrt(u2);
    double gamma = photon ? um : sqrt(1.0 + u2);
    ev->nprod = 0;
    if (chi_qed_min > 0.0 && chi < chi_qed_min) {
        if (!photon) {
            classical_drag(u, chi, dt);
            p->ux[i] = u[0]; p->uy[i] = u[1]; p->uz[i] = u[2];
        }
        return 0;
    }
    double rate = photon ? orc_rate_bw(bw, chi, gamma) : orc_rate_qs(qs, chi, gamma);
    double tau = p->tau[i] - rate * dt;
    if (!(tau < 0.0)) {
        p->tau[i] = tau;
        return 0;
    }
    double d[4];
    orc_draws(seed, (uint64_t)(p->id_base + i), step, (uint64_t)p->species, 0, d);
    if (photon) {
        int esel;
        double xi = orc_sample_bw(bw, chi, d[0], &esel);
        double sel[3] = {xi * u[0], xi * u[1], xi * u[2]};
        double oth[3] = {u[0] - sel[0], u[1] - sel[1], u[2] - sel[2]};
        const double* pe = esel ? sel : oth;
        const double* pp = esel ? oth : sel;
        double w = p->w[i];
        double ea[5] = {pe[0], pe[1], pe[2], w, -log(d[1])};
        double pa[5] = {pp[0], pp[1], pp[2], w, -log(d[2])};
        memcpy(ev->pa, ea, sizeof ea);
        memcpy(ev->pb, pa, sizeof pa);
        ev->nprod = 2;
        p->tau[i] = INFINITY;
    } else {
        double lnxi = orc_sample_qs_lnxi(qs, chi, d[0]);
        double xi = exp(lnxi);
        /* gamma - 1 written as |u|^2/(gamma + 1), the same number without
         * cancellation for slow particles */
        double gg = (u2 / (gamma + 1.0)) * xi;
        double pg[3] = {0.0, 0.0, 0.0};
        if (um > 0.0) { pg[0] = gg * u[0] / um; pg[1] = gg * u[1] / um; pg[2] = gg * u[2] / um; }
        p->ux[i] = u[0] - pg[0];
        p->uy[i] = u[1] - pg[1];
        p->uz[i] = u[2] - pg[2];
        p->tau[i] = -log(d[1]);
        if (gg >= photon_min_energy) {
            double ph[5] = {pg[0], pg[1], pg[2], p->w[i], -log(d[2])};
            memcpy(ev->pa, ph, sizeof ph);
            ev->nprod = 1;
        }
    }
    return 1;
}

/* One step for one species, particles in index order.  Leptons append
 * photons to a1; photons append electrons to a1 and positrons to a2 at the
 * same slot.  Products beyond capacity are dropped; count always holds the
 * total required.  flags (nullable) receives 1 for an event, else 0. */
int64_t orc_step(const orc_table* bw, const orc_table* qs, orc_particles* p, double dt,
                 uint64_t seed, uint64_t step, double photon_min_energy, double chi_qed_min, uint8_t* flags,
                 orc_append* a1, orc_append* a2) {
    orc_event_out* ev = (orc_event_out*)malloc(sizeof(orc_event_out) * (size_t)(p->n > 0 ? p->n : 1));
    int64_t events = 0;
#pragma omp parallel for reduction(+ : events) schedule(static)
    for (int64_t i = 0; i < p->n; ++i) {
        int e = step_one(bw, qs, p, i, dt, seed, step, photon_min_energy, chi_qed_min, &ev[i]);
        if (flags) flags[i] = (uint8_t)e;
        events += e;
    }
    /* sequential, parent-ordered append */
    for (int64_t i = 0; i < p->n; ++i) {
        if (ev[i].nprod == 0) continue;
        int64_t parent = p->id_base + i;
        if (ev[i].nprod == 1) {
            put(a1, a1->count, ev[i].pa[0], ev[i].pa[1], ev[i].pa[2], ev[i].pa[3], ev[i].pa[4], parent);
            a1->count += 1;
        } else {
            put(a1, a1->count, ev[i].pa[0], ev[i].pa[1], ev[i].pa[2], ev[i].pa[3], ev[i].pa[4], parent);
            put(a2, a2->count, ev[i].pb[0], ev[i].pb[1], ev[i].pb[2], ev[i].pb[3], ev[i].pb[4], parent);
            a1->count += 1;
            a2->count += 1;
        }
    }
    free(ev);
    return events;
}

/* Product generation for already-flagged particles (the paper's pair
 * production and photon emission kernels, Sec. 4): every flagged particle
 * undergoes an event, sequential append in index order. */
int64_t orc_generate(const orc_table* bw, const orc_table* qs, orc_particles* p,
                     const uint8_t* flags, uint64_t seed, uint64_t step,
                     double photon_min_energy, orc_append* a1, orc_append* a2) {
    int64_t events = 0;
    for (int64_t i = 0; i < p->n; ++i) {
        if (!flags[i]) continue;
        p->tau[i] = -1.0;   /* forces the event branch with rate*dt = 0 */
        orc_event_out ev;
        step_one(bw, qs, p, i, 0.0, seed, step, photon_min_energy, 0.0, &ev);
        int64_t parent = p->id_base + i;
        if (ev.nprod == 1) {
            put(a1, a1->count, ev.pa[0], ev.pa[1], ev.pa[2], ev.pa[3], ev.pa[4], parent);
            a1->count += 1;
        } else if (ev.nprod == 2) {
            put(a1, a1->count, ev.pa[0], ev.pa[1], ev.pa[2], ev.pa[3], ev.pa[4], parent);
            put(a2, a2->count, ev.pb[0], ev.pb[1], ev.pb[2], ev.pb[3], ev.pb[4], parent);
            a1->count += 1;
            a2->count += 1;
        }
        ++events;
    }
    return events;
}

/* Optical-depth evolution only (the paper's evolution kernels, Sec. 4):
 * tau <- tau - rate dt and flags[i] = (tau < 0), no products. */
void orc_evolve(const orc_table* t, orc_particles* p, double dt, uint8_t* flags) {
    int photon = (p->species == ORC_PHOTON);
    for (int64_t i = 0; i < p->n; ++i) {
        double u[3] = {p->ux[i], p->uy[i], p->uz[i]};
        double e[3] = {p->ex[i], p->ey[i], p->ez[i]};
        double b[3] = {p->bx[i], p->by[i], p->bz[i]};
        double chi = chi_common(u, e, b, photon);
        double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double gamma = photon ? sqrt(u2) : sqrt(1.0 + u2);
        double rate = photon ? orc_rate_bw(t, chi, gamma) : orc_rate_qs(t, chi, gamma);
        p->tau[i] -= rate * dt;
        if (flags) flags[i] = (uint8_t)(p->tau[i] < 0.0);
    }
}

/* ------------------------------------------------------------------------ */
/* Batch forms of the scalar functions above (loops, for the tests).        */
/* ------------------------------------------------------------------------ */
void orc_chi_n(int64_t n, const double* ux, const double* uy, const double* uz,
               const double* ex, const double* ey, const double* ez,
               const double* bx, const double* by, const double* bz, int photon, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double u[3] = {ux[i], uy[i], uz[i]}, e[3] = {ex[i], ey[i], ez[i]}, b[3] = {bx[i], by[i], bz[i]};
        out[i] = chi_common(u, e, b, photon);
    }
}

/* binary128 literal chi for n particles (precision studies). */
void orc_chi_literal_q_n(int64_t n, const double* ux, const double* uy, const double* uz,
                         const double* ex, const double* ey, const double* ez,
                         const double* bx, const double* by, const double* bz, int photon, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = orc_chi_literal_q(ux[i], uy[i], uz[i], ex[i], ey[i], ez[i], bx[i], by[i], bz[i], photon);
}

void orc_rate_n(const orc_table* t, int64_t n, const double* chi, const double* gamma, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = (t->proc == ORC_BW) ? orc_rate_bw(t, chi[i], gamma[i]) : orc_rate_qs(t, chi[i], gamma[i]);
}

void orc_sample_n(const orc_table* t, int64_t n, const double* chi, const double* r, double* out,
                  uint8_t* electron_selected) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (t->proc == ORC_BW) {
            int e;
            out[i] = orc_sample_bw(t, chi[i], r[i], &e);
            if (electron_selected) electron_selected[i] = (uint8_t)e;
        } else {
            out[i] = orc_sample_qs_lnxi(t, chi[i], r[i]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* MLP reference for the learned inverse-CDF surrogate (not in the paper:   */
/* the library's learned replacement of the Sec. 3.1 / 3.2 table lookup).   */
/* 2 -> 64 -> 64 -> 1, SiLU, loss 0.5 sum_i w_i (y_i - t_i)^2 / n.          */
/* Parameter layout: W1[64][2], b1[64], W2[64][64] (row = output unit),     */
/* b2[64], W3[64], b3.  FP64 throughout; with `bf16` set, the operands the  */
/* library feeds to its BF16 matrix instructions (W2 and h1 forward; dz2    */
/* and h1 for dW2; dz2 and W2 for dh1) are rounded to bfloat16 first.       */
/* ------------------------------------------------------------------------ */
static double orc_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}
static double orc_silu(double z) { return z / (1.0 + exp(-z)); }
static double orc_dsilu(double z) {
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

#define H 64
double orc_mlp_grad(const double* p, int64_t n, const double* x, const double* t, const double* w, double* grad,
                    double* y_out, int bf16) {
    const double *W1 = p, *b1 = p + 128, *W2 = p + 192, *b2 = p + 192 + 4096, *W3 = p + 192 + 4096 + 64;
    double b3 = p[192 + 4096 + 128];
    if (grad) memset(grad, 0, sizeof(double) * 4417);
    double loss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double z1[H], h1[H], h1q[H], z2[H], h2[H];
        for (int k = 0; k < H; ++k) {
            z1[k] = W1[2 * k] * x[2 * i] + W1[2 * k + 1] * x[2 * i + 1] + b1[k];
            h1[k] = orc_silu(z1[k]);
            h1q[k] = bf16 ? orc_bf16(h1[k]) : h1[k];
        }
        double y = b3;
        for (int j = 0; j < H; ++j) {
            double s = 0.0;
            for (int k = 0; k < H; ++k) s += (bf16 ? orc_bf16(W2[j * H + k]) : W2[j * H + k]) * h1q[k];
            z2[j] = s + b2[j];
            h2[j] = orc_silu(z2[j]);
            y += W3[j] * h2[j];
        }
        if (y_out) y_out[i] = y;
        if (!t || !grad) continue;
        double wi = w ? w[i] : 1.0;
        double r = y - t[i];
        loss += 0.5 * wi * r * r / (double)n;
        double dy = wi * r / (double)n;
        double *gW1 = grad, *gb1 = grad + 128, *gW2 = grad + 192, *gb2 = grad + 192 + 4096, *gW3 = gb2 + 64;
        grad[192 + 4096 + 128] += dy;
        double dz2[H], dz2q[H];
        for (int j = 0; j < H; ++j) {
            gW3[j] += dy * h2[j];
            dz2[j] = dy * W3[j] * orc_dsilu(z2[j]);
            dz2q[j] = bf16 ? orc_bf16(dz2[j]) : dz2[j];
            gb2[j] += dz2[j];
            for (int k = 0; k < H; ++k) gW2[j * H + k] += dz2q[j] * h1q[k];
        }
        for (int k = 0; k < H; ++k) {
            double dh = 0.0;
            for (int j = 0; j < H; ++j) dh += dz2q[j] * (bf16 ? orc_bf16(W2[j * H + k]) : W2[j * H + k]);
            double dz1 = dh * orc_dsilu(z1[k]);
            gW1[2 * k] += dz1 * x[2 * i];
            gW1[2 * k + 1] += dz1 * x[2 * i + 1];
            gb1[k] += dz1;
        }
    }
    return loss;
}
#undef H

/* ------------------------------------------------------------------------ */
/* Sequential ordered compaction: parent ids of the products of one stream  */
/* given per-particle event flags, tiles visited in order (tile = set,      */
/* begin, end), particles in index order inside a tile.  `set_stream[s]`   */
/* tells which product stream set s feeds (0 leptons, 1 photons, -1 none).  */
/* Returns the number of parents written (<= cap).                          */
/* ------------------------------------------------------------------------ */
int64_t orc_compact(int64_t n_tiles, const int64_t* tiles, const int32_t* set_stream,
                    const uint8_t* const* flags, const int64_t* id_base, int32_t stream,
                    int64_t* parents, int64_t cap) {
    int64_t k = 0;
    for (int64_t t = 0; t < n_tiles; ++t) {
        int64_t s = tiles[3 * t], b = tiles[3 * t + 1], e = tiles[3 * t + 2];
        if (set_stream[s] != stream) continue;
        for (int64_t i = b; i < e; ++i) {
            if (!flags[s][i]) continue;
            if (k < cap) parents[k] = id_base[s] + i;
            ++k;
        }
    }
    return k;
}

/* ------------------------------------------------------------------------ */
/* Schwinger pair production (Sec. 2.3): rate per unit volume               */
/*   d2N/(dt dV) = q_e^2 E_s^2 / (4 pi^2 hbar^2 c) eps eta coth(pi eta/eps)  */
/*                 exp(-pi/eps),                                            */
/* eps = calE/E_s, eta = calH/E_s, calE = sqrt(sqrt(F^2+G^2) + F),          */
/* calH = sqrt(sqrt(F^2+G^2) - F), F = (E^2 - c^2 B^2)/2, G = c E.B.        */
/* Evaluated as printed, in binary128.  eta coth(pi eta/eps) tends to       */
/* eps/pi as eta -> 0; eps = 0 gives rate 0.                                */
/* ------------------------------------------------------------------------ */
double orc_schwinger_rate(double ex, double ey, double ez, double bx, double by, double bz) {
    const __float128 c = ORC_C, es = (__float128)ORC_ME * ORC_ME * c * c * c / ((__float128)ORC_QE * ORC_HBAR);
    const __float128 pi = M_PIq;
    const __float128 e2 = (__float128)ex * ex + (__float128)ey * ey + (__float128)ez * ez;
    const __float128 b2 = (__float128)bx * bx + (__float128)by * by + (__float128)bz * bz;
    const __float128 F = (e2 - c * c * b2) / 2;
    const __float128 G = c * ((__float128)ex * bx + (__float128)ey * by + (__float128)ez * bz);
    const __float128 s = sqrtq(F * F + G * G);
    const __float128 calE = sqrtq(fmaxq(s + F, 0)), calH = sqrtq(fmaxq(s - F, 0));
    const __float128 eps = calE / es, eta = calH / es;
    if (eps == 0) return 0.0;
    const __float128 pref = (__float128)ORC_QE * ORC_QE * es * es / (4 * pi * pi * (__float128)ORC_HBAR * ORC_HBAR * c);
    const __float128 x = pi * eta / eps;
    const __float128 eta_coth = (x == 0) ? eps / pi : eta / tanhq(x);
    return (double)(pref * eps * eta_coth * expq(-pi / eps));
}

void orc_schwinger_rate_n(int64_t n, const double* ex, const double* ey, const double* ez, const double* bx,
                          const double* by, const double* bz, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = orc_schwinger_rate(ex[i], ey[i], ez[i], bx[i], by[i], bz[i]);
}

/* Macro-pairs created in one cell in one step.  The paper gives the rate and
 * puts the pairs at rest; the count is this library's reading: Poisson with
 * mean lambda = rate dV dt / W (W physical pairs per macro-pair), drawn by
 * inversion with the first uniform of block 0 of the cell's counter
 * (cell id, step, species 4); for lambda > 25 a Gaussian of mean and
 * variance lambda (Box-Muller on the first two uniforms), rounded to the
 * nearest integer and clipped at 0.  `margin` (may be NULL) receives the
 * distance of the deciding uniform from the nearest CDF boundary (Poisson)
 * or of the Gaussian value from the nearest half-integer, so that a test can
 * tell a rounding-level disagreement from a real one. */
int64_t orc_schwinger_count(double lambda, uint64_t seed, uint64_t cell, uint64_t step, double* margin) {
    double u[4];
    orc_draws(seed, cell, step, 4, 0, u);
    if (!(lambda > 0.0)) {
        if (margin) *margin = INFINITY;
        return 0;
    }
    if (lambda <= 25.0) {
        double p = exp(-lambda), cum = p, m = fabs(u[0] - cum);
        int64_t k = 0;
        while (u[0] > cum && k < 1000) {
            ++k;
            p *= lambda / (double)k;
            cum += p;
            if (fabs(u[0] - cum) < m) m = fabs(u[0] - cum);
        }
        if (margin) *margin = m;
        return k;
    }
    const double z = sqrt(-2.0 * log(u[0])) * cos(2.0 * M_PI * u[1]);
    const double v = lambda + sqrt(lambda) * z;
    if (margin) *margin = fabs(v - floor(v) - 0.5);
    if (v < 0.5) return 0;
    return (int64_t)floor(v + 0.5);
}

/* Pairs for n cells, appended in cell order (electron and positron of the
 * same pair share a slot index in their buffers): momentum 0 (at rest),
 * weight W, optical depth -ln u from the pair's own block (cell, step,
 * species 4, block 1 + i/2: uniforms 2(i%2) and 2(i%2)+1 for the electron
 * and the positron of pair i).  Returns the number of pairs. */
int64_t orc_schwinger_pairs(int64_t n, const double* ex, const double* ey, const double* ez, const double* bx,
                            const double* by, const double* bz, int64_t cell_id_base, double dv, double dt,
                            double weight, uint64_t seed, uint64_t step, orc_append* el, orc_append* po) {
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double lam = orc_schwinger_rate(ex[i], ey[i], ez[i], bx[i], by[i], bz[i]) * dv * dt / weight;
        const uint64_t cell = (uint64_t)(cell_id_base + i);
        const int64_t k = orc_schwinger_count(lam, seed, cell, step, NULL);
        for (int64_t q = 0; q < k; ++q) {
            double u[4];
            orc_draws(seed, cell, step, 4, (uint64_t)(1 + q / 2), u);
            const int h = (int)(q % 2);
            put(el, total, 0.0, 0.0, 0.0, weight, -log(u[2 * h]), cell_id_base + i);
            put(po, total, 0.0, 0.0, 0.0, weight, -log(u[2 * h + 1]), cell_id_base + i);
            ++total;
        }
    }
    el->count = total;
    po->count = total;
    return total;
}

/* ------------------------------------------------------------------------ */
/* Particle push in prescribed fields (the Sec. 5.1 benchmark geometries:   */
/* a static B perpendicular to the electrons; a circularly polarised plane  */
/* wave).  Leptons by the relativistic Boris scheme (Boris 1970): half      */
/* electric kick, rotation about B by the angle 2 atan(q B dt/(2 m gamma)), */
/* half kick; positions advanced with the new velocity.  Photons move at c. */
/* After the move the fields at the new position and time are stored in the */
/* particle, as the QED step reads them.                                    */
/*   kind 0: uniform E0, B0.  kind 1: CP wave along dir * x with amplitude  */
/*   A: E = A (0, cos ph, sin ph), B = (dir x_hat) x E / c,                 */
/*   ph = 2 pi (dir x - c t)/lambda + phase.                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind, dir;
    double e0[3], b0[3];
    double amp, lambda, phase;
} orc_field;

static void orc_field_at(const orc_field* f, double x, double t, double e[3], double b[3]) {
    if (f->kind == 0) {
        for (int k = 0; k < 3; ++k) { e[k] = f->e0[k]; b[k] = f->b0[k]; }
        return;
    }
    double ph = 2.0 * M_PI / f->lambda * (f->dir * x - ORC_C * t) + f->phase;
    e[0] = 0.0; e[1] = f->amp * cos(ph); e[2] = f->amp * sin(ph);
    b[0] = 0.0; b[1] = -f->dir * e[2] / ORC_C; b[2] = f->dir * e[1] / ORC_C;
}

void orc_push(orc_particles* p, double* x, double* y, double* z, const orc_field* f, double t, double dt) {
    double qm = p->species == 0 ? -ORC_QE / ORC_ME : (p->species == 1 ? ORC_QE / ORC_ME : 0.0);
    for (int64_t i = 0; i < p->n; ++i) {
        double u[3] = {p->ux[i], p->uy[i], p->uz[i]};
        double r[3] = {x[i], y[i], z[i]};
        if (qm != 0.0) {
            double e[3], b[3];
            orc_field_at(f, r[0], t, e, b);
            double kick = qm * dt / (2.0 * ORC_C);
            double um[3];
            for (int k = 0; k < 3; ++k) um[k] = u[k] + kick * e[k];
            double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
            double tv[3];
            for (int k = 0; k < 3; ++k) tv[k] = qm * dt / (2.0 * gm) * b[k];
            double t2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
            double sv[3];
            for (int k = 0; k < 3; ++k) sv[k] = 2.0 * tv[k] / (1.0 + t2);
            double w[3] = {um[0] + (um[1] * tv[2] - um[2] * tv[1]), um[1] + (um[2] * tv[0] - um[0] * tv[2]),
                           um[2] + (um[0] * tv[1] - um[1] * tv[0])};
            double up[3] = {um[0] + (w[1] * sv[2] - w[2] * sv[1]), um[1] + (w[2] * sv[0] - w[0] * sv[2]),
                            um[2] + (w[0] * sv[1] - w[1] * sv[0])};
            for (int k = 0; k < 3; ++k) u[k] = up[k] + kick * e[k];
            double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int k = 0; k < 3; ++k) r[k] += ORC_C * u[k] / g * dt;
        } else {
            double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (um > 0.0)
                for (int k = 0; k < 3; ++k) r[k] += ORC_C * u[k] / um * dt;
        }
        double e[3], b[3];
        orc_field_at(f, r[0], t + dt, e, b);
        p->ux[i] = u[0]; p->uy[i] = u[1]; p->uz[i] = u[2];
        p->ex[i] = e[0]; p->ey[i] = e[1]; p->ez[i] = e[2];
        p->bx[i] = b[0]; p->by[i] = b[1]; p->bz[i] = b[2];
        x[i] = r[0]; y[i] = r[1]; z[i] = r[2];
    }
}

/* Threads of the OpenMP loops (baseline timing at one and at all threads). */
void orc_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}

int orc_max_threads(void) { return omp_get_max_threads(); }
