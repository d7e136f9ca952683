// Host-side lookup-table generation (paper Sec. 3.1, 3.2).
#pragma once

namespace qedmi {

// chi grid point n of n_chi log-spaced points in [chi_min, chi_max].
double grid_chi(double chi_min, double chi_max, int n_chi, int n);

// process 0 = BW, 1 = QS.  Fills ln_rate[n_chi] and cdf[n_chi * n_frac]
// (row-major): BW stores ln T and P on linear xi in [0, 1/2]; QS stores
// ln G and ln P on log-spaced xi in [frac_min, 1].
void generate_tables(int process, double chi_min, double chi_max, int n_chi, int n_frac,
                     double frac_min, int n_threads, double* ln_rate, double* cdf);

// e^x K_nu(x) and e^x int_x^inf K_nu(s) ds (exported for tests).
double bessel_k_scaled(double nu, double x);
double bessel_ik_scaled(double nu, double x);

}  // namespace qedmi
