// Lookup-table generation on the GPU (paper Sec. 3.1, 3.2 tables from the
// Bessel-function integrals of Sec. 2.1 and 2.2), FP64.  The paper generates
// its tables on the CPU; every entry is an independent quadrature, so one
// block per chi row does the whole row here.
//
// Quadrature (differs from the host generator on purpose, so that the two
// check each other):
//  * e^x K_nu(x) and e^x IK_nu(x) (IK_nu = int_x^inf K_nu) by the
//    trapezoidal rule in t on exp(-2 x sinh^2(t/2)) cosh(nu t) [/ cosh t]
//    (DLMF 10.32.9, integrated once in x for IK), which converges
//    geometrically for these even analytic integrands.
//  * Each table interval [xi_{m-1}, xi_m] by composite Gauss-Legendre with
//    kGlPanels panels of kGlNodes nodes: BW on linear xi (0, 1/2]; QS in
//    s = ln xi on the log-spaced knots, the last interval in ln(1 - xi)
//    (where 1 - xi must keep its digits), and [0, xi_min] with
//    xi = xi_min v^3, which removes the xi^{-2/3} growth at 0.
//  * Interval integrals are summed in xi order per row (fixed order, so the
//    result does not depend on the launch), then normalised as in Sec. 3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "constants.hpp"
#include "internal.hpp"

namespace qedmi {
namespace {

constexpr int kGlNodes = 12;
constexpr int kGlPanels = 2;
constexpr int kGenBlock = 256;

struct GenArgs {
    int process;          // 0 BW, 1 QS
    int n_chi, n_frac;
    double ln_chi_min, dln_chi;
    double ln_frac_min;
    double gl_x[kGlNodes], gl_w[kGlNodes];   // Gauss-Legendre on [-1, 1]
    double* ln_rate;      // [n_chi]
    double* cdf;          // [n_chi][n_frac]
    double* part;         // scratch [n_chi][n_frac]: interval integrals
};

struct Pair {
    double ek, eik;
};

// e^x K_nuk(x) and e^x IK_nuik(x).
__device__ Pair bessel_pair(double x, double nu_k, double nu_ik) {
    const double h = fmin(0.25, 0.5 / sqrt(x));
    const double grow = fmax(nu_k, nu_ik);
    double sk = 0.5, sik = 0.5;
    for (int j = 1; j < 200000; ++j) {
        const double t = j * h;
        const double sh = sinh(0.5 * t);
        const double ex = -2.0 * x * sh * sh;
        const double e = exp(ex);
        const double ck = cosh(nu_k * t);
        const double cik = cosh(nu_ik * t) / cosh(t);
        sk += e * ck;
        sik += e * cik;
        if (ex + grow * t < -40.0 && 2.0 * x * sinh(t) > grow && e * ck < 1e-18 * sk && e * cik < 1e-18 * sik) break;
    }
    return {sk * h, sik * h};
}

// BW integrand scaled by e^{8/(3 chi)}: IK_{1/3}(z) + (1/q - 2) K_{2/3}(z),
// q = xi (1 - xi), z = 2/(3 chi q).
__device__ double bw_integrand(double chi, double xi) {
    const double om = 1.0 - xi;
    const double q = xi * om;
    if (!(q > 0.0)) return 0.0;
    const double d = (2.0 / (3.0 * chi)) * (om - xi) * (om - xi) / q;
    if (d > 740.0) return 0.0;
    const Pair p = bessel_pair(2.0 / (3.0 * chi * q), 2.0 / 3.0, 1.0 / 3.0);
    return exp(-d) * (p.eik + (1.0 / q - 2.0) * p.ek);
}

// QS number spectrum bracket: IK_{5/3}(Y) + xi^2/(1 - xi) K_{2/3}(Y),
// Y = 2 xi / (3 chi (1 - xi)); om = 1 - xi to full precision.
__device__ double qs_integrand(double chi, double xi, double om) {
    if (!(om > 0.0) || !(xi > 0.0)) return 0.0;
    const double y = 2.0 * xi / (3.0 * chi * om);
    if (y > 740.0) return 0.0;
    const Pair p = bessel_pair(y, 2.0 / 3.0, 5.0 / 3.0);
    return exp(-y) * (p.eik + xi * xi / om * p.ek);
}

// Integral over table interval m (1 <= m < n_frac; QS m = 0 is [0, xi_min])
// by composite Gauss-Legendre in the interval's variable.  The first BW
// interval takes xi = xi_1 v^3 (the integrand grows like xi^{-1/3} at large
// chi before its exp(-2/(3 chi xi)) cut-off), the last QS interval runs in
// r = ln(1 - xi) over 36 e-folds below ln(1 - xi_{N-2}) (the integrand falls
// off like exp(-2/(3 chi (1 - xi)))), both on more panels.
__device__ double interval_integral(const GenArgs& a, double chi, int m) {
    const int nf = a.n_frac;
    const bool bw = a.process == 0;
    const bool first_bw = bw && m == 1;
    const bool last_qs = !bw && m == nf - 1;
    const int panels = last_qs ? 48 : (first_bw || (!bw && m == 0)) ? 8 : kGlPanels;
    double sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        for (int g = 0; g < kGlNodes; ++g) {
            const double tt = (p + 0.5 * (a.gl_x[g] + 1.0)) / panels;   // in (0, 1)
            const double w = a.gl_w[g] * 0.5 / panels;
            double f;
            if (first_bw) {
                const double x1 = 0.5 / (nf - 1);
                const double xi = x1 * tt * tt * tt;
                f = 3.0 * x1 * tt * tt * bw_integrand(chi, xi);
            } else if (bw) {
                const double lo = 0.5 * (m - 1) / (nf - 1), hi = 0.5 * m / (nf - 1);
                f = (hi - lo) * bw_integrand(chi, lo + (hi - lo) * tt);
            } else if (m == 0) {
                // xi = xi_min v^3, dxi = 3 xi_min v^2 dv
                const double xmin = exp(a.ln_frac_min);
                const double xi = xmin * tt * tt * tt;
                f = 3.0 * xmin * tt * tt * qs_integrand(chi, xi, 1.0 - xi);
            } else if (!last_qs) {
                const double s0 = a.ln_frac_min * (1.0 - double(m - 1) / (nf - 1));
                const double s1 = a.ln_frac_min * (1.0 - double(m) / (nf - 1));
                const double sv = s0 + (s1 - s0) * tt;
                const double xi = exp(sv);
                f = (s1 - s0) * xi * qs_integrand(chi, xi, -expm1(sv));
            } else {
                const double xa = exp(a.ln_frac_min / (nf - 1));
                const double r0 = log1p(-xa), r1 = r0 - 36.0;
                const double r = r0 + (r1 - r0) * tt;
                const double om = exp(r);
                f = (r0 - r1) * om * qs_integrand(chi, -expm1(r), om);
            }
            sum += w * f;
        }
    }
    return sum;
}

__global__ void __launch_bounds__(kGenBlock) gen_intervals_kernel(GenArgs a) {
    const int n = blockIdx.y;
    const double chi = exp(a.ln_chi_min + n * a.dln_chi);
    const int m = blockIdx.x * kGenBlock + threadIdx.x;
    const int first = a.process == 0 ? 1 : 0;
    if (m < first || m >= a.n_frac) return;
    a.part[static_cast<size_t>(n) * a.n_frac + m] = interval_integral(a, chi, m);
}

// One thread per row: cumulative sums in xi order and normalisation.
__global__ void __launch_bounds__(64) gen_rows_kernel(GenArgs a) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.n_chi) return;
    const double chi = exp(a.ln_chi_min + n * a.dln_chi);
    const double* part = a.part + static_cast<size_t>(n) * a.n_frac;
    double* row = a.cdf + static_cast<size_t>(n) * a.n_frac;
    constexpr double kPiD = 3.141592653589793;
    if (a.process == 0) {
        double s = 0.0;
        row[0] = 0.0;
        for (int m = 1; m < a.n_frac; ++m) {
            s += part[m];
            row[m] = s;
        }
        const double total = 2.0 * s;   // symmetric under xi -> 1 - xi
        a.ln_rate[n] = log(total) - 8.0 / (3.0 * chi) - log(kPiD * sqrt(3.0) * chi);
        for (int m = 1; m < a.n_frac - 1; ++m) row[m] /= total;
        row[a.n_frac - 1] = 0.5;
    } else {
        double s = 0.0;
        for (int m = 0; m < a.n_frac; ++m) {
            s += part[m];
            row[m] = s;
        }
        a.ln_rate[n] = log(sqrt(3.0) / (2.0 * kPiD) * s);
        for (int m = 0; m < a.n_frac - 1; ++m) row[m] = log(row[m] / s);
        row[a.n_frac - 1] = 0.0;
    }
}

void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(3.141592653589793 * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                break;
            }
        }
        // recompute the weight at the converged node
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

// Fill host arrays ln_rate[n_chi], cdf[n_chi * n_frac] by generating on the
// current device (synchronous on `stream`).
int32_t generate_tables_device(const qed_table_params& p, double* ln_rate, double* cdf, hipStream_t stream) {
    GenArgs a{};
    a.process = p.process;
    a.n_chi = p.n_chi;
    a.n_frac = p.n_frac;
    a.ln_chi_min = std::log(p.chi_min);
    a.dln_chi = (std::log(p.chi_max) - a.ln_chi_min) / (p.n_chi - 1);
    a.ln_frac_min = p.process == QED_PROC_QS ? std::log(p.frac_min) : 0.0;
    gauss_legendre(kGlNodes, a.gl_x, a.gl_w);
    const size_t nc = static_cast<size_t>(p.n_chi) * p.n_frac;
    double *d_lr = nullptr, *d_cdf = nullptr, *d_part = nullptr;
    hipError_t e = hipMalloc(&d_lr, sizeof(double) * p.n_chi);
    if (e == hipSuccess) e = hipMalloc(&d_cdf, sizeof(double) * nc);
    if (e == hipSuccess) e = hipMalloc(&d_part, sizeof(double) * nc);
    if (e != hipSuccess) {
        hipFree(d_lr);
        hipFree(d_cdf);
        hipFree(d_part);
        set_error("device allocation for table generation failed");
        return QED_ERR_ALLOC;
    }
    a.ln_rate = d_lr;
    a.cdf = d_cdf;
    a.part = d_part;
    const dim3 grid((p.n_frac + kGenBlock - 1) / kGenBlock, p.n_chi);
    hipLaunchKernelGGL(gen_intervals_kernel, grid, dim3(kGenBlock), 0, stream, a);
    hipLaunchKernelGGL(gen_rows_kernel, dim3((p.n_chi + 63) / 64), dim3(64), 0, stream, a);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(ln_rate, d_lr, sizeof(double) * p.n_chi, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(cdf, d_cdf, sizeof(double) * nc, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    hipFree(d_lr);
    hipFree(d_cdf);
    hipFree(d_part);
    if (e != hipSuccess) {
        set_error(std::string("device table generation: ") + hipGetErrorString(e));
        return QED_ERR_HIP;
    }
    return QED_OK;
}

}  // namespace qedmi
