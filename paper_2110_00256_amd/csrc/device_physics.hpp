// Device-side physics of the QED step: counter-based random numbers, the
// quantum parameter chi, table rates and inverse-CDF sampling.
// Paper references: Sec. 2 (chi, total rates), Sec. 3.1 / 3.2 (tables,
// interpolation, sampling), Sec. 3.3 (caller-supplied uniform numbers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "constants.hpp"
#include "internal.hpp"

namespace qedmi {
namespace dev {

// ------------------------------------------------------------------ Philox
// The 128-bit product m c as (lo, hi).  kSplit: from four 32x32->64 partial
// products chained through their carries (each one v_mad_u64_u32, no
// separate 32-bit low multiplies: a third fewer quarter-rate instructions
// than the compiler's own lowering of the 64-bit product and its high
// half).  Both give the same bits; which one a kernel runs faster with
// depends on the code around it (measured: the split form takes the FP32
// step's generate calls 6-7% faster and the FP64 ones 13-15% slower).
template <bool kSplit>
__device__ __forceinline__ void mulhilo64(unsigned long long m, unsigned long long c, unsigned long long& lo,
                                          unsigned long long& hi) {
    if constexpr (!kSplit) {
        lo = m * c;
        hi = __umul64hi(m, c);
        return;
    }
    const unsigned ml = static_cast<unsigned>(m), mh = static_cast<unsigned>(m >> 32);
    const unsigned cl = static_cast<unsigned>(c), ch = static_cast<unsigned>(c >> 32);
    const unsigned long long p0 = static_cast<unsigned long long>(ml) * cl;
    const unsigned long long p1 = static_cast<unsigned long long>(ml) * ch + (p0 >> 32);
    const unsigned long long p2 = static_cast<unsigned long long>(mh) * cl + static_cast<unsigned>(p1);
    hi = static_cast<unsigned long long>(mh) * ch + (p1 >> 32) + (p2 >> 32);
    lo = (p2 << 32) | static_cast<unsigned>(p0);
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with Weyl-sequence key bumps.
template <bool kSplit = false>
__device__ __forceinline__ void philox4x64_10(unsigned long long& c0, unsigned long long& c1,
                                              unsigned long long& c2, unsigned long long& c3,
                                              unsigned long long k0, unsigned long long k1) {
    constexpr unsigned long long kM0 = 0xD2E7470EE14C6C93ULL, kM1 = 0xCA5A826395121157ULL;
    constexpr unsigned long long kW0 = 0x9E3779B97F4A7C15ULL, kW1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        unsigned long long lo0, hi0, lo1, hi1;
        mulhilo64<kSplit>(kM0, c0, lo0, hi0);
        mulhilo64<kSplit>(kM1, c2, lo1, hi1);
        const unsigned long long n0 = hi1 ^ c1 ^ k0;
        const unsigned long long n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kW0;
        k1 += kW1;
    }
}

// (2m + 1) 2^-53 from the top 52 bits: in (0, 1), exact, and 1 - u exact.
__device__ __forceinline__ double u01(unsigned long long w) {
    return static_cast<double>(2ULL * (w >> 12) + 1ULL) * 0x1.0p-53;
}

struct Draws {
    double u[4];
};

// Block `blk` of particle `id` at `step` for `species` under `seed`
// (kSplit: the form of the 64-bit products, same bits either way).
template <bool kSplit = false>
__device__ __forceinline__ Draws draws(unsigned long long seed, unsigned long long id,
                                       unsigned long long step, unsigned long long species,
                                       unsigned long long blk) {
    unsigned long long c0 = id, c1 = step, c2 = species, c3 = blk;
    philox4x64_10<kSplit>(c0, c1, c2, c3, seed, 0ULL);
    Draws d;
    d.u[0] = u01(c0);
    d.u[1] = u01(c1);
    d.u[2] = u01(c2);
    d.u[3] = u01(c3);
    return d;
}

constexpr unsigned long long kInitStep = ~0ULL;

// ------------------------------------------------------------------ chi
// chi E_s = sqrt(|a|^2 + (gamma^2 - |u|^2) E_par^2), a = gamma E_perp + c u x B,
// E_par = E.n, n = u/|u|; gamma^2 - |u|^2 is 1 for leptons, 0 for photons.
// (Sec. 2 definitions of chi and chi_gamma, with gamma (E + v x B) =
// gamma E + c u x B and gamma v.E/c = u.E.)
struct ChiGamma {
    double chi;
    double gamma;
    double u2;
};

template <bool kPhoton>
__device__ __forceinline__ ChiGamma chi_f64(double ux, double uy, double uz, double ex, double ey,
                                            double ez, double bx, double by, double bz) {
    ChiGamma r;
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double um = sqrt(u2);
    const double g = kPhoton ? um : sqrt(1.0 + u2);
    r.gamma = g;
    r.u2 = u2;
    if (um == 0.0) {
        r.chi = kPhoton ? 0.0 : sqrt(ex * ex + ey * ey + ez * ez) * kInvEs;
        return r;
    }
    const double inv = 1.0 / um;
    const double nx = ux * inv, ny = uy * inv, nz = uz * inv;
    const double ep = ex * nx + ey * ny + ez * nz;
    const double ax = g * (ex - ep * nx) + kC * (uy * bz - uz * by);
    const double ay = g * (ey - ep * ny) + kC * (uz * bx - ux * bz);
    const double az = g * (ez - ep * nz) + kC * (ux * by - uy * bx);
    double s = ax * ax + ay * ay + az * az;
    if (!kPhoton) s += ep * ep;
    r.chi = sqrt(s) * kInvEs;
    return r;
}

// Plain FP32 evaluation of the same decomposition; fields pre-scaled by
// 2^-60 (exact) so that gamma |E| stays inside the FP32 range.
template <bool kPhoton>
__device__ __forceinline__ ChiGamma chi_f32(float ux, float uy, float uz, float ex, float ey, float ez,
                                            float bx, float by, float bz) {
    constexpr float kScale = 0x1.0p-60f;
    constexpr float kCs = static_cast<float>(kC);
    constexpr double kBack = 0x1.0p60 * kInvEs;
    ChiGamma r;
    ex *= kScale; ey *= kScale; ez *= kScale;
    bx *= kScale * kCs; by *= kScale * kCs; bz *= kScale * kCs;
    const float u2 = ux * ux + uy * uy + uz * uz;
    const float um = sqrtf(u2);
    const float g = kPhoton ? um : sqrtf(1.0f + u2);
    r.gamma = g;
    r.u2 = u2;
    if (um == 0.0f) {
        r.chi = kPhoton ? 0.0 : static_cast<double>(sqrtf(ex * ex + ey * ey + ez * ez)) * kBack;
        return r;
    }
    const float inv = 1.0f / um;
    const float nx = ux * inv, ny = uy * inv, nz = uz * inv;
    const float ep = ex * nx + ey * ny + ez * nz;
    const float ax = g * (ex - ep * nx) + (uy * bz - uz * by);
    const float ay = g * (ey - ep * ny) + (uz * bx - ux * bz);
    const float az = g * (ez - ep * nz) + (ux * by - uy * bx);
    float s = ax * ax + ay * ay + az * az;
    if (!kPhoton) s += ep * ep;
    r.chi = static_cast<double>(sqrtf(s)) * kBack;
    return r;
}

// ------------------------------------------------------ compensated FP32
// Double-float arithmetic (value = hi + lo, |lo| <= ulp(hi)/2) built from
// the error-free transformations TwoSum (Knuth) and TwoProd (fma).  These
// need every product and sum rounded as written, so contraction into fused
// multiply-adds is switched off inside them.
struct DF {
    float hi, lo;
};
__device__ __forceinline__ DF df_two_sum(float a, float b) {
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ DF df_fast_sum(float a, float b) {
#pragma clang fp contract(off)
    const float s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ DF df_add(DF x, DF y) {
#pragma clang fp contract(off)
    DF s = df_two_sum(x.hi, y.hi);
    return df_fast_sum(s.hi, s.lo + x.lo + y.lo);
}
__device__ __forceinline__ DF df_neg(DF x) { return {-x.hi, -x.lo}; }
__device__ __forceinline__ DF df_mul(DF x, DF y) {
#pragma clang fp contract(off)
    const float p = x.hi * y.hi;
    const float e = fmaf(x.hi, y.hi, -p);
    return df_fast_sum(p, e + (x.hi * y.lo + x.lo * y.hi));
}
__device__ __forceinline__ DF df_from(float a) { return {a, 0.0f}; }
__device__ __forceinline__ DF df_sqrt(DF x) {
#pragma clang fp contract(off)
    if (!(x.hi > 0.0f)) return {0.0f, 0.0f};
    const float s = sqrtf(x.hi);
    const float p = s * s;
    const float e = fmaf(s, s, -p);
    const float r = ((x.hi - p) - e + x.lo) / (2.0f * s);
    return df_fast_sum(s, r);
}
__device__ __forceinline__ DF df_div(DF x, DF y) {
#pragma clang fp contract(off)
    const float q1 = x.hi / y.hi;
    const DF r = df_add(x, df_neg(df_mul(df_from(q1), y)));
    const float q2 = r.hi / y.hi;
    return df_fast_sum(q1, q2);
}

template <bool kPhoton>
__device__ __forceinline__ ChiGamma chi_comp32(float fux, float fuy, float fuz, float fex, float fey,
                                               float fez, float fbx, float fby, float fbz) {
    constexpr float kScale = 0x1.0p-60f;
    constexpr double kBack = 0x1.0p60 * kInvEs;
    // c as an exact float pair: c = chi_ + clo
    constexpr float kChi = static_cast<float>(kC);
    constexpr float kClo = static_cast<float>(kC - static_cast<double>(kChi));
    const DF c{kChi, kClo};
    ChiGamma r;
    const DF ux = df_from(fux), uy = df_from(fuy), uz = df_from(fuz);
    const DF ex = df_from(fex * kScale), ey = df_from(fey * kScale), ez = df_from(fez * kScale);
    const DF bx = df_mul(c, df_from(fbx * kScale)), by = df_mul(c, df_from(fby * kScale)),
             bz = df_mul(c, df_from(fbz * kScale));
    const DF u2 = df_add(df_add(df_mul(ux, ux), df_mul(uy, uy)), df_mul(uz, uz));
    const DF um = df_sqrt(u2);
    const DF g = kPhoton ? um : df_sqrt(df_add(df_from(1.0f), u2));
    r.gamma = static_cast<double>(g.hi) + static_cast<double>(g.lo);
    r.u2 = static_cast<double>(u2.hi) + static_cast<double>(u2.lo);
    if (um.hi == 0.0f) {
        const DF e2 = df_add(df_add(df_mul(ex, ex), df_mul(ey, ey)), df_mul(ez, ez));
        r.chi = kPhoton ? 0.0 : static_cast<double>(df_sqrt(e2).hi) * kBack;
        return r;
    }
    const DF nx = df_div(ux, um), ny = df_div(uy, um), nz = df_div(uz, um);
    const DF ep = df_add(df_add(df_mul(ex, nx), df_mul(ey, ny)), df_mul(ez, nz));
    const DF ax = df_add(df_mul(g, df_add(ex, df_neg(df_mul(ep, nx)))),
                         df_add(df_mul(uy, bz), df_neg(df_mul(uz, by))));
    const DF ay = df_add(df_mul(g, df_add(ey, df_neg(df_mul(ep, ny)))),
                         df_add(df_mul(uz, bx), df_neg(df_mul(ux, bz))));
    const DF az = df_add(df_mul(g, df_add(ez, df_neg(df_mul(ep, nz)))),
                         df_add(df_mul(ux, by), df_neg(df_mul(uy, bx))));
    DF s = df_add(df_add(df_mul(ax, ax), df_mul(ay, ay)), df_mul(az, az));
    if (!kPhoton) s = df_add(s, df_mul(ep, ep));
    const DF rt = df_sqrt(s);
    r.chi = (static_cast<double>(rt.hi) + static_cast<double>(rt.lo)) * kBack;
    return r;
}

// Dispatch on element type and chi mode.  FP64 data always uses FP64.
template <typename T, bool kPhoton>
__device__ __forceinline__ ChiGamma chi_of(int chi_mode, T ux, T uy, T uz, T ex, T ey, T ez, T bx, T by,
                                           T bz) {
    if constexpr (sizeof(T) == 8) {
        return chi_f64<kPhoton>(ux, uy, uz, ex, ey, ez, bx, by, bz);
    } else {
        if (chi_mode == QED_CHI_FP32) return chi_f32<kPhoton>(ux, uy, uz, ex, ey, ez, bx, by, bz);
        if (chi_mode == QED_CHI_COMP32) return chi_comp32<kPhoton>(ux, uy, uz, ex, ey, ez, bx, by, bz);
        return chi_f64<kPhoton>(ux, uy, uz, ex, ey, ez, bx, by, bz);
    }
}

// ------------------------------------------------------------------ rates
// Precision-generic helpers.
__device__ __forceinline__ double dlog(double x) { return log(x); }
__device__ __forceinline__ float dlog(float x) { return logf(x); }
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dexp(float x) { return expf(x); }

// A uniform parameter in the compute precision: the FP64 value, or its copy
// rounded to FP32 on the host (the same value a conversion here would give).
template <typename T>
__device__ __forceinline__ T par(double d, float f) {
    if constexpr (sizeof(T) == 8) return d;
    else return f;
}

// Interval index n in [0, N-2] and weight f = t - n for ln chi on the grid.
template <typename T>
__device__ __forceinline__ void grid_pos(const TableDev& t, T lnchi, int& n, T& f) {
    const T x = (lnchi - par<T>(t.ln_chi_min, t.ln_chi_min_f)) * par<T>(t.inv_dlnchi, t.inv_dlnchi_f);
    int k = static_cast<int>(floor(x));
    k = k < 0 ? 0 : (k > t.n_chi - 2 ? t.n_chi - 2 : k);
    n = k;
    f = x - static_cast<T>(k);
}

// BF16 table storage, read as FP32 (precision studies).
struct Bf16 {
    uint16_t bits;
};
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(static_cast<unsigned>(b) << 16); }

// Table element of storage type S read as arithmetic type T.
template <typename T>
__device__ __forceinline__ T tload(const double* p, int i) { return static_cast<T>(p[i]); }
template <typename T>
__device__ __forceinline__ T tload(const float* p, int i) { return static_cast<T>(p[i]); }
template <typename T>
__device__ __forceinline__ T tload(const Bf16* p, int i) { return static_cast<T>(bf16_to_f32(p[i].bits)); }

// Entry k of a row pair (both rows' values with one load).
template <typename T>
__device__ __forceinline__ void tload2(const double* pp, int k, T& a0, T& a1) {
    const double2 v = *reinterpret_cast<const double2*>(pp + 2 * k);
    a0 = static_cast<T>(v.x);
    a1 = static_cast<T>(v.y);
}
template <typename T>
__device__ __forceinline__ void tload2(const float* pp, int k, T& a0, T& a1) {
    const float2 v = *reinterpret_cast<const float2*>(pp + 2 * k);
    a0 = static_cast<T>(v.x);
    a1 = static_cast<T>(v.y);
}
template <typename T>
__device__ __forceinline__ void tload2(const Bf16* pp, int k, T& a0, T& a1) {
    const unsigned v = *reinterpret_cast<const unsigned*>(pp + 2 * k);
    a0 = static_cast<T>(bf16_to_f32(static_cast<uint16_t>(v & 0xffffu)));
    a1 = static_cast<T>(bf16_to_f32(static_cast<uint16_t>(v >> 16)));
}

// BW: dN/dt = (alpha m c^2/hbar) (chi_gamma/gamma_gamma) T(chi_gamma)
// (Sec. 2.1); ln T interpolated linearly in ln chi (Sec. 3.1); outside the
// table, the asymptotes of the integral definition matched at the edges:
// ln T - (8/3)(1/chi - 1/chi_min) below, ln T - (1/3) ln(chi/chi_max) above.
template <typename T, typename S>
__device__ __forceinline__ T rate_bw(const S* ln_t, const TableDev& t, T chi, T gamma_g) {
    if (!(chi > T(0)) || !(gamma_g > T(0))) return T(0);
    T y;
    if (chi < par<T>(t.chi_min, t.chi_min_f)) {
        y = tload<T>(ln_t, 0) - T(8.0 / 3.0) * (T(1) / chi - par<T>(t.inv_chi_min, t.inv_chi_min_f));
    } else if (chi > par<T>(t.chi_max, t.chi_max_f)) {
        y = tload<T>(ln_t, t.n_chi - 1) - T(1.0 / 3.0) * (dlog(chi) - par<T>(t.ln_chi_max, t.ln_chi_max_f));
    } else {
        int n;
        T f;
        grid_pos<T>(t, dlog(chi), n, f);
        const T y0 = tload<T>(ln_t, n), y1 = tload<T>(ln_t, n + 1);
        y = y0 + f * (y1 - y0);
    }
    return static_cast<T>(kRateR0) * (chi / gamma_g) * dexp(y);
}

// QS: dN/dt = (2/3)(alpha m c^2/hbar) G(chi)/gamma (Sec. 2.2); ln G
// interpolated in ln chi; first/last stored value outside (Sec. 3.2).
template <typename T, typename S>
__device__ __forceinline__ T rate_qs(const S* ln_g, const TableDev& t, T chi, T gamma) {
    T y;
    if (!(chi >= par<T>(t.chi_min, t.chi_min_f))) {
        y = tload<T>(ln_g, 0);
    } else if (chi > par<T>(t.chi_max, t.chi_max_f)) {
        y = tload<T>(ln_g, t.n_chi - 1);
    } else {
        int n;
        T f;
        grid_pos<T>(t, dlog(chi), n, f);
        const T y0 = tload<T>(ln_g, n), y1 = tload<T>(ln_g, n + 1);
        y = y0 + f * (y1 - y0);
    }
    return static_cast<T>(2.0 / 3.0 * kRateR0) * dexp(y) / gamma;
}

// Row position for the 2D tables: chi clamped to [chi_min, chi_max].
template <typename T>
__device__ __forceinline__ void row_pos(const TableDev& t, T chi, int& n, T& f) {
    T c = chi;
    if (!(c >= par<T>(t.chi_min, t.chi_min_f))) c = par<T>(t.chi_min, t.chi_min_f);
    if (c > par<T>(t.chi_max, t.chi_max_f)) c = par<T>(t.chi_max, t.chi_max_f);
    grid_pos<T>(t, dlog(c), n, f);
}

template <typename S>
__device__ __forceinline__ const S* cdf_ptr(const TableDev& t);
template <>
__device__ __forceinline__ const double* cdf_ptr<double>(const TableDev& t) { return t.cdf64; }
template <>
__device__ __forceinline__ const float* cdf_ptr<float>(const TableDev& t) { return t.cdf32; }
template <>
__device__ __forceinline__ const Bf16* cdf_ptr<Bf16>(const TableDev& t) {
    return reinterpret_cast<const Bf16*>(t.cdf16);
}


// Row interpolated between the two rows of a pair with weight f, at k.
template <typename T, typename S>
__device__ __forceinline__ T pair_value(const S* pp, T f, int k) {
    T a0, a1;
    tload2<T>(pp, k, a0, a1);
    return a0 + f * (a1 - a0);
}

// Upper-bound binary search over the row pair pp interpolated with weight f:
// starting from [0, nf - 1], halve while hi - lo > 1, keeping lo when the
// interpolated value at mid is <= r; returns lo.  Two levels per round: the
// probe at mid and both possible next probes are loaded together, so the
// chain of dependent table reads is half as long, and the decisions (hence
// the result) are those of the plain one-level search.
template <typename T, typename S>
__device__ __forceinline__ int upper_bound_row(const S* pp, T f, T r, int nf) {
    int lo = 0, hi = nf - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        const int ml = (lo + mid) >> 1;   // next probe if the search goes left
        const int mr = (mid + hi) >> 1;   // next probe if it goes right
        const T vm = pair_value<T, S>(pp, f, mid);
        const T vl = pair_value<T, S>(pp, f, ml);
        const T vr = pair_value<T, S>(pp, f, mr);
        if (vm <= r) {
            lo = mid;
            if (hi - lo > 1) {
                if (vr <= r) lo = mr;
                else hi = mr;
            }
        } else {
            hi = mid;
            if (hi - lo > 1) {
                if (vl <= r) lo = ml;
                else hi = ml;
            }
        }
    }
    return lo;
}

// BW pair sampling (Sec. 3.1) for a folded uniform r in (0, 1/2]: rows n,
// n+1 interpolated in ln chi_gamma; binary search for P_m <= r < P_{m+1};
// linear inverse in xi.
template <typename T, typename S = T>
__device__ __forceinline__ T sample_bw_folded(const TableDev& t, T chi, T r) {
    int n;
    T f;
    row_pos<T>(t, chi, n, f);
    const int nf = t.n_frac;
    const S* pp = cdf_ptr<S>(t) + 2 * static_cast<size_t>(n) * nf;
    const int lo = upper_bound_row<T, S>(pp, f, r, nf);
    const T pa = pair_value<T, S>(pp, f, lo);
    const T pb = pair_value<T, S>(pp, f, lo + 1);
    const T scale = T(0.5) / static_cast<T>(nf - 1);
    const T xa = scale * static_cast<T>(lo), xb = scale * static_cast<T>(lo + 1);
    return xa + (r - pa) * (xb - xa) / (pb - pa);
}

// The fold of Sec. 3.1: r <= 1/2 selects the electron, otherwise r -> 1 - r
// selects the positron.
template <typename T, typename S = T>
__device__ __forceinline__ T sample_bw(const TableDev& t, T chi, T r, bool& electron) {
    electron = (r <= T(0.5));
    if (!electron) r = T(1) - r;
    return sample_bw_folded<T, S>(t, chi, r);
}

// QS photon sampling (Sec. 3.2) given lr = ln r: ln P rows interpolated in
// ln chi; binary search on ln r; log-log inverse.  Below the first knot the
// small-xi law P ~ xi^{1/3} continues the table: ln xi = ln xi_min + 3 (ln r
// - ln P_0).  Returns ln xi.
template <typename T, typename S = T>
__device__ __forceinline__ T sample_qs_lnxi_lr(const TableDev& t, T chi, T lr) {
    int n;
    T f;
    row_pos<T>(t, chi, n, f);
    const int nf = t.n_frac;
    const S* pp = cdf_ptr<S>(t) + 2 * static_cast<size_t>(n) * nf;
    const T lmin = par<T>(t.ln_frac_min, t.ln_frac_min_f);
    const T l0 = pair_value<T, S>(pp, f, 0);
    if (lr < l0) return lmin + T(3) * (lr - l0);
    const int lo = upper_bound_row<T, S>(pp, f, lr, nf);
    const T la = pair_value<T, S>(pp, f, lo);
    const T lb = pair_value<T, S>(pp, f, lo + 1);
    const T inv = T(1) / static_cast<T>(nf - 1);
    const T xa = lmin * (T(1) - static_cast<T>(lo) * inv);
    const T xb = lmin * (T(1) - static_cast<T>(lo + 1) * inv);
    return xa + (lr - la) * (xb - xa) / (lb - la);
}

template <typename T, typename S = T>
__device__ __forceinline__ T sample_qs_lnxi(const TableDev& t, T chi, T r) {
    return sample_qs_lnxi_lr<T, S>(t, chi, dlog(r));
}

// The random inputs of one event's sample, taken from the 53-bit uniform u
// before any narrowing to T: ln u for QS (near u = 1 the FP32 spacing is
// all of 1 - u), and for BW the fold min(u, 1 - u), exact in FP64, with the
// electron chosen on u itself.
template <typename T>
__device__ __forceinline__ T qs_log_uniform(double u) {
    return static_cast<T>(log(u));
}
template <typename T>
__device__ __forceinline__ T bw_folded_uniform(double u, bool& electron) {
    electron = u <= 0.5;
    return static_cast<T>(electron ? u : 1.0 - u);
}

// A redrawn optical depth -ln u.  FP32 takes the logarithm of the rounded
// uniform: its absolute error stays near the FP32 spacing of u (about 6e-8
// where u -> 1 and t -> 0, and relative 6e-8 where t is large), which is
// what the FP32 path's optical depths carry anyway.
template <typename T>
__device__ __forceinline__ T neg_log_uniform(double u);
template <>
__device__ __forceinline__ double neg_log_uniform<double>(double u) { return -log(u); }
template <>
__device__ __forceinline__ float neg_log_uniform<float>(double u) { return -logf(static_cast<float>(u)); }

}  // namespace dev
}  // namespace qedmi
