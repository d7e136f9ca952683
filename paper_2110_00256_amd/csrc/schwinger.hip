// Schwinger pair production (paper Sec. 2.3): the pair creation rate per
// unit volume from the field invariants, and macro-pairs created at rest
// with a per-cell count drawn from Philox, appended in cell order.
//
// Rate: d2N/(dt dV) = q_e^2 E_s^2 / (4 pi^2 hbar^2 c) eps eta
//                     coth(pi eta / eps) exp(-pi / eps),
// eps, eta = sqrt(sqrt(F^2 + G^2) +- F) / E_s, F = (E^2 - c^2 B^2)/2,
// G = c E.B.  Evaluated on e = E/E_s, b = cB/E_s (no overflow in FP32 data)
// and without the cancellation of sqrt(F^2 + G^2) - |F|: with
// s = hypot(f, g), (s + |f|)(s - |f|) = g^2, so the smaller of eps^2, eta^2
// is g^2 / (s + |f|).
//
// Count per cell: Poisson with mean lambda = rate dV dt / W, by inversion
// with the first uniform of the cell's block 0 (counter: cell id, step,
// species 4); above lambda = 25 a Gaussian of mean and variance lambda
// (Box-Muller), rounded and clipped at 0.  Pair i of a cell takes its two
// optical depths from block 1 + i/2.
//
// Ordered append in three launches: per-block totals, one-block scan of the
// totals, per-block recount + LDS scan + writes.
#include <hip/hip_runtime.h>

#include <cmath>

#include "constants.hpp"
#include "device_physics.hpp"
#include "internal.hpp"

namespace qedmi {
namespace {

constexpr int kSwBlock = 256;
constexpr int kSwPerThread = 16;
constexpr int kSwCells = kSwBlock * kSwPerThread;   // cells per block
constexpr unsigned long long kSwSpecies = 4;
constexpr double kPoissonMax = 25.0;

struct SwArgs {
    const void* f[6];
    int64_t n;
    int64_t id_base;
    double pref;          // q_e^2 E_s^2 / (4 pi^2 hbar^2 c)
    double scale;         // dV dt / W
    double weight;        // W, the products' weight
    unsigned long long seed, step;
    void* rate_out;
    int64_t* bsum;        // per-block pair totals, then exclusive offsets
    AppendDev el, po;
    int64_t* total_out;   // device: number of pairs of this call
    int64_t* cnt;         // device: pairs of each cell (written by the count pass)
};

template <typename T>
__device__ __forceinline__ double field(const SwArgs& a, int k, int64_t i) {
    return static_cast<double>(static_cast<const T*>(a.f[k])[i]);
}

template <typename T>
__device__ double sw_rate(const SwArgs& a, int64_t i) {
    constexpr double kPi = 3.141592653589793;
    const double ex = field<T>(a, 0, i) * kInvEs, ey = field<T>(a, 1, i) * kInvEs, ez = field<T>(a, 2, i) * kInvEs;
    const double bx = field<T>(a, 3, i) * (kC * kInvEs), by = field<T>(a, 4, i) * (kC * kInvEs),
                 bz = field<T>(a, 5, i) * (kC * kInvEs);
    const double f = 0.5 * ((ex * ex + ey * ey + ez * ez) - (bx * bx + by * by + bz * bz));
    const double g = ex * bx + ey * by + ez * bz;
    const double s = hypot(f, g);
    const double big = s + fabs(f);
    const double small = big > 0.0 ? g * g / big : 0.0;
    const double eps2 = f >= 0.0 ? big : small;
    const double eta2 = f >= 0.0 ? small : big;
    if (!(eps2 > 0.0)) return 0.0;
    const double eps = sqrt(eps2), eta = sqrt(eta2);
    const double x = kPi * eta / eps;
    const double eta_coth = x < 1e-8 ? eps / kPi : eta / tanh(x);
    const double pre = a.pref * eps * eta_coth, b = kPi / eps;
    // exp(-b) is normal up to b = 708; beyond that it would go subnormal (and
    // lose its digits) long before the rate does, so the rate is taken as one
    // exponential of the whole logarithm there
    return b < 700.0 ? pre * exp(-b) : exp(log(pre) - b);
}

__device__ int64_t sw_count(const SwArgs& a, double lambda, int64_t cell) {
    if (!(lambda > 0.0)) return 0;
    const dev::Draws d = dev::draws(a.seed, static_cast<unsigned long long>(cell), a.step, kSwSpecies, 0ULL);
    if (lambda <= kPoissonMax) {
        double p = exp(-lambda), cum = p;
        int64_t k = 0;
        while (d.u[0] > cum && k < 1000) {
            ++k;
            p *= lambda / static_cast<double>(k);
            cum += p;
        }
        return k;
    }
    const double z = sqrt(-2.0 * log(d.u[0])) * cos(2.0 * 3.141592653589793 * d.u[1]);
    const double v = lambda + sqrt(lambda) * z;
    return v < 0.5 ? 0 : static_cast<int64_t>(floor(v + 0.5));
}

template <typename T>
__device__ __forceinline__ int64_t cell_pairs(const SwArgs& a, int64_t i) {
    return sw_count(a, sw_rate<T>(a, i) * a.scale, a.id_base + i);
}

template <typename T>
__global__ void __launch_bounds__(256) sw_rate_kernel(SwArgs a) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * blockDim.x)
        static_cast<double*>(a.rate_out)[i] = sw_rate<T>(a, i);
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t* lds) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    int64_t t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kSwBlock / 64; ++w) t += lds[w];
    return t;   // valid on thread 0
}

// Exclusive block-wide scan of v (all threads call).
__device__ __forceinline__ int64_t block_exclusive(int64_t v, int64_t* lds, int64_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < kSwBlock / 64; ++w) {
        if (w < wave) before += lds[w];
        all += lds[w];
    }
    *total = all;
    return before + incl - v;
}

template <typename T>
__global__ void __launch_bounds__(kSwBlock) sw_total_kernel(SwArgs a) {
    __shared__ int64_t lds[kSwBlock / 64];
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kSwCells;
    int64_t v = 0;
    for (int q = 0; q < kSwPerThread; ++q) {
        const int64_t i = first + q * kSwBlock + threadIdx.x;
        if (i < a.n) {
            const int64_t k = cell_pairs<T>(a, i);
            a.cnt[i] = k;
            v += k;
        }
    }
    const int64_t t = block_sum(v, lds);
    if (threadIdx.x == 0) a.bsum[blockIdx.x] = t;
}

// One block: exclusive offsets of the per-block totals, in place; the final
// counts of both append buffers.
__global__ void __launch_bounds__(kSwBlock) sw_scan_kernel(SwArgs a, int nb) {
    __shared__ int64_t lds[kSwBlock / 64];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += kSwBlock) {
        const int b = b0 + threadIdx.x;
        const int64_t v = b < nb ? a.bsum[b] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive(v, lds, &tot);
        if (b < nb) a.bsum[b] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *a.total_out = carry;
        *a.el.count += carry;
        *a.po.count += carry;
    }
}

template <typename T>
__device__ __forceinline__ void put(const AppendDev& o, int64_t slot, T w, T tau, int64_t parent) {
    if (slot >= o.capacity) return;
    static_cast<T*>(o.ux)[slot] = T(0);
    static_cast<T*>(o.uy)[slot] = T(0);
    static_cast<T*>(o.uz)[slot] = T(0);
    static_cast<T*>(o.w)[slot] = w;
    static_cast<T*>(o.tau)[slot] = tau;
    if (o.parent) o.parent[slot] = parent;
}

// Slots: each thread owns kSwPerThread consecutive cells of the block's
// range, so a block-wide exclusive scan of the thread totals orders the
// pairs by cell.  base_e / base_p: the buffers' counts before this call
// (count - total after the scan kernel).
// The count pass's per-cell counts are staged through LDS with consecutive
// lanes on consecutive cells (coalesced), then each thread takes its own
// cells'.
template <typename T>
__global__ void __launch_bounds__(kSwBlock) sw_write_kernel(SwArgs a) {
    __shared__ int64_t lds[kSwBlock / 64];
    __shared__ int64_t cnt[kSwCells];
    const int64_t bfirst = static_cast<int64_t>(blockIdx.x) * kSwCells;
    for (int q = 0; q < kSwPerThread; ++q) {
        const int64_t i = bfirst + q * kSwBlock + threadIdx.x;
        cnt[q * kSwBlock + threadIdx.x] = i < a.n ? a.cnt[i] : 0;
    }
    __syncthreads();
    const int64_t first = bfirst + threadIdx.x * kSwPerThread;
    int64_t k[kSwPerThread];
    int64_t v = 0;
    for (int q = 0; q < kSwPerThread; ++q) {
        k[q] = cnt[threadIdx.x * kSwPerThread + q];
        v += k[q];
    }
    int64_t tot;
    int64_t slot = a.bsum[blockIdx.x] + block_exclusive(v, lds, &tot);
    const int64_t total = *a.total_out;
    const int64_t base_e = *a.el.count - total, base_p = *a.po.count - total;
    const T w = static_cast<T>(a.weight);
    for (int q = 0; q < kSwPerThread; ++q) {
        const int64_t cell = a.id_base + first + q;
        for (int64_t p = 0; p < k[q]; ++p, ++slot) {
            const dev::Draws d = dev::draws(a.seed, static_cast<unsigned long long>(cell), a.step, kSwSpecies,
                                            static_cast<unsigned long long>(1 + p / 2));
            const int h = static_cast<int>(p & 1);
            put<T>(a.el, base_e + slot, w, static_cast<T>(-log(d.u[2 * h])), cell);
            put<T>(a.po, base_p + slot, w, static_cast<T>(-log(d.u[2 * h + 1])), cell);
        }
    }
}

int32_t check_cells(const qed_cells* c) {
    if (!c) { set_error("cells is null"); return QED_ERR_INVALID; }
    if (c->n < 0 || c->cell_id_base < 0) { set_error("cells.n and cells.cell_id_base must be >= 0"); return QED_ERR_INVALID; }
    if (c->dtype != QED_FP64 && c->dtype != QED_FP32) { set_error("cells.dtype must be FP64 or FP32"); return QED_ERR_INVALID; }
    if (c->n > 0 && (!c->ex || !c->ey || !c->ez || !c->bx || !c->by || !c->bz)) {
        set_error("a cell field pointer is null");
        return QED_ERR_INVALID;
    }
    return QED_OK;
}

SwArgs make_args(const qed_cells* c) {
    SwArgs a{};
    const void* f[6] = {c->ex, c->ey, c->ez, c->bx, c->by, c->bz};
    for (int k = 0; k < 6; ++k) a.f[k] = f[k];
    a.n = c->n;
    a.id_base = c->cell_id_base;
    constexpr double kPi = 3.141592653589793;
    a.pref = kQe * kQe * kEs * kEs / (4.0 * kPi * kPi * kHbar * kHbar * kC);
    return a;
}

int grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return static_cast<int>(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

}  // namespace
}  // namespace qedmi

using namespace qedmi;

extern "C" int32_t qed_schwinger_rate(qed_context* ctx, const qed_cells* cells, void* rate_out, void* stream) {
    if (!ctx) { set_error("context is null"); return QED_ERR_INVALID; }
    int32_t r = check_cells(cells);
    if (r) return r;
    if (cells->n == 0) return QED_OK;
    if (!rate_out) { set_error("rate_out is null"); return QED_ERR_INVALID; }
    SwArgs a = make_args(cells);
    a.rate_out = rate_out;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (cells->dtype == QED_FP64)
        hipLaunchKernelGGL(sw_rate_kernel<double>, dim3(grid_for(a.n)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(sw_rate_kernel<float>, dim3(grid_for(a.n)), dim3(256), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("qed_schwinger_rate launch: ") + hipGetErrorString(e));
        return QED_ERR_HIP;
    }
    return QED_OK;
}

extern "C" int32_t qed_schwinger_pairs(qed_context* ctx, const qed_cells* cells, double cell_volume, double dt,
                                       double weight, uint64_t seed, uint64_t step, qed_append* electrons,
                                       qed_append* positrons, void* stream) {
    if (!ctx) { set_error("context is null"); return QED_ERR_INVALID; }
    int32_t r = check_cells(cells);
    if (r) return r;
    if (!(cell_volume > 0.0) || !(dt >= 0.0) || !(weight > 0.0) || !std::isfinite(cell_volume * dt / weight)) {
        set_error("need cell_volume > 0, dt >= 0, weight > 0");
        return QED_ERR_INVALID;
    }
    if ((r = check_append_dtype(electrons, cells->dtype, "electrons"))) return r;
    if ((r = check_append_dtype(positrons, cells->dtype, "positrons"))) return r;
    if (cells->n == 0) return QED_OK;
    const int64_t nb = (cells->n + kSwCells - 1) / kSwCells;
    if (nb > INT32_MAX) { set_error("too many cells"); return QED_ERR_INVALID; }
    // scratch: per-block totals, the call's total, then one count per cell
    if ((r = reserve_scratch(ctx, (nb + 1 + cells->n) * static_cast<int64_t>(sizeof(int64_t))))) return r;
    SwArgs a = make_args(cells);
    a.scale = cell_volume * dt / weight;
    a.weight = weight;
    a.seed = seed;
    a.step = step;
    a.bsum = static_cast<int64_t*>(ctx->d_scratch);
    a.total_out = a.bsum + nb;
    a.cnt = a.total_out + 1;
    a.el = append_view(electrons);
    a.po = append_view(positrons);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (cells->dtype == QED_FP64) {
        hipLaunchKernelGGL(sw_total_kernel<double>, dim3(nb), dim3(kSwBlock), 0, s, a);
        hipLaunchKernelGGL(sw_scan_kernel, dim3(1), dim3(kSwBlock), 0, s, a, static_cast<int>(nb));
        hipLaunchKernelGGL(sw_write_kernel<double>, dim3(nb), dim3(kSwBlock), 0, s, a);
    } else {
        hipLaunchKernelGGL(sw_total_kernel<float>, dim3(nb), dim3(kSwBlock), 0, s, a);
        hipLaunchKernelGGL(sw_scan_kernel, dim3(1), dim3(kSwBlock), 0, s, a, static_cast<int>(nb));
        hipLaunchKernelGGL(sw_write_kernel<float>, dim3(nb), dim3(kSwBlock), 0, s, a);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("qed_schwinger_pairs launch: ") + hipGetErrorString(e));
        return QED_ERR_HIP;
    }
    return QED_OK;
}
