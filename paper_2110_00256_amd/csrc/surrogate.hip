// Learned inverse-CDF surrogate: training-set generation from the tables,
// BF16-MFMA forward/backward training kernels, Adam, batched inference,
// and the host side of the qed_surrogate_* C ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "device_physics.hpp"
#include "internal.hpp"
#include "surrogate.hpp"
#include "surrogate_api.hpp"

using namespace qedmi;

struct qed_surrogate {
    int device = -1;
    qed_surrogate_cfg cfg{};
    TableDev table{};            // fallback / training table view (device)
    float* d_p = nullptr;        // FP32 master parameters
    float* d_m = nullptr;        // Adam first moment
    float* d_v = nullptr;        // Adam second moment
    uint16_t* d_w2 = nullptr;    // BF16 copy of W2
    unsigned long long band_mask = ~0ULL;   // bands the network serves (all until validated)
    float band_err[kSurrBands] = {};        // largest CDF-space error found per band
    bool validated = false;
    SurrogateDev view() const {
        SurrogateDev s{};
        s.p = d_p;
        s.w2 = d_w2;
        s.process = cfg.process;
        const double l0 = std::log(cfg.chi_lo), l1 = std::log(cfg.chi_hi);
        s.mid = static_cast<float>(0.5 * (l0 + l1));
        s.inv_half = static_cast<float>(2.0 / (l1 - l0));
        s.chi_lo = static_cast<float>(cfg.chi_lo);
        s.chi_hi = static_cast<float>(cfg.chi_hi);
        s.probe_tol = cfg.probe_tol;
        s.probe_every = cfg.probe_every > 0 ? cfg.probe_every : 1;
        s.band_mask = band_mask;
        s.ln_chi_lo = static_cast<float>(l0);
        s.band_inv_w = static_cast<float>(kSurrBands / (l1 - l0));
        return s;
    }
};

namespace qedmi {

constexpr unsigned long long kTrainStep = 0x5452414E494E4700ULL;   // draw stream of the training set

// ------------------------------------------------------------ training set
// Sample i: chi log-uniform over the given range, u uniform over the
// network's input domain, target from the FP64 table inverse CDF (Sec. 3.1 /
// 3.2), weight (du/dy)^2 with y the sampled quantity in the network's output
// units, so that the loss measures error in CDF space (the
// quantity a KS distance sees).
__device__ __forceinline__ double surr_target(const TableDev& t, int process, double chi, double u) {
    if (process == 1) {
        const double lx = dev::sample_qs_lnxi<double>(t, chi, u);
        const double lny = lx - log(1.5 * chi) - log1p(-exp(lx));
        return lny - 3.0 * log(u);
    }
    bool e;
    const double xi = dev::sample_bw<double>(t, chi, u, e);
    const double sc = sqrt(3.0 * chi) * 0.125;
    return (0.5 - xi) / (sc / (1.0 + 2.0 * sc));
}

__global__ void __launch_bounds__(256) surr_make_set(TableDev t, SurrogateDev s, unsigned long long seed, int n,
                                                     double ln_lo, double ln_hi, double tail_frac, float4* out) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const dev::Draws d = dev::draws(seed, static_cast<unsigned long long>(i), kTrainStep,
                                        static_cast<unsigned long long>(s.process), 0ULL);
        const double chi = exp(ln_lo + (ln_hi - ln_lo) * d.u[0]);
        double u;
        if (d.u[2] < tail_frac) {
            // even in the network's second input x1 over [-1, 1]
            const double x1 = 2.0 * d.u[1] - 1.0;
            if (s.process == 1) {
                const double logit = kSurrLogitMid + x1 / kSurrLogitInvHalf;
                u = fmin(fmax(1.0 / (1.0 + exp(-logit)), kSurrUMin), static_cast<double>(kSurrUMaxQs));
            } else {
                const double q = 0.5 * (x1 - 1.0) * kBwQMin;          // Phi^{-1}(r) in [-qmin, 0]
                u = fmin(fmax(0.5 * erfc(-q * 0.70710678118654752), kSurrUMin), 0.5);
            }
        } else if (s.process == 1) {
            u = kSurrUMin + (static_cast<double>(kSurrUMaxQs) - kSurrUMin) * d.u[1];
        } else {
            u = kSurrUMin + (0.5 - kSurrUMin) * d.u[1];
        }
        const double tgt = surr_target(t, s.process, chi, u);
        // slope of the sampled quantity itself (QS: ln Y = target + 3 ln u;
        // BW: the target is linear in xi), so that w (dy)^2 = (du)^2
        const double h = 1e-6 * (s.process == 1 ? fmin(u, 1.0 - u) : u) + 1e-12;
        const double ua = fmax(u - h, 1e-15), ub = fmin(u + h, 1.0 - 1e-15);
        double ta = surr_target(t, s.process, chi, ua), tb = surr_target(t, s.process, chi, ub);
        if (s.process == 1) {
            ta += 3.0 * log(ua);
            tb += 3.0 * log(ub);
        }
        const double slope = fabs(tb - ta) / (ub - ua);
        const double w = 1.0 / fmax(slope * slope, 1e-2);
        float x0, x1;
        surr_features(s, static_cast<float>(chi), static_cast<float>(u), x0, x1);
        out[i] = make_float4(x0, x1, static_cast<float>(tgt), static_cast<float>(w));
    }
}

// ------------------------------------------------------------ training step
// Loss 0.5 * sum_i w_i (y_i - t_i)^2 / n over the minibatch.  Each wave
// takes 16-sample tiles of its slice and accumulates a full gradient; per
// wave partials go to part[wave][kNParam + 1] (last slot: loss), reduced in
// a fixed order by the update kernel, so training is deterministic.
__global__ void __launch_bounds__(256) surr_train_kernel(SurrogateDev s, const float4* set, long long first,
                                                         long long set_n, int batch, float* part) {
    __shared__ float lds_dz[4][16][65];
    const int lane = static_cast<int>(__lane_id());
    const int col = lane & 15, grp = lane >> 4;
    const int wave = threadIdx.x >> 6;
    const int wave_global = blockIdx.x * 4 + wave;
    const int n_waves = gridDim.x * 4;
    const int per_wave = batch / n_waves;   // multiple of 16 (host checks)
    const float* p = s.p;
    const float inv_b = 1.0f / static_cast<float>(batch);

    surr_v4s bw2[4][4];   // forward: B[k][n] = W2[n][k]
    surr_v4s bw2t[4][4];  // backward dh1: B[kk = n][col = k] = W2[n][k]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            bw2[nt][ks] = *reinterpret_cast<const surr_v4s*>(s.w2 + (nt * 16 + col) * 64 + ks * 16 + 4 * grp);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                bw2t[nt][ks][e] = static_cast<short>(s.w2[(ks * 16 + 4 * grp + e) * 64 + nt * 16 + col]);
        }
    float b2[4], w3[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        b2[nt] = p[kOffB2 + nt * 16 + col];
        w3[nt] = p[kOffW3 + nt * 16 + col];
    }
    const float b3 = p[kOffB3];

    surr_v4f gw2[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) gw2[a][b] = surr_v4f{0.f, 0.f, 0.f, 0.f};
    float gw1a[4] = {0, 0, 0, 0}, gw1b[4] = {0, 0, 0, 0}, gb1[4] = {0, 0, 0, 0};
    float gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0}, gb3 = 0.f, loss = 0.f;

    for (int tile = 0; tile < per_wave / 16; ++tile) {
        const long long base = first + static_cast<long long>(wave_global) * per_wave + tile * 16;
        // forward, A layout: sample col, units k = ks*16 + 4 grp + e
        const float4 me = set[(base + col) % set_n];
        surr_v4s a[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = ks * 16 + 4 * grp + e;
                a[ks][e] = surr_bf16(surr_silu(p[kOffW1 + 2 * k] * me.x + p[kOffW1 + 2 * k + 1] * me.y + p[kOffB1 + k]));
            }
        // this lane's four samples in C layout: rows 4 grp + e
        float4 cs[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) cs[e] = set[(base + 4 * grp + e) % set_n];
        float z2[4][4], yp[4] = {0, 0, 0, 0};
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            surr_v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[ks], bw2[nt][ks], acc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                z2[nt][e] = acc[e] + b2[nt];
                yp[e] += w3[nt] * surr_silu(z2[nt][e]);
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) yp[e] += __shfl_xor(yp[e], o);
        float dy[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float r = yp[e] + b3 - cs[e].z;
            dy[e] = cs[e].w * r * inv_b;
            if (col == 0) {
                loss += 0.5f * cs[e].w * r * r * inv_b;
                gb3 += dy[e];
            }
        }
        // output layer and dz2 (C layout)
        float dz2[4][4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                gw3[nt] += dy[e] * surr_silu(z2[nt][e]);
                dz2[nt][e] = dy[e] * w3[nt] * surr_dsilu(z2[nt][e]);
                gb2[nt] += dz2[nt][e];
            }
        // h1 in C layout (sample 4 grp + e, unit kt*16 + col), recomputed
        float z1c[4][4];
        surr_v4s bh1[4];
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            const int k = kt * 16 + col;
            const float wa = p[kOffW1 + 2 * k], wb = p[kOffW1 + 2 * k + 1], bb = p[kOffB1 + k];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                z1c[kt][e] = wa * cs[e].x + wb * cs[e].y + bb;
                bh1[kt][e] = surr_bf16(surr_silu(z1c[kt][e]));
            }
        }
        // dW2[n][k] += sum_s dz2[s][n] h1[s][k]:  M = n, N = k, K = 16 samples
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            surr_v4s adz;
#pragma unroll
            for (int e = 0; e < 4; ++e) adz[e] = surr_bf16(dz2[mt][e]);
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) gw2[mt][kt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(adz, bh1[kt], gw2[mt][kt], 0, 0, 0);
        }
        // dh1[s][k] = sum_n dz2[s][n] W2[n][k]: A needs dz2 with the sample
        // along lanes -> transpose through LDS
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int e = 0; e < 4; ++e) lds_dz[wave][4 * grp + e][nt * 16 + col] = dz2[nt][e];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        surr_v4s adt[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int e = 0; e < 4; ++e) adt[ks][e] = surr_bf16(lds_dz[wave][col][ks * 16 + 4 * grp + e]);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            surr_v4f dh = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) dh = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(adt[ks], bw2t[kt][ks], dh, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float dz1 = dh[e] * surr_dsilu(z1c[kt][e]);
                gw1a[kt] += dz1 * cs[e].x;
                gw1b[kt] += dz1 * cs[e].y;
                gb1[kt] += dz1;
            }
        }
    }
    // reduce the four lane groups (same unit, different samples)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
#pragma unroll
        for (int o = 16; o < 64; o <<= 1) {
            gw1a[kt] += __shfl_xor(gw1a[kt], o);
            gw1b[kt] += __shfl_xor(gw1b[kt], o);
            gb1[kt] += __shfl_xor(gb1[kt], o);
            gb2[kt] += __shfl_xor(gb2[kt], o);
            gw3[kt] += __shfl_xor(gw3[kt], o);
        }
    }
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
        gb3 += __shfl_xor(gb3, o);
        loss += __shfl_xor(loss, o);
    }
    float* out = part + static_cast<size_t>(wave_global) * (kNParam + 1);
    if (grp == 0) {
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            const int k = kt * 16 + col;
            out[kOffW1 + 2 * k] = gw1a[kt];
            out[kOffW1 + 2 * k + 1] = gw1b[kt];
            out[kOffB1 + k] = gb1[kt];
            out[kOffB2 + k] = gb2[kt];
            out[kOffW3 + k] = gw3[kt];
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int e = 0; e < 4; ++e) out[kOffW2 + (mt * 16 + 4 * grp + e) * 64 + kt * 16 + col] = gw2[mt][kt][e];
    if (lane == 0) {
        out[kOffB3] = gb3;
        out[kNParam] = loss;
    }
}

// Sum the wave partials in a fixed order; Adam step (or plain reduction to
// `grad_out` when it is non-null); refresh the BF16 copy of W2.
__global__ void __launch_bounds__(256) surr_update_kernel(float* params, float* m, float* v, uint16_t* w2, const float* part,
                                                          int n_waves, float lr, float b1t, float b2t, float* grad_out,
                                                          float* loss_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kNParam) return;
    // the partials are added in wave order (deterministic); loads go out 64
    // at a time so that one memory latency covers 64 of them
    constexpr int kGroup = 64;
    float g = 0.f;
    int w = 0;
    for (; w + kGroup <= n_waves; w += kGroup) {
        float t[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) t[q] = part[static_cast<size_t>(w + q) * (kNParam + 1) + i];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) g += t[q];
    }
    for (; w < n_waves; ++w) g += part[static_cast<size_t>(w) * (kNParam + 1) + i];
    if (i == kNParam) {
        if (loss_out) *loss_out = g;
        return;
    }
    if (grad_out) {
        grad_out[i] = g;
        return;
    }
    constexpr float kB1 = 0.9f, kB2 = 0.999f, kEps = 1e-8f;
    const float mi = kB1 * m[i] + (1.f - kB1) * g;
    const float vi = kB2 * v[i] + (1.f - kB2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.f - b1t), vh = vi / (1.f - b2t);
    const float pi = params[i] - lr * mh / (sqrtf(vh) + kEps);
    params[i] = pi;
    if (i >= kOffW2 && i < kOffW2 + 4096) w2[i - kOffW2] = static_cast<uint16_t>(surr_bf16(pi));
}

__global__ void __launch_bounds__(256) surr_refresh_w2(const float* params, uint16_t* w2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4096) w2[i] = static_cast<uint16_t>(surr_bf16(params[kOffW2 + i]));
}

// Forward on raw network inputs x[n][2] (FP32) -> y[n].
__global__ void __launch_bounds__(256) surr_forward_kernel(SurrogateDev s, const float* x, float* y, long long n) {
    const int wave = threadIdx.x >> 6, lane = static_cast<int>(__lane_id());
    for (long long b = (static_cast<long long>(blockIdx.x) * 4 + wave) * 64; b < n;
         b += static_cast<long long>(gridDim.x) * 256) {
        const long long i = b + lane;
        const bool ok = i < n;
        const float x0 = ok ? x[2 * i] : 0.f, x1 = ok ? x[2 * i + 1] : 0.f;
        const float out = surr_forward_wave(s, x0, x1);
        if (ok) y[i] = out;
    }
}

// The table's cumulative distribution at a sample (QS: ln xi; BW: xi in
// [0, 1/2]) for the row interpolated at chi, in FP64: the exact inverse of
// the table sampler (rows interpolated in ln chi, then linear in ln xi for
// QS with the small-xi law below the first knot, linear in xi for BW).
__device__ double table_cdf_at(const TableDev& t, int process, double chi, double sample) {
    int n;
    double f;
    dev::row_pos<double>(t, chi, n, f);
    const int nf = t.n_frac;
    const double* pp = t.cdf64 + 2 * static_cast<size_t>(n) * nf;
    if (process == 1) {
        const double lmin = t.ln_frac_min;
        const double x = (sample - lmin) * (nf - 1) / (-lmin);
        if (x < 0.0) return exp(dev::pair_value<double, double>(pp, f, 0) + (sample - lmin) / 3.0);
        if (x >= nf - 1) return 1.0;
        const int m = static_cast<int>(x);
        const double la = dev::pair_value<double, double>(pp, f, m), lb = dev::pair_value<double, double>(pp, f, m + 1);
        return exp(la + (x - m) * (lb - la));
    }
    const double x = fmin(fmax(sample, 0.0), 0.5) * (nf - 1) / 0.5;
    const int m = min(static_cast<int>(x), nf - 2);
    const double pa = dev::pair_value<double, double>(pp, f, m), pb = dev::pair_value<double, double>(pp, f, m + 1);
    return pa + (x - m) * (pb - pa);
}

constexpr int kValChiPerBand = 8;   // chi points per band, both band edges included
constexpr int kValU = 4096;         // uniforms per chi point: half even in x1, half even in u

// Validation: for each (band, chi point) block, the largest |F_table(network
// sample) - u| over kValU uniforms of the network's domain.  For a monotone
// map this is the Kolmogorov-Smirnov distance between the network's and the
// table's sampled spectra at that chi.  Block maxima go to band_err (as
// ordered bit patterns of non-negative floats).
__global__ void __launch_bounds__(256) surr_validate_kernel(SurrogateDev s, TableDev t, double ln_lo, double ln_hi,
                                                            unsigned* band_err) {
    __shared__ float s_max[4];
    const int band = blockIdx.x / kValChiPerBand, cj = blockIdx.x % kValChiPerBand;
    const int wave = threadIdx.x >> 6, lane = static_cast<int>(__lane_id());
    const double lc = ln_lo + (ln_hi - ln_lo) * (band + cj / static_cast<double>(kValChiPerBand - 1)) / kSurrBands;
    const float chi = fminf(fmaxf(static_cast<float>(exp(lc)), s.chi_lo), s.chi_hi);
    const double u_hi = s.process == 1 ? static_cast<double>(kSurrUMaxQs) : 0.5;
    float worst = 0.0f;
    for (int i0 = wave * 64; i0 < kValU; i0 += 256) {
        const int i = i0 + lane;
        double u;
        if (i < kValU / 2) {
            const double x1 = -1.0 + 2.0 * (i + 0.5) / (kValU / 2);
            if (s.process == 1) u = 1.0 / (1.0 + exp(-(kSurrLogitMid + x1 / kSurrLogitInvHalf)));
            else u = 0.5 * erfc(-0.5 * (x1 - 1.0) * kBwQMin * 0.70710678118654752);
        } else {
            u = kSurrUMin + (u_hi - kSurrUMin) * ((i - kValU / 2) + 0.5) / (kValU / 2);
        }
        const float uf = fminf(fmaxf(static_cast<float>(u), kSurrUMin), static_cast<float>(u_hi));
        float x0, x1f;
        surr_features(s, chi, uf, x0, x1f);
        const float y = surr_forward_wave(s, x0, x1f);
        const float smp = surr_output(s, chi, uf, y);
        const double err = fabs(table_cdf_at(t, s.process, chi, smp) - static_cast<double>(uf));
        worst = fmaxf(worst, static_cast<float>(err));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) worst = fmaxf(worst, __shfl_xor(worst, o));
    if (lane == 0) s_max[wave] = worst;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float m = fmaxf(fmaxf(s_max[0], s_max[1]), fmaxf(s_max[2], s_max[3]));
        atomicMax(band_err + band, __float_as_uint(m));
    }
}

// Sampling for (chi, u) arrays: surrogate inside its domain, table outside.
__global__ void __launch_bounds__(256) surr_sample_kernel(SurrogateDev s, TableDev t, const float* chi, const float* u,
                                                          float* out, long long n) {
    const int wave = threadIdx.x >> 6, lane = static_cast<int>(__lane_id());
    for (long long b = (static_cast<long long>(blockIdx.x) * 4 + wave) * 64; b < n;
         b += static_cast<long long>(gridDim.x) * 256) {
        const long long i = b + lane;
        const bool valid = i < n;
        const float c = valid ? chi[i] : 1.f, r = valid ? u[i] : 0.5f;
        float x0 = 0.f, x1 = 0.f;
        const bool inside = valid && surr_inputs(s, c, r, x0, x1);
        const float yv = surr_forward_wave(s, x0, x1);
        if (!valid) continue;
        float res;
        if (inside) {
            res = surr_output(s, c, r, yv);
        } else if (s.process == 1) {
            res = dev::sample_qs_lnxi<float>(t, c, r);
        } else {
            bool e;
            res = dev::sample_bw<float>(t, c, r, e);
        }
        out[i] = res;
    }
}

}  // namespace qedmi

// ---------------------------------------------------------------- host side
namespace {

int32_t hfail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return QED_ERR_HIP;
}

bool check_cfg(const qed_table* t, const qed_surrogate_cfg* c) {
    if (!t || !c) { set_error("table/cfg is null"); return false; }
    if (c->process != t->p.process) { set_error("cfg.process differs from the table's"); return false; }
    if (!(c->chi_lo > 0) || !(c->chi_hi > c->chi_lo)) { set_error("need 0 < chi_lo < chi_hi"); return false; }
    if (c->chi_lo < t->p.chi_min || c->chi_hi > t->p.chi_max) {
        set_error("trained chi range must lie inside the table range");
        return false;
    }
    return true;
}

qed_surrogate* alloc_surrogate(const qed_table* t, const qed_surrogate_cfg* c) {
    qed_surrogate* s = new (std::nothrow) qed_surrogate;
    if (!s) return nullptr;
    s->cfg = *c;
    s->table = t->view();
    hipGetDevice(&s->device);
    if (hipMalloc(&s->d_p, sizeof(float) * kNParam) != hipSuccess ||
        hipMalloc(&s->d_m, sizeof(float) * kNParam) != hipSuccess ||
        hipMalloc(&s->d_v, sizeof(float) * kNParam) != hipSuccess ||
        hipMalloc(&s->d_w2, sizeof(uint16_t) * 4096) != hipSuccess) {
        qed_surrogate_destroy(s);
        return nullptr;
    }
    return s;
}

// Deterministic host initialisation (uniform, fan-in scaled; splitmix64).
void init_params(std::vector<float>& p, uint64_t seed) {
    uint64_t st = seed ^ 0x9E3779B97F4A7C15ULL;
    auto next = [&]() {
        st += 0x9E3779B97F4A7C15ULL;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        return (static_cast<double>(z >> 11) + 0.5) * 0x1.0p-53 * 2.0 - 1.0;
    };
    p.assign(kNParam, 0.f);
    for (int i = 0; i < 128; ++i) p[kOffW1 + i] = static_cast<float>(1.5 * next());
    for (int i = 0; i < 64; ++i) p[kOffB1 + i] = static_cast<float>(1.5 * next());
    for (int i = 0; i < 4096; ++i) p[kOffW2 + i] = static_cast<float>(next() * std::sqrt(6.0 / 128.0));
    for (int i = 0; i < 64; ++i) p[kOffW3 + i] = static_cast<float>(next() * std::sqrt(6.0 / 65.0));
}

// Validate the network band by band against the table (when the cfg sets a
// budget): a band is served by the network only if its largest CDF-space
// error over the validation points is within ks_budget.  Synchronous.
int32_t validate_bands(qed_surrogate* s, hipStream_t st) {
    s->band_mask = ~0ULL;
    s->validated = false;
    for (float& x : s->band_err) x = 0.f;
    if (!(s->cfg.ks_budget > 0.f)) return QED_OK;
    unsigned* d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(unsigned) * kSurrBands);
    if (e != hipSuccess) { set_error("validation buffer: allocation failed"); return QED_ERR_ALLOC; }
    e = hipMemsetAsync(d, 0, sizeof(unsigned) * kSurrBands, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(surr_validate_kernel, dim3(kSurrBands * kValChiPerBand), dim3(256), 0, st, s->view(),
                           s->table, std::log(s->cfg.chi_lo), std::log(s->cfg.chi_hi), d);
        e = hipGetLastError();
    }
    unsigned h[kSurrBands] = {};
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(d);
    if (e != hipSuccess) return hfail(e, "band validation");
    unsigned long long mask = 0ULL;
    for (int b = 0; b < kSurrBands; ++b) {
        float v;
        std::memcpy(&v, &h[b], sizeof v);
        s->band_err[b] = v;
        if (v <= s->cfg.ks_budget) mask |= 1ULL << b;
    }
    s->band_mask = mask;
    s->validated = true;
    return QED_OK;
}

}  // namespace

namespace qedmi {
int32_t surrogate_bind(StepArgs& a, const qed_surrogate* bw, const qed_surrogate* qs) {
    a.use_bw_surr = 0;
    a.use_qs_surr = 0;
    if (bw) {
        if (bw->cfg.process != QED_PROC_BW) { set_error("bw_surrogate is not a BW surrogate"); return QED_ERR_INVALID; }
        a.bw_surr = bw->view();
        a.use_bw_surr = 1;
    }
    if (qs) {
        if (qs->cfg.process != QED_PROC_QS) { set_error("qs_surrogate is not a QS surrogate"); return QED_ERR_INVALID; }
        a.qs_surr = qs->view();
        a.use_qs_surr = 1;
    }
    return QED_OK;
}
}  // namespace qedmi

extern "C" int32_t qed_surrogate_from_host(const qed_table* table, const qed_surrogate_cfg* cfg, const float* params,
                                           qed_surrogate** out) {
    if (!out) { set_error("out is null"); return QED_ERR_INVALID; }
    *out = nullptr;
    if (!check_cfg(table, cfg)) return QED_ERR_INVALID;
    if (!params) { set_error("params is null"); return QED_ERR_INVALID; }
    if (table->device < 0) { set_error("table is not on the device"); return QED_ERR_STATE; }
    qed_surrogate* s = alloc_surrogate(table, cfg);
    if (!s) { set_error("surrogate allocation failed"); return QED_ERR_ALLOC; }
    hipError_t e = hipMemcpy(s->d_p, params, sizeof(float) * kNParam, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s->d_m, 0, sizeof(float) * kNParam);
    if (e == hipSuccess) e = hipMemset(s->d_v, 0, sizeof(float) * kNParam);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(surr_refresh_w2, dim3(16), dim3(256), 0, 0, s->d_p, s->d_w2);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        qed_surrogate_destroy(s);
        return hfail(e, "surrogate upload");
    }
    const int32_t r = validate_bands(s, nullptr);
    if (r != QED_OK) {
        qed_surrogate_destroy(s);
        return r;
    }
    *out = s;
    return QED_OK;
}

extern "C" int32_t qed_surrogate_train(qed_context* ctx, const qed_table* table, const qed_surrogate_cfg* cfg,
                                       qed_surrogate** out, float* final_loss, void* stream) {
    if (!out) { set_error("out is null"); return QED_ERR_INVALID; }
    *out = nullptr;
    if (!ctx) { set_error("context is null"); return QED_ERR_INVALID; }
    if (!check_cfg(table, cfg)) return QED_ERR_INVALID;
    if (table->device < 0 || !table->d_cdf64) { set_error("table is not on the device"); return QED_ERR_STATE; }
    const int n_blocks = 64, n_waves = n_blocks * 4;
    if (cfg->batch <= 0 || cfg->batch % (16 * n_waves) != 0) {
        set_error("batch must be a positive multiple of 4096");
        return QED_ERR_INVALID;
    }
    if (cfg->n_samples < cfg->batch || cfg->steps <= 0 || !(cfg->lr > 0)) {
        set_error("need n_samples >= batch, steps > 0, lr > 0");
        return QED_ERR_INVALID;
    }
    std::vector<float> init;
    init_params(init, cfg->seed);
    qed_surrogate* s = nullptr;
    int32_t r = qed_surrogate_from_host(table, cfg, init.data(), &s);
    if (r) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float4* set = nullptr;
    float* part = nullptr;
    float* losses = nullptr;
    hipError_t e = hipMalloc(&set, sizeof(float4) * static_cast<size_t>(cfg->n_samples));
    if (e == hipSuccess) e = hipMalloc(&part, sizeof(float) * (kNParam + 1) * n_waves);
    if (e == hipSuccess) e = hipMalloc(&losses, sizeof(float) * cfg->steps);
    if (e != hipSuccess) {
        hipFree(set);
        hipFree(part);
        hipFree(losses);
        qed_surrogate_destroy(s);
        set_error("training buffers: allocation failed");
        return QED_ERR_ALLOC;
    }
    const SurrogateDev v = s->view();
    // the training set reaches 1/16 of the log range beyond each end of the
    // domain the network serves, so that its ends are fitted like its middle
    const double ln_lo = std::log(cfg->chi_lo), ln_hi = std::log(cfg->chi_hi);
    const double margin = (ln_hi - ln_lo) / 16.0;
    hipLaunchKernelGGL(surr_make_set, dim3(2048), dim3(256), 0, st, table->view(), v, cfg->seed, cfg->n_samples,
                       ln_lo - margin, ln_hi + margin, std::min(std::max(cfg->tail_permille, 0), 1000) * 1e-3,
                       set);
    e = hipGetLastError();
    double b1t = 1.0, b2t = 1.0;
    for (int it = 0; it < cfg->steps && e == hipSuccess; ++it) {
        const long long first = (static_cast<long long>(it) * cfg->batch) % cfg->n_samples;
        hipLaunchKernelGGL(surr_train_kernel, dim3(n_blocks), dim3(256), 0, st, v, set, first,
                           static_cast<long long>(cfg->n_samples), cfg->batch, part);
        b1t *= 0.9;
        b2t *= 0.999;
        // cosine decay from lr to lr / 100
        const double frac = static_cast<double>(it) / cfg->steps;
        const float lr = static_cast<float>(cfg->lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(3.141592653589793 * frac))));
        hipLaunchKernelGGL(surr_update_kernel, dim3((kNParam + 256) / 256), dim3(256), 0, st, s->d_p, s->d_m, s->d_v,
                           s->d_w2, part, n_waves, lr, static_cast<float>(b1t), static_cast<float>(b2t), nullptr,
                           losses + it);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && final_loss) {
        const int k = std::min(64, cfg->steps);
        std::vector<float> tail(k);
        e = hipMemcpy(tail.data(), losses + cfg->steps - k, sizeof(float) * k, hipMemcpyDeviceToHost);
        double acc = 0;
        for (float x : tail) acc += x;
        *final_loss = static_cast<float>(acc / k);
    }
    hipFree(set);
    hipFree(part);
    hipFree(losses);
    if (e != hipSuccess) {
        qed_surrogate_destroy(s);
        return hfail(e, "surrogate training");
    }
    const int32_t rv = validate_bands(s, st);
    if (rv != QED_OK) {
        qed_surrogate_destroy(s);
        return rv;
    }
    *out = s;
    return QED_OK;
}

extern "C" int32_t qed_surrogate_bands(const qed_surrogate* s, float* band_err, uint64_t* served_mask) {
    if (!s || !band_err || !served_mask) { set_error("surrogate/band_err/served_mask is null"); return QED_ERR_INVALID; }
    for (int b = 0; b < kSurrBands; ++b) band_err[b] = s->band_err[b];
    *served_mask = s->band_mask;
    return QED_OK;
}

extern "C" int32_t qed_surrogate_get_params(const qed_surrogate* s, float* host_params) {
    if (!s || !host_params) { set_error("surrogate/params is null"); return QED_ERR_INVALID; }
    const hipError_t e = hipMemcpy(host_params, s->d_p, sizeof(float) * kNParam, hipMemcpyDeviceToHost);
    return e == hipSuccess ? QED_OK : hfail(e, "parameter readback");
}

extern "C" int32_t qed_surrogate_forward(const qed_surrogate* s, const float* x, float* y, int64_t n, void* stream) {
    if (!s) { set_error("surrogate is null"); return QED_ERR_INVALID; }
    if (n < 0) { set_error("n < 0"); return QED_ERR_INVALID; }
    if (n == 0) return QED_OK;
    if (!x || !y) { set_error("x/y is null"); return QED_ERR_INVALID; }
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(surr_forward_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), s->view(), x, y, static_cast<long long>(n));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? QED_OK : hfail(e, "forward launch");
}

extern "C" int32_t qed_surrogate_grad(const qed_surrogate* s, const float* x, const float* t, int64_t n, float* grad,
                                      float* loss, void* stream) {
    if (!s || !x || !t || !grad || !loss) { set_error("null argument"); return QED_ERR_INVALID; }
    const int n_blocks = 1, n_waves = 4;
    if (n <= 0 || n % (16 * n_waves) != 0 || n > (1 << 24)) {
        set_error("n must be a positive multiple of 64 (at most 2^24)");
        return QED_ERR_INVALID;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    float4* set = nullptr;
    float* part = nullptr;
    hipError_t e = hipMalloc(&set, sizeof(float4) * n);
    if (e == hipSuccess) e = hipMalloc(&part, sizeof(float) * (kNParam + 1) * n_waves);
    std::vector<float> hx(2 * n), ht(n);
    if (e == hipSuccess) e = hipMemcpyAsync(hx.data(), x, sizeof(float) * 2 * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ht.data(), t, sizeof(float) * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
        std::vector<float> packed(4 * n);
        for (int64_t i = 0; i < n; ++i) {
            packed[4 * i] = hx[2 * i];
            packed[4 * i + 1] = hx[2 * i + 1];
            packed[4 * i + 2] = ht[i];
            packed[4 * i + 3] = 1.0f;
        }
        e = hipMemcpy(set, packed.data(), sizeof(float4) * n, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(surr_train_kernel, dim3(n_blocks), dim3(256), 0, st, s->view(), set, 0LL,
                           static_cast<long long>(n), static_cast<int>(n), part);
        hipLaunchKernelGGL(surr_update_kernel, dim3((kNParam + 256) / 256), dim3(256), 0, st, s->d_p, s->d_m, s->d_v,
                           s->d_w2, part, n_waves, 0.f, 1.f, 1.f, grad, loss);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(set);
    hipFree(part);
    return e == hipSuccess ? QED_OK : hfail(e, "gradient");
}

extern "C" int32_t qed_surrogate_sample(const qed_surrogate* s, const float* chi, const float* u, float* out, int64_t n,
                                        void* stream) {
    if (!s) { set_error("surrogate is null"); return QED_ERR_INVALID; }
    if (n < 0) { set_error("n < 0"); return QED_ERR_INVALID; }
    if (n == 0) return QED_OK;
    if (!chi || !u || !out) { set_error("null array"); return QED_ERR_INVALID; }
    const long long blocks = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(surr_sample_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), s->view(), s->table, chi, u, out, static_cast<long long>(n));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? QED_OK : hfail(e, "sample launch");
}

extern "C" void qed_surrogate_destroy(qed_surrogate* s) {
    if (!s) return;
    hipFree(s->d_p);
    hipFree(s->d_m);
    hipFree(s->d_v);
    hipFree(s->d_w2);
    delete s;
}
