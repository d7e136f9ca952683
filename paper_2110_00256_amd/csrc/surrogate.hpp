// Learned inverse-CDF surrogate: an MLP 2 -> 64 -> 64 -> 1 with SiLU
// activations.  The 64 x 64 hidden layer runs on BF16 MFMA with FP32
// accumulation (v_mfma_f32_16x16x16_bf16, 64-sample tiles per wave); the
// 2 -> 64 input layer and the 64 -> 1 output layer are FP32 VALU work (K = 2
// and N = 1 are not matrix shapes).  It replaces the 2D table inverse CDF of
// paper Sec. 3.1 / 3.2 inside the trained chi range; the table remains the
// fallback.
//
// Input / output maps (shared by training targets and inference):
//   x0 = (ln chi - mid) / half, mid/half of ln chi over the trained range.
//   QS: x1 = logit(u) scaled to [-1, 1]; output y -> ln Y = y + 3 ln u with
//       Y = 2 xi / (3 chi (1 - xi)) (the argument of the Bessel functions of
//       Sec. 2.2; the cube term is the small-xi law P ~ xi^{1/3}), so
//       xi = k Y / (1 + k Y), k = 3 chi / 2.
//   BW: r = min(u, 1 - u) (the fold of Sec. 3.1); x1 = 1 + 2 q / |q(u_min)|
//       with q = Phi^{-1}(r) the standard-normal quantile; output y -> xi =
//       1/2 - sigma(chi) y, sigma = s / (1 + 2 s), s = sqrt(3 chi)/8 (the
//       small-chi width of the pair spectrum about xi = 1/2).
//   Outside [chi_lo, chi_hi] or for u (r) below u_min the table is used.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qedmi {

constexpr int kHidden = 64;
constexpr int kNParam = 64 * 2 + 64 + 64 * 64 + 64 + 64 + 1;   // 4417
constexpr int kOffW1 = 0, kOffB1 = 128, kOffW2 = 192, kOffB2 = 192 + 4096, kOffW3 = kOffB2 + 64,
              kOffB3 = kOffW3 + 64;
constexpr float kSurrUMin = 1e-4f;
constexpr int kSurrBands = 64;
constexpr float kBwQMin = 3.7190165f;   // -Phi^{-1}(1e-4)

struct SurrogateDev {
    const float* p;          // FP32 master parameters (layout above)
    const uint16_t* w2;      // BF16 copy of W2, [n][k] row-major
    int32_t process;         // 0 BW, 1 QS
    float mid, inv_half;     // x0 = (ln chi - mid) * inv_half
    float chi_lo, chi_hi;
    float probe_tol;
    int32_t probe_every;     // probe one wave batch in this many (>= 1)
    // served bands: the trained range split into kSurrBands equal bands in
    // ln chi; bit b set: band b is sampled by the network, else by the table
    unsigned long long band_mask;
    float ln_chi_lo, band_inv_w;   // b = floor((ln chi - ln_chi_lo) * band_inv_w)
};

typedef short surr_v4s __attribute__((ext_vector_type(4)));
typedef float surr_v4f __attribute__((ext_vector_type(4)));

// SiLU and its derivative with the hardware reciprocal (1 ulp) in place of
// an IEEE division: the activation is two transcendental instructions.
__device__ __forceinline__ float surr_sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float surr_silu(float z) { return z * surr_sigmoid(z); }
__device__ __forceinline__ float surr_dsilu(float z) {
    const float s = surr_sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

// FP32 -> BF16 bits, round to nearest even.
__device__ __forceinline__ short surr_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<short>(u >> 16);
}

__device__ __forceinline__ float surr_ndtri_lower(float r) {
    // Phi^{-1}(r) = -sqrt(2) erfcinv(2 r)
    return -1.41421356237f * erfcinvf(2.0f * r);
}

constexpr float kSurrUMaxQs = 1.0f - 1e-5f;   // above: the hard-photon tail goes to the table
// logit(u) = ln u - ln(1 - u) spans [-9.21024, 11.51292] over [1e-4, 1 - 1e-5]
constexpr float kSurrLogitMid = 1.15134f;
constexpr float kSurrLogitInvHalf = 1.0f / 10.36158f;

// Network features for (chi, u) without domain checks.
__device__ __forceinline__ void surr_features(const SurrogateDev& s, float chi, float u, float& x0, float& x1) {
    x0 = (logf(chi) - s.mid) * s.inv_half;
    if (s.process == 1) {
        // logit of u over [1e-4, 1 - 1e-5] -> [-1, 1]: resolves both the
        // soft end (xi ~ u^3) and the hard tail, where ln Y grows like
        // -ln(1 - u)
        x1 = (logf(u) - log1pf(-u) - kSurrLogitMid) * kSurrLogitInvHalf;
    } else {
        const float r = u <= 0.5f ? u : 1.0f - u;
        x1 = 1.0f + 2.0f * surr_ndtri_lower(r) / kBwQMin;
    }
}

// chi inside the trained range and in a band the network serves?
__device__ __forceinline__ bool surr_serves_chi(const SurrogateDev& s, float chi) {
    if (!(chi >= s.chi_lo && chi <= s.chi_hi)) return false;
    const int band = min(kSurrBands - 1, max(0, static_cast<int>((logf(chi) - s.ln_chi_lo) * s.band_inv_w)));
    return (s.band_mask >> band) & 1ULL;
}

// Inside the trained domain?  (Otherwise the table is used.)
__device__ __forceinline__ bool surr_inside(const SurrogateDev& s, float chi, float u) {
    if (!surr_serves_chi(s, chi)) return false;
    if (s.process == 1) return u >= kSurrUMin && u <= kSurrUMaxQs;
    const float r = u <= 0.5f ? u : 1.0f - u;
    return r >= kSurrUMin;
}

// Network inputs for (chi, u); returns false if the table must be used.
__device__ __forceinline__ bool surr_inputs(const SurrogateDev& s, float chi, float u, float& x0, float& x1) {
    if (!surr_inside(s, chi, u)) return false;
    surr_features(s, chi, u, x0, x1);
    return true;
}

// The network's target for a sample xi of the table (QS: ln xi given), in
// the output space used by training and by the per-batch probe.
__device__ __forceinline__ float surr_target_of(int process, float chi, float u, float sample) {
    if (process == 1) return sample - logf(1.5f * chi) - log1pf(-expf(sample)) - 3.0f * logf(u);
    const float sc = sqrtf(3.0f * chi) * 0.125f;
    return (0.5f - sample) / (sc / (1.0f + 2.0f * sc));
}

__device__ __forceinline__ float surr_bw_sigma(float chi) {
    const float sc = sqrtf(3.0f * chi) * 0.125f;
    return sc / (1.0f + 2.0f * sc);
}

// Network output -> sample: QS returns ln xi, BW returns xi in [0, 1/2].
__device__ __forceinline__ float surr_output(const SurrogateDev& s, float chi, float u, float y) {
    if (s.process == 1) {
        const float lnky = logf(1.5f * chi) + y + 3.0f * logf(u);   // ln(k Y)
        return -log1pf(expf(-lnky));                                 // ln(kY/(1+kY))
    }
    float xi = 0.5f - surr_bw_sigma(chi) * y;
    return fminf(fmaxf(xi, 0.0f), 0.5f);
}

// Forward pass for the 64 samples of one wave: lane l owns sample l
// (inputs x0, x1) and gets that sample's output.  The layers run in the
// transposed orientation (hidden units along the MFMA rows, samples along
// its columns), so that each layer's output fragment is the next layer's
// operand fragment in the same lane and nothing is exchanged between layers:
//   layer 1  Z^T  = [W1 | b1 | 0] [x0 x1 1 0]^T: FP32 MFMA 16x16x4, one per
//            16 hidden units (K = 4 holds the two inputs and the bias);
//   layer 2  H^T  = W2 silu(Z)^T: BF16 MFMA 16x16x16, FP32 accumulation;
//   layer 3  y    = b3 + w3 . silu(H + b2): each lane sums its 16 hidden
//            units, two cross-lane adds sum the four lane groups of a column.
// Samples are taken 16 at a time (one MFMA column block).
__device__ __forceinline__ float surr_forward_wave(const SurrogateDev& s, float x0, float x1) {
    const int lane = static_cast<int>(__lane_id());
    const int col = lane & 15, grp = lane >> 4;
    const float* p = s.p;
    // layer-1 A operand: row = hidden unit ks*16 + col, k = grp
    float a1[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        const int h = ks * 16 + col;
        a1[ks] = grp == 0 ? p[kOffW1 + 2 * h] : grp == 1 ? p[kOffW1 + 2 * h + 1] : grp == 2 ? p[kOffB1 + h] : 0.0f;
    }
    // layer-2 A operand: A[i][k] = W2[nt*16 + i][ks*16 + k], i = col, k = 4 grp + e
    surr_v4s aw2[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            aw2[nt][ks] = *reinterpret_cast<const surr_v4s*>(s.w2 + (nt * 16 + col) * 64 + ks * 16 + 4 * grp);
    // layer-2 output rows held by this lane: hidden unit nt*16 + 4 grp + e
    float b2[4][4], w3[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            b2[nt][e] = p[kOffB2 + nt * 16 + 4 * grp + e];
            w3[nt][e] = p[kOffW3 + nt * 16 + 4 * grp + e];
        }
    const float b3 = p[kOffB3];
    float y = 0.0f;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        // layer-1 B operand: k = grp, column = sample q*16 + col
        const float sx0 = __shfl(x0, q * 16 + col);
        const float sx1 = __shfl(x1, q * 16 + col);
        const float bx = grp == 0 ? sx0 : grp == 1 ? sx1 : grp == 2 ? 1.0f : 0.0f;
        surr_v4s h1[4];   // layer-2 B operand: k = hidden ks*16 + 4 grp + e, column = sample
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const surr_v4f zero = {0.0f, 0.0f, 0.0f, 0.0f};
            const surr_v4f z = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[ks], bx, zero, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) h1[ks][e] = surr_bf16(surr_silu(z[e]));
        }
        float part = 0.0f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            surr_v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aw2[nt][ks], h1[ks], acc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) part += w3[nt][e] * surr_silu(acc[e] + b2[nt][e]);
        }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (grp == q) y = part + b3;
    }
    return y;
}

// One network's weights in the layout that the fused step's forward pass
// reads from LDS: the 16 BF16 fragments of W2 (fragment 4 nt + ks, lane l:
// W2[16 nt + (l & 15)][16 ks + 4 (l >> 4) + 0..3], the layer-2 A operand),
// each lane's layer-1 operand for the four hidden-unit blocks, b2, w3, b3.
// Every fragment read is 64 consecutive 8-byte words (no bank conflict), so
// the weights need not stay in registers between batches.
struct alignas(16) SurrLds {
    surr_v4s w2f[16][64];
    float a1[4][64];
    float b2[64];
    float w3[64];
    float b3[4];
};
constexpr size_t kSurrLdsBytes = sizeof(SurrLds);

// Fill `L` from the device parameters (all threads of the block take part;
// the caller synchronises before the first forward pass).
__device__ __forceinline__ void surr_stage(const SurrogateDev& s, SurrLds* L, int tid, int nthreads) {
    const float* p = s.p;
    for (int i = tid; i < 16 * 64; i += nthreads) {
        const int f = i >> 6, l = i & 63, nt = f >> 2, ks = f & 3;
        L->w2f[f][l] = *reinterpret_cast<const surr_v4s*>(s.w2 + (nt * 16 + (l & 15)) * 64 + ks * 16 + 4 * (l >> 4));
    }
    for (int i = tid; i < 4 * 64; i += nthreads) {
        const int ks = i >> 6, l = i & 63, grp = l >> 4, h = ks * 16 + (l & 15);
        L->a1[ks][l] = grp == 0 ? p[kOffW1 + 2 * h] : grp == 1 ? p[kOffW1 + 2 * h + 1] : grp == 2 ? p[kOffB1 + h] : 0.0f;
    }
    for (int i = tid; i < 64; i += nthreads) {
        L->b2[i] = p[kOffB2 + i];
        L->w3[i] = p[kOffW3 + i];
    }
    if (tid < 4) L->b3[tid] = p[kOffB3];
}

// surr_forward_wave with the weights read from a staged SurrLds, fragment by
// fragment as the MFMAs need them: the same operations in the same order, so
// the same output bits.
__device__ __forceinline__ float surr_forward_wave_lds(const SurrLds* L, float x0, float x1) {
    const int lane = static_cast<int>(__lane_id());
    const int col = lane & 15, grp = lane >> 4;
    float y = 0.0f;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        const float sx0 = __shfl(x0, q * 16 + col);
        const float sx1 = __shfl(x1, q * 16 + col);
        const float bx = grp == 0 ? sx0 : grp == 1 ? sx1 : grp == 2 ? 1.0f : 0.0f;
        surr_v4s h1[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const surr_v4f zero = {0.0f, 0.0f, 0.0f, 0.0f};
            const surr_v4f z = __builtin_amdgcn_mfma_f32_16x16x4f32(L->a1[ks][lane], bx, zero, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) h1[ks][e] = surr_bf16(surr_silu(z[e]));
        }
        float part = 0.0f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            surr_v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(L->w2f[nt * 4 + ks][lane], h1[ks], acc, 0, 0, 0);
            const surr_v4f b2v = *reinterpret_cast<const surr_v4f*>(L->b2 + nt * 16 + 4 * grp);
            const surr_v4f w3v = *reinterpret_cast<const surr_v4f*>(L->w3 + nt * 16 + 4 * grp);
#pragma unroll
            for (int e = 0; e < 4; ++e) part += w3v[e] * surr_silu(acc[e] + b2v[e]);
        }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (grp == q) y = part + L->b3[0];
    }
    return y;
}

}  // namespace qedmi
