// Learned inverse-CDF surrogate: device-side description (weights in BF16,
// FP32 biases) shared by the step kernel and the surrogate kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qedmi {

constexpr int kHidden = 64;

struct SurrogateDev {
    int32_t process;            // 0 BW, 1 QS
    int32_t pad_;
    float chi_lo, chi_hi;       // trained chi range
    float x_shift, x_scale;     // x0 = (ln chi - x_shift) * x_scale
    float probe_tol;
    float pad2_;
};

}  // namespace qedmi
