// Traffic calibration, a measurement aid beside the fused step: streams a
// buffer with the access pattern of the step's streaming phase (non-temporal
// 8-byte loads and stores, grid-stride), so that the hardware's fetch and
// write counters can be scaled by what they report for a known number of
// bytes.  mode 0 reads n_bytes of src (the sum is stored only if it is NaN,
// which finite data never gives); mode 1 writes n_bytes to dst; mode 2
// copies src to dst.  Modes 3 and 4 read and write like 0 and 1 with
// ordinary (temporal) loads and stores, the kind the event pass uses.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace qedmi {
namespace {

__global__ void __launch_bounds__(256) calib_kernel(const double* src, double* dst, int64_t n, int mode) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * 256) {
        if (mode == 1) {
            __builtin_nontemporal_store(static_cast<double>(i), dst + i);
        } else if (mode == 3) {
            acc += src[i];
        } else if (mode == 4) {
            dst[i] = static_cast<double>(i);
        } else {
            const double v = __builtin_nontemporal_load(src + i);
            if (mode == 2) __builtin_nontemporal_store(v, dst + i);
            else acc += v;
        }
    }
    // a read-only pass stores nothing unless the sum is NaN (never, for finite data)
    if ((mode == 0 || mode == 3) && acc != acc) dst[0] = acc;
}

}  // namespace
}  // namespace qedmi

extern "C" int32_t qed_traffic_calibrate(const void* src, void* dst, int64_t n_bytes, int32_t mode, void* stream) {
    using namespace qedmi;
    if (mode < 0 || mode > 4) {
        set_error("mode must be 0 (read), 1 (write), 2 (copy), 3 (temporal read) or 4 (temporal write)");
        return QED_ERR_INVALID;
    }
    if (n_bytes < 0 || n_bytes % 8 != 0) { set_error("n_bytes must be a non-negative multiple of 8"); return QED_ERR_INVALID; }
    if (n_bytes == 0) return QED_OK;
    if ((mode != 1 && mode != 4 && !src) || !dst) { set_error("src/dst is null"); return QED_ERR_INVALID; }
    int cus = 256;
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipLaunchKernelGGL(calib_kernel, dim3(2 * cus), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const double*>(src), static_cast<double*>(dst), n_bytes / 8, mode);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("calibration launch: ") + hipGetErrorString(e));
        return QED_ERR_HIP;
    }
    return QED_OK;
}
