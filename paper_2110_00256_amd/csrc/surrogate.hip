// Learned inverse-CDF surrogate (MLP 2 -> 64 -> 64 -> 1): placeholder until
// the MFMA kernels are in place.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "surrogate.hpp"
#include "surrogate_api.hpp"

struct qed_surrogate {
    int process = 0;
};

namespace qedmi {
int32_t surrogate_bind(StepArgs& a, const qed_surrogate* bw, const qed_surrogate* qs) {
    a.bw_surr = nullptr;
    a.qs_surr = nullptr;
    if (bw || qs) {
        set_error("surrogate sampling is not available in this build");
        return QED_ERR_STATE;
    }
    return QED_OK;
}
}  // namespace qedmi

using namespace qedmi;

static int32_t not_ready() {
    set_error("surrogate is not available in this build");
    return QED_ERR_STATE;
}

extern "C" int32_t qed_surrogate_train(qed_context*, const qed_table*, const qed_surrogate_cfg*, qed_surrogate** out,
                                       float*, void*) {
    if (out) *out = nullptr;
    return not_ready();
}
extern "C" int32_t qed_surrogate_from_host(const qed_table*, const qed_surrogate_cfg*, const float*,
                                           qed_surrogate** out) {
    if (out) *out = nullptr;
    return not_ready();
}
extern "C" int32_t qed_surrogate_get_params(const qed_surrogate*, float*) { return not_ready(); }
extern "C" int32_t qed_surrogate_forward(const qed_surrogate*, const float*, float*, int64_t, void*) {
    return not_ready();
}
extern "C" int32_t qed_surrogate_grad(const qed_surrogate*, const float*, const float*, int64_t, float*, float*,
                                      void*) {
    return not_ready();
}
extern "C" int32_t qed_surrogate_sample(const qed_surrogate*, const float*, const float*, float*, int64_t, void*) {
    return not_ready();
}
extern "C" void qed_surrogate_destroy(qed_surrogate* s) { delete s; }
