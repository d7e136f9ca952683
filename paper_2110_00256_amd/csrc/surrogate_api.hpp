// Internal hooks between the C-ABI layer and the surrogate implementation.
#pragma once

#include "internal.hpp"

namespace qedmi {

// Attach the surrogates (may be null) to a step launch; validates them.
int32_t surrogate_bind(StepArgs& a, const qed_surrogate* bw, const qed_surrogate* qs);

}  // namespace qedmi
