// Host-side launcher of the Bayes-inversion kernels (k_inverse.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vup.h"

namespace vup {

hipError_t launch_posterior(const vup_mm& mm, const vup_dists& d, int64_t n_sel,
                            const int64_t* sel, const float* P, const double* Z, float* post,
                            double* mean, hipStream_t s);

}  // namespace vup
