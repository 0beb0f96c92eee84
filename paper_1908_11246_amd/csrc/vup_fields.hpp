// Host-side launchers of the column kernels (IPSA statistics, probability
// matrix, field lines), the marginal and the point evaluation (k_fields.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/vup.h"

namespace vup {

constexpr int kMaxLevels = VUP_MAX_LEVELS;

// binned mean, variance and entropy of each column (vup_ipsa)
hipError_t launch_ipsa_stats(const double* edges, int B, int64_t K, const float* P,
                             double* mean_hist, double* var, double* entropy, hipStream_t s);
hipError_t launch_eval_points(const vup_model& m, int ndim, int64_t n, const double* x,
                              int64_t ldx, double* y, hipStream_t s);
hipError_t launch_ipsa_matrix(const double* edges, int B, int64_t K, const float* P,
                              const double* y_ref, double dy_lo, double dy_width, int n_dy,
                              float* Q, double* lost, hipStream_t s);
hipError_t launch_ipsa_fields(const double* edges, int B, int64_t K, const float* P,
                              const double* y_ref, int n_levels, const double* levels,
                              double* y_mode, double* p_max, double* quant, double* dev,
                              double* delta2, hipStream_t s);
// chunks of rows the marginal splits K into, and its workspace size
int marginal_chunks(int64_t K, int n);
size_t marginal_workspace_bytes(int64_t K, int n);
hipError_t launch_marginalize(int64_t K, int n, const float* A, const double* rho, void* ws,
                              double* out, hipStream_t s);
// the same with the partial sums in the library's own device array (no
// caller workspace); needs marginal_workspace_bytes(K, n) <= kStaticMarginalBytes
constexpr size_t kStaticMarginalBytes = (size_t)8 << 20;
hipError_t launch_marginalize_static(int64_t K, int n, const float* A, const double* rho,
                                     double* out, hipStream_t s);

}  // namespace vup
