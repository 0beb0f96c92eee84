// Bayes inversion over the model matrix (Sec. 3, the Bayes theorem paragraph
// and its footnote): the columns of the "inverted model matrix",
//   post[t][i] = [bin(i) = b] p_k(x_i) / P[k][b],  k = sel[t],
// i.e. the posterior over input cells given that the output fell in bin b,
// relative to the forward propagation that produced P (and its per-component
// normalisation Z). p_k is the same truncated, normalised Gaussian mixture the
// propagation sums: FP32 per-axis factors (gauss_factor_r), their product, the
// mixture weight and 1/Z_{k,c} in FP64.
//   k_posterior       one thread per cell, the distribution's windows and
//                     reciprocal deviations staged per workgroup in LDS
//   k_posterior_mean  E[x_d | y in b, k] = sum over the bin's cells of
//                     post x_d, one wave per (t, b) walking the model
//                     matrix's compressed-by-bin cell list in order (fixed
//                     summation order)
#include <hip/hip_runtime.h>

#include "vup_device.hpp"
#include "vup_inverse.hpp"

namespace vup {

struct PostArgs {
  int ndim;
  int n[4];
  double lo[4], hi[4];
  int pitch;                // padded length of the fastest axis in the bin map
  const uint16_t* binmap;   // 4 * bin, 4 * B for no bin
  const long long* offsets; // CSR row starts [B + 1]
  const int* perm;          // cells sorted by bin
  long long N, rows;
  int B;
  // distributions
  long long K;
  int C;
  double ns;
  const double* mu;
  const double* sigma;
  const double* weight;
  const long long* sel;
  long long n_sel;
  const float* P;
  const double* Z;
  float* post;
  double* mean;
};

__device__ __forceinline__ void unflatten(const PostArgs& a, long long i, int (&j)[4]) {
  long long t = i;
  for (int d = a.ndim - 1; d >= 0; --d) {
    j[d] = (int)(t % a.n[d]);
    t /= a.n[d];
  }
}

__global__ __launch_bounds__(256) void k_posterior(PostArgs a) {
  __shared__ int swin[VUP_MAX_COMP][VUP_MAX_DIM][2];
  __shared__ double smu[VUP_MAX_COMP][VUP_MAX_DIM], srs[VUP_MAX_COMP][VUP_MAX_DIM];
  __shared__ double sfac[VUP_MAX_COMP];  // pi_c / Z_{k,c}
  __shared__ int sbad;
  const long long t = blockIdx.y;
  const long long k = a.sel[t];
  const bool kok = k >= 0 && k < a.K;
  if (threadIdx.x == 0) sbad = kok ? 0 : 1;
  __syncthreads();
  if (threadIdx.x < a.C * a.ndim && kok) {
    const int c = threadIdx.x / a.ndim, d = threadIdx.x % a.ndim;
    const long long pidx = (k * a.C + c) * a.ndim + d;
    const double mu = a.mu[pidx], sg = a.sigma[pidx];
    int lo, hi;
    const bool ok = axis_window(a.lo[d], a.hi[d], a.n[d], mu, sg, a.ns, lo, hi);
    swin[c][d][0] = lo;
    swin[c][d][1] = hi;
    smu[c][d] = mu;
    srs[c][d] = 1.0 / sg;
    if (!ok) atomicOr(&sbad, 1);
    if (d == 0) {
      const double z = a.Z[k * a.C + c];
      const double w = a.C > 1 ? a.weight[k * a.C + c] : 1.0;
      sfac[c] = w / z;
      if (!isfinite(z)) atomicOr(&sbad, 1);
    }
  }
  __syncthreads();
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  float* out = a.post + t * a.N + i;
  if (sbad) {
    *out = __builtin_nanf("");
    return;
  }
  int j[4] = {0, 0, 0, 0};
  unflatten(a, i, j);
  double p = 0.0;
  for (int c = 0; c < a.C; ++c) {
    bool in = true;
    for (int d = 0; d < a.ndim; ++d) in = in && j[d] >= swin[c][d][0] && j[d] <= swin[c][d][1];
    if (!in) continue;
    float w = 1.0f;
    for (int d = 0; d < a.ndim; ++d)
      w *= gauss_factor_r(cell_centre(a.lo[d], a.hi[d], a.n[d], j[d]), smu[c][d], srs[c][d]);
    p += (double)w * sfac[c];
  }
  const long long row = i / a.n[a.ndim - 1];
  const int col = (int)(i - row * a.n[a.ndim - 1]);
  const uint32_t code = a.binmap[row * a.pitch + col];
  float v = 0.0f;
  if (code < 4u * (uint32_t)a.B) {
    const float ev = a.P[k * a.B + (code >> 2)];
    if (!isfinite(ev)) v = __builtin_nanf("");
    else if (ev > 0.0f && p > 0.0) v = (float)(p / (double)ev);
  }
  *out = v;
}

// one wave per (t, b): lanes take the bin's cells lane, lane + 64, ... of the
// compressed-by-bin list; the wave sum fixes the order
__global__ __launch_bounds__(256) void k_posterior_mean(PostArgs a) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  const long long t = blockIdx.y;
  if (b >= a.B) return;  // whole waves leave together
  const long long s0 = a.offsets[b], s1 = a.offsets[b + 1];
  const float* post = a.post + t * a.N;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long s = s0 + lane; s < s1; s += 64) {
    const long long i = a.perm[s];
    const double q = (double)post[i];
    int j[4] = {0, 0, 0, 0};
    unflatten(a, i, j);
#pragma unroll
    for (int d = 0; d < 4; ++d)
      if (d < a.ndim) acc[d] += q * cell_centre(a.lo[d], a.hi[d], a.n[d], j[d]);
  }
  double* out = a.mean + (t * a.B + b) * a.ndim;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (d < a.ndim) {
      const double s = wave_sum(acc[d]);
      if (lane == 0) out[d] = s;
    }
  }
}

hipError_t launch_posterior(const vup_mm& mm, const vup_dists& d, int64_t n_sel,
                            const int64_t* sel, const float* P, const double* Z, float* post,
                            double* mean, hipStream_t s) {
  if (n_sel == 0) return hipSuccess;
  PostArgs a{};
  a.ndim = mm.grid.ndim;
  for (int x = 0; x < 4; ++x) {
    a.n[x] = x < a.ndim ? mm.grid.n[x] : 1;
    a.lo[x] = mm.grid.lo[x];
    a.hi[x] = mm.grid.hi[x];
  }
  a.pitch = mm.pitch;
  const char* ws = static_cast<const char*>(mm.ws);
  a.binmap = reinterpret_cast<const uint16_t*>(ws + mm.off_binmap);
  a.offsets = reinterpret_cast<const long long*>(ws + mm.off_offsets);
  a.perm = reinterpret_cast<const int*>(ws + mm.off_perm);
  a.N = mm.N;
  a.rows = mm.rows;
  a.B = mm.B;
  a.K = d.K;
  a.C = d.ncomp;
  a.ns = d.n_sigma;
  a.mu = d.mu;
  a.sigma = d.sigma;
  a.weight = d.weight;
  a.sel = reinterpret_cast<const long long*>(sel);
  a.n_sel = n_sel;
  a.P = P;
  a.Z = Z;
  a.post = post;
  a.mean = mean;
  hipLaunchKernelGGL(k_posterior, dim3((unsigned)((mm.N + 255) / 256), (unsigned)n_sel),
                     dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !mean) return e;
  hipLaunchKernelGGL(k_posterior_mean, dim3((unsigned)((mm.B + 3) / 4), (unsigned)n_sel),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace vup
