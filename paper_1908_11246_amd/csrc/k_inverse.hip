// Bayes inversion over the model matrix (Sec. 3, the Bayes theorem paragraph
// and its footnote): the columns of the "inverted model matrix",
//   post[t][i] = [bin(i) = b] p_k(x_i) / P[k][b],  k = sel[t],
// i.e. the posterior over input cells given that the output fell in bin b,
// relative to the forward propagation that produced P (and its per-component
// normalisation Z). p_k is the same truncated, normalised Gaussian mixture the
// propagation sums: FP32 per-axis factors (gauss_factor_r) and their product;
// the mixture weight, 1/Z_{k,c} and 1/P_b are combined in FP64 per bin and
// applied in FP32.
//   k_posterior       workgroups over grid rows: per-bin factors
//                     pi_c / (Z_c P_b), the fastest-axis factors and the
//                     row's factor product staged, one multiply-add per cell
//                     and component
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
  int gtab;                 // the fastest-axis factor table fits in LDS
  double rn[4];             // 1 / n_d, for the index arithmetic of the means
};

// One workgroup per (rows of the grid, selected distribution t). Per
// workgroup: the distribution's windows and reciprocal deviations, and the
// factor f[c][b] = pi_c / (Z_c P[k][b]) of every bin (0 where P is 0), so a
// cell costs its fastest-axis factor and one multiply-add per component.
// Per row: the product of the other axes' factors (uniform over the row).
__global__ __launch_bounds__(256) void k_posterior(PostArgs a) {
  extern __shared__ float sfb[];  // [C][B], then (when it fits) the fastest-axis factors [C][n_L]
  __shared__ int swin[VUP_MAX_COMP][VUP_MAX_DIM][2];
  __shared__ double smu[VUP_MAX_COMP][VUP_MAX_DIM], srs[VUP_MAX_COMP][VUP_MAX_DIM];
  __shared__ double sfac[VUP_MAX_COMP];  // pi_c / Z_{k,c}
  __shared__ int sbad;
  const int t = blockIdx.y;
  const long long k = a.sel[t];
  const bool kok = k >= 0 && k < a.K;
  const int D = a.ndim, C = a.C, B = a.B;
  if (threadIdx.x == 0) sbad = kok ? 0 : 1;
  __syncthreads();
  if (threadIdx.x < C * D && kok) {
    const int c = threadIdx.x / D, d = threadIdx.x % D;
    const long long pidx = (k * C + c) * D + d;
    const double mu = a.mu[pidx], sg = a.sigma[pidx];
    int lo, hi;
    const bool ok = axis_window(a.lo[d], a.hi[d], a.n[d], mu, sg, a.ns, lo, hi);
    swin[c][d][0] = lo;
    swin[c][d][1] = hi;
    smu[c][d] = mu;
    srs[c][d] = 1.0 / sg;
    if (!ok) atomicOr(&sbad, 1);
    if (d == 0) {
      const double z = a.Z[k * C + c];
      const double w = C > 1 ? a.weight[k * C + c] : 1.0;
      sfac[c] = w / z;
      if (!isfinite(z)) atomicOr(&sbad, 1);
    }
  }
  __syncthreads();
  if (kok) {
    for (int e = threadIdx.x; e < C * B; e += blockDim.x) {
      const int c = e / B, b = e - c * B;
      const float ev = a.P[k * B + b];
      if (!isfinite(ev)) atomicOr(&sbad, 1);
      sfb[e] = ev > 0.0f ? (float)(sfac[c] / (double)ev) : 0.0f;
    }
  }
  const int nL = a.n[D - 1];
  // the fastest-axis factor of every column inside each component's window,
  // shared by all rows of this distribution
  float* gtab = sfb + C * B;
  if (a.gtab && kok) {
    for (int e = threadIdx.x; e < C * nL; e += blockDim.x) {
      const int c = e / nL, col = e - c * nL;
      float g = 0.0f;
      if (col >= swin[c][D - 1][0] && col <= swin[c][D - 1][1])
        g = gauss_factor_r(cell_centre(a.lo[D - 1], a.hi[D - 1], nL, col), smu[c][D - 1],
                           srs[c][D - 1]);
      gtab[e] = g;
    }
  }
  __syncthreads();
  const bool bad = sbad != 0;
  float* post = a.post + (long long)t * a.N;
  for (int r = blockIdx.x; r < a.rows; r += gridDim.x) {
    // the row's multi-index and, per component, the product of the factors of
    // all axes but the fastest (0 when the row is outside the window)
    int j[4] = {0, 0, 0, 0};
    {
      int q = r;
      for (int d = D - 2; d >= 0; --d) {
        j[d] = q % a.n[d];
        q /= a.n[d];
      }
    }
    float rf[VUP_MAX_COMP];
    int clo[VUP_MAX_COMP], chi[VUP_MAX_COMP];
#pragma unroll
    for (int c = 0; c < VUP_MAX_COMP; ++c) {
      rf[c] = 0.0f;
      clo[c] = 0;
      chi[c] = -1;
      if (c < C) {
        bool in = true;
        float f = 1.0f;
        for (int d = 0; d + 1 < D; ++d) {
          in = in && j[d] >= swin[c][d][0] && j[d] <= swin[c][d][1];
          if (in) f *= gauss_factor_r(cell_centre(a.lo[d], a.hi[d], a.n[d], j[d]), smu[c][d],
                                      srs[c][d]);
        }
        if (in) {
          rf[c] = f;
          clo[c] = swin[c][D - 1][0];
          chi[c] = swin[c][D - 1][1];
        }
      }
    }
    const uint16_t* brow = a.binmap + (long long)r * a.pitch;
    float* prow = post + (long long)r * nL;
    for (int col = threadIdx.x; col < nL; col += blockDim.x) {
      const uint32_t code = brow[col];
      float v = 0.0f;
      if (code < 4u * (uint32_t)B) {
        const int b = (int)(code >> 2);
#pragma unroll
        for (int c = 0; c < VUP_MAX_COMP; ++c) {
          if (c < C && col >= clo[c] && col <= chi[c]) {
            const float g = a.gtab ? gtab[c * nL + col]
                                   : gauss_factor_r(cell_centre(a.lo[D - 1], a.hi[D - 1], nL, col),
                                                    smu[c][D - 1], srs[c][D - 1]);
            v = fmaf(rf[c] * g, sfb[c * B + b], v);
          }
        }
      }
      prow[col] = bad ? __builtin_nanf("") : v;
    }
  }
}

// one wave per (t, b): lanes take the bin's cells lane, lane + 64, ... of the
// compressed-by-bin list; the wave sum fixes the order. With cell centres
// x_d = lo_d + (j_d + 1/2) h_d, the sums are kept as S0 = sum q and
// S_d = sum q j_d (FP64) and combined at the end; the row-major index is split
// with a double reciprocal and one correction step.
__global__ __launch_bounds__(256) void k_posterior_mean(PostArgs a) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  const long long t = blockIdx.y;
  if (b >= a.B) return;  // whole waves leave together
  const long long s0 = a.offsets[b], s1 = a.offsets[b + 1];
  const float* post = a.post + t * a.N;
  const int D = a.ndim;
  double S0 = 0.0, S[4] = {0.0, 0.0, 0.0, 0.0};
  constexpr int U = 4;
  for (long long s = s0 + lane; s < s1; s += 64 * U) {
    int ci[U];
    float q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long su = s + 64 * u;
      ci[u] = su < s1 ? a.perm[su] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = ci[u] >= 0 ? post[ci[u]] : 0.0f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ci[u] < 0) continue;
      const double qd = (double)q[u];
      S0 += qd;
      int rest = ci[u];
#pragma unroll
      for (int d = 3; d >= 1; --d) {
        if (d < D) {
          const int n = a.n[d];
          int quo = (int)((double)rest * a.rn[d]);
          int rem = rest - quo * n;
          if (rem < 0) {
            --quo;
            rem += n;
          } else if (rem >= n) {
            ++quo;
            rem -= n;
          }
          S[d] += qd * (double)rem;
          rest = quo;
        }
      }
      S[0] += qd * (double)rest;
    }
  }
  S0 = wave_sum(S0);
  double* out = a.mean + (t * a.B + b) * a.ndim;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (d < D) {
      const double Sd = wave_sum(S[d]);
      const double h = (a.hi[d] - a.lo[d]) / a.n[d];
      if (lane == 0) out[d] = a.lo[d] * S0 + h * (Sd + 0.5 * S0);
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
  for (int x = 0; x < 4; ++x) a.rn[x] = 1.0 / a.n[x];
  const int nL = a.n[a.ndim - 1];
  a.gtab = (size_t)d.ncomp * (mm.B + nL) * sizeof(float) <= 65536 ? 1 : 0;
  const size_t lds = (size_t)d.ncomp * (mm.B + (a.gtab ? nL : 0)) * sizeof(float);
  // about eight rows per workgroup, so the per-bin factors are set up rarely
  long long gx = (mm.rows + 7) / 8;
  gx = gx < 1 ? 1 : (gx > 4096 ? 4096 : gx);
  hipLaunchKernelGGL(k_posterior, dim3((unsigned)gx, (unsigned)n_sel), dim3(256), lds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !mean) return e;
  hipLaunchKernelGGL(k_posterior_mean, dim3((unsigned)((mm.B + 3) / 4), (unsigned)n_sel),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace vup
