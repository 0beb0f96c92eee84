// Bayes inversion over the model matrix (Sec. 3, the Bayes theorem paragraph
// and its footnote): the columns of the "inverted model matrix",
//   post[t][i] = [bin(i) = b] p_k(x_i) / P[k][b],  k = sel[t],
// i.e. the posterior over input cells given that the output fell in bin b,
// relative to the forward propagation that produced P (and its per-component
// normalisation Z). p_k is the same truncated, normalised Gaussian mixture the
// propagation sums: FP32 per-axis factors (gauss_factor_r, each axis scaled by
// its power of two 2^m) and their product; the mixture weight, 2^-sum m,
// 1/Z_{k,c} and 1/P_b are combined in FP64 per bin and applied in FP32.
//   k_posterior       workgroups over grid rows: per-bin factors
//                     pi_c / (Z_c P_b), the fastest-axis factors and the
//                     row's factor product staged, one multiply-add per cell
//                     and component
//   k_posterior_mean  E[x_d | y in b, k] = sum over the bin's cells of
//                     post x_d, one wave per (t, b) walking the part of the
//                     model matrix's compressed-by-bin cell list inside the
//                     window's index range (fixed summation order)
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
  int vec;                  // rows of post take float4 stores (n_L % 4 == 0, aligned)
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
  __shared__ int sm[VUP_MAX_COMP][VUP_MAX_DIM];  // the factors' scale exponents
  __shared__ double sfac[VUP_MAX_COMP];            // pi_c 2^-sum_d m_d / Z_{k,c}
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
    sm[c][d] = (ok && hi >= lo) ? axis_scale_exp(a.lo[d], a.hi[d], a.n[d], lo, hi, mu, 1.0 / sg)
                                : 0;
    if (!ok) atomicOr(&sbad, 1);
  }
  __syncthreads();
  if (threadIdx.x < C && kok) {
    // the scaled factors' product is 2^(sum_d m_d) times the density, as in
    // the propagation that reported Z
    const int c = threadIdx.x;
    int ms = 0;
    for (int d = 0; d < D; ++d) ms += sm[c][d];
    const double z = a.Z[k * C + c];
    const double w = C > 1 ? a.weight[k * C + c] : 1.0;
    sfac[c] = ldexp(w / z, -ms);
    if (!isfinite(z)) atomicOr(&sbad, 1);
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
    // only the window's columns: the cells read no others
    for (int c = 0; c < C; ++c) {
      const int wlo = swin[c][D - 1][0], whi = swin[c][D - 1][1];
      for (int col = wlo + (int)threadIdx.x; col <= whi; col += blockDim.x)
        gtab[c * nL + col] = gauss_factor_r(cell_centre(a.lo[D - 1], a.hi[D - 1], nL, col),
                                            smu[c][D - 1], srs[c][D - 1],
                                            scale_log(sm[c][D - 1]));
    }
  }
  __syncthreads();
  const bool bad = sbad != 0;
  float* post = a.post + (long long)t * a.N;
  // a row's factor product per component (0 outside the component's window)
  // and the columns any window covers; outside them, and in rows no window
  // covers, post is 0 (NaN for an invalid distribution)
  struct RowInfo {
    float rf[VUP_MAX_COMP];
    int clo[VUP_MAX_COMP], chi[VUP_MAX_COMP];
    int ulo, uhi;
  };
  auto row_info = [&](int r, RowInfo& ri) {
    int j[4] = {0, 0, 0, 0};
    int q = r;
    for (int d = D - 2; d >= 0; --d) {
      j[d] = q % a.n[d];
      q /= a.n[d];
    }
    ri.ulo = 0x7fffffff;
    ri.uhi = -1;
#pragma unroll
    for (int c = 0; c < VUP_MAX_COMP; ++c) {
      ri.rf[c] = 0.0f;
      ri.clo[c] = 0;
      ri.chi[c] = -1;
      if (c < C) {
        bool in = true;
        float f = 1.0f;
        for (int d = 0; d + 1 < D; ++d) {
          in = in && j[d] >= swin[c][d][0] && j[d] <= swin[c][d][1];
          if (in) f *= gauss_factor_r(cell_centre(a.lo[d], a.hi[d], a.n[d], j[d]), smu[c][d],
                                      srs[c][d], scale_log(sm[c][d]));
        }
        if (in && swin[c][D - 1][1] >= swin[c][D - 1][0]) {
          ri.rf[c] = f;
          ri.clo[c] = swin[c][D - 1][0];
          ri.chi[c] = swin[c][D - 1][1];
          ri.ulo = min(ri.ulo, ri.clo[c]);
          ri.uhi = max(ri.uhi, ri.chi[c]);
        }
      }
    }
  };
  auto cell = [&](const RowInfo& ri, int col, uint32_t code) {
    float v = 0.0f;
    if (code < 4u * (uint32_t)B) {
      const int b = (int)(code >> 2);
#pragma unroll
      for (int c = 0; c < VUP_MAX_COMP; ++c) {
        if (c < C && col >= ri.clo[c] && col <= ri.chi[c]) {
          const float g = a.gtab ? gtab[c * nL + col]
                                 : gauss_factor_r(cell_centre(a.lo[D - 1], a.hi[D - 1], nL, col),
                                                  smu[c][D - 1], srs[c][D - 1],
                                                  scale_log(sm[c][D - 1]));
          v = fmaf(ri.rf[c] * g, sfb[c * B + b], v);
        }
      }
    }
    return v;
  };
  if (a.vec) {
    // four columns per thread: one 8-byte load of bin codes, one 16-byte store
    const float fill = bad ? __builtin_nanf("") : 0.0f;
    for (int r = blockIdx.x; r < a.rows; r += gridDim.x) {
      RowInfo ri;
      row_info(r, ri);
      const uint16_t* brow = a.binmap + (long long)r * a.pitch;
      float4* prow4 = reinterpret_cast<float4*>(post + (long long)r * nL);
      for (int c4 = threadIdx.x; c4 < (nL >> 2); c4 += blockDim.x) {
        const int col0 = 4 * c4;
        float4 o = make_float4(fill, fill, fill, fill);
        if (!bad && col0 + 3 >= ri.ulo && col0 <= ri.uhi) {
          const uint2 cw = *reinterpret_cast<const uint2*>(brow + col0);
          o.x = cell(ri, col0, cw.x & 0xFFFFu);
          o.y = cell(ri, col0 + 1, cw.x >> 16);
          o.z = cell(ri, col0 + 2, cw.y & 0xFFFFu);
          o.w = cell(ri, col0 + 3, cw.y >> 16);
        }
        prow4[c4] = o;
      }
    }
  } else {
    for (int r = blockIdx.x; r < a.rows; r += gridDim.x) {
      RowInfo ri;
      row_info(r, ri);
      const uint16_t* brow = a.binmap + (long long)r * a.pitch;
      float* prow = post + (long long)r * nL;
      for (int col = threadIdx.x; col < nL; col += blockDim.x) {
        float v = 0.0f;
        if (col >= ri.ulo && col <= ri.uhi) v = cell(ri, col, brow[col]);
        prow[col] = bad ? __builtin_nanf("") : v;
      }
    }
  }
}

// first positions s in [s0, s1) of the ascending cell list with list[s] >= x0
// and with list[s] >= x1 (s1 if none), by the whole wave, both searches in the
// same rounds (their loads in flight together): each round probes 64
// positions spread over a search's remaining range and keeps the part between
// the last probe below its target and the first at or above it, so a range of
// n shrinks to n / 65 per round
struct WaveSearch {
  long long lo, hi;  // the answer lies in [lo, hi]
};

__device__ __forceinline__ long long probe_at(const WaveSearch& w, int i) {
  return w.lo + ((w.hi - w.lo) * (i + 1)) / 65;  // in (lo, hi) while hi - lo > 64
}

__device__ __forceinline__ void narrow(WaveSearch& w, bool ge) {
  const unsigned long long m = __ballot(ge);
  const int f = m ? __builtin_ctzll(m) : 64;  // first probe at or above the target
  const long long pf = probe_at(w, f), pb = probe_at(w, f - 1);
  if (f < 64) w.hi = pf;
  if (f > 0) w.lo = pb + 1;
}

__device__ __forceinline__ long long finish_search(const int* list, const WaveSearch& w,
                                                   long long x, int lane) {
  const long long p = w.lo + lane;
  const bool ge = p < w.hi && (long long)list[p] >= x;
  const unsigned long long m = __ballot(ge);
  return m ? w.lo + __builtin_ctzll(m) : w.hi;
}

__device__ __forceinline__ void wave_lower_bounds(const int* list, long long s0, long long s1,
                                                  long long x0, long long x1, int lane,
                                                  long long& r0, long long& r1) {
  WaveSearch a{s0, s1}, b{s0, s1};
  for (;;) {
    const bool on_a = a.hi - a.lo > 64, on_b = b.hi - b.lo > 64;  // uniform
    if (!on_a && !on_b) break;
    const int va = on_a ? list[probe_at(a, lane)] : 0;
    const int vb = on_b ? list[probe_at(b, lane)] : 0;
    if (on_a) narrow(a, (long long)va >= x0);
    if (on_b) narrow(b, (long long)vb >= x1);
  }
  r0 = finish_search(list, a, x0, lane);
  r1 = finish_search(list, b, x1, lane);
}

// one wave per (t, b): lanes take the bin's cells lane, lane + 64, ... of the
// compressed-by-bin list; the wave sum fixes the order. Only the part of the
// list inside the row-major index range of the distribution's window (the
// bounding box of its components' windows) can hold nonzero posteriors: the
// wave finds it by search and walks it with the same lane assignment as a
// walk of the whole list, skipping the loads of cells outside the box (their
// terms are exact zeros), so the sums do not depend on the skipping. With
// cell centres x_d = lo_d + (j_d + 1/2) h_d, the sums are kept as S0 = sum q
// and S_d = sum q j_d (FP64) and combined at the end; the row-major index is
// split with a double reciprocal and one correction step.
__global__ __launch_bounds__(256) void k_posterior_mean(PostArgs a) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  const long long t = blockIdx.y;
  if (b >= a.B) return;  // whole waves leave together
  const long long s0 = a.offsets[b], s1 = a.offsets[b + 1];
  const float* post = a.post + t * a.N;
  const int D = a.ndim, C = a.C;
  double* out = a.mean + (t * a.B + b) * a.ndim;
  // the posterior row is NaN (the same conditions as k_posterior): mean NaN,
  // 0 for a bin without cells
  const long long k = a.sel[t];
  bool bad = !(k >= 0 && k < a.K);
  int blo[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff}, bhi[4] = {-1, -1, -1, -1};
  bool any = false;  // some component's window is not empty
  if (!bad) {
    for (int c = 0; c < C; ++c) {
      bool cin = true;
      int wl[4], wh[4];
      for (int d = 0; d < D; ++d) {
        const long long pidx = (k * C + c) * D + d;
        if (!axis_window(a.lo[d], a.hi[d], a.n[d], a.mu[pidx], a.sigma[pidx], a.ns, wl[d], wh[d]))
          bad = true;
        cin = cin && wh[d] >= wl[d];
      }
      if (!isfinite(a.Z[k * C + c])) bad = true;
      if (cin) {
        any = true;
        for (int d = 0; d < D; ++d) {
          blo[d] = min(blo[d], wl[d]);
          bhi[d] = max(bhi[d], wh[d]);
        }
      }
    }
    for (int e = lane; e < a.B; e += 64)
      if (!isfinite(a.P[k * a.B + e])) bad = true;
    bad = __ballot(bad) != 0;
  }
  // a bin without mass has post 0 on all its cells (k_posterior's factor is 0
  // there): its sums are exact zeros, so the mean is 0 without a walk
  if (bad || !any || !(a.P[k * a.B + b] > 0.0f)) {
    if (lane < D) out[lane] = (bad && s1 > s0) ? __builtin_nan("") : 0.0;
    return;
  }
  // row-major index range of the window box, and its part of the list
  long long first = 0, last = 0;
  for (int d = 0; d < D; ++d) {
    first = first * a.n[d] + blo[d];
    last = last * a.n[d] + bhi[d];
  }
  long long sa, sb;
  wave_lower_bounds(a.perm, s0, s1, first, last + 1, lane, sa, sb);
  double S0 = 0.0, S[4] = {0.0, 0.0, 0.0, 0.0};
  // four cells per lane per pass, their loads in flight together; lane l
  // takes the cells s0 + l + 64 m in increasing m whatever the pass size, so
  // the sums are those of a walk of the whole list
  constexpr int U = 4;
  // start at the pass of the whole-list walk that reaches sa
  const long long sstart = s0 + ((sa - s0) / (64 * U)) * (64 * U);
  for (long long s = sstart + lane; s < sb; s += 64 * U) {
    int ci[U], jd[U][4];
    bool in[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long su = s + 64 * u;
      ci[u] = (su >= sa && su < sb) ? a.perm[su] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      in[u] = ci[u] >= 0;
      int rest = ci[u] < 0 ? 0 : ci[u];
#pragma unroll
      for (int d = 3; d >= 1; --d) {
        jd[u][d] = 0;
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
          jd[u][d] = rem;
          in[u] = in[u] && rem >= blo[d] && rem <= bhi[d];
          rest = quo;
        }
      }
      jd[u][0] = rest;
      in[u] = in[u] && rest >= blo[0] && rest <= bhi[0];
    }
    float q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = in[u] ? post[ci[u]] : 0.0f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!in[u]) continue;
      const double qd = (double)q[u];
      S0 += qd;
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (d < D) S[d] += qd * (double)jd[u][d];
    }
  }
  S0 = wave_sum(S0);
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
  a.vec = (nL % 4 == 0) && ((reinterpret_cast<uintptr_t>(post) & 15u) == 0);
  const size_t lds = (size_t)d.ncomp * (mm.B + (a.gtab ? nL : 0)) * sizeof(float);
  // about 32 rows per workgroup, so the per-bin factors and the factor table
  // are set up rarely, but at least 4096 workgroups in all while rows last
  long long gx = (mm.rows + 31) / 32;
  const long long want = (4096 + n_sel - 1) / n_sel;
  if (gx < want) gx = want < mm.rows ? want : mm.rows;
  gx = gx < 1 ? 1 : (gx > 4096 ? 4096 : gx);
  hipLaunchKernelGGL(k_posterior, dim3((unsigned)gx, (unsigned)n_sel), dim3(256), lds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !mean) return e;
  hipLaunchKernelGGL(k_posterior_mean, dim3((unsigned)((mm.B + 3) / 4), (unsigned)n_sel),
                     dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace vup
