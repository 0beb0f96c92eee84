// Kernels over the columns of the propagated output matrix (Sec. 5.2) and the
// model at the input pdfs' maxima (Sec. 5.3):
//   k_eval_points    y_i = M(x_i) at caller-given points, FP64
//   k_ipsa           binned mean, two-pass variance and entropy per column
//   k_ipsa_matrix    IPSA probability matrix: each column of P, read as a
//                    piecewise-constant density over its bins, is translated
//                    by y(l) and integrated over a uniform Delta-y grid; done
//                    as differences of its piecewise-linear FP64 CDF
//   k_ipsa_fields    per column: most probable bin, quantiles of the same
//                    CDF, expected deviation from y(l) and the binned local
//                    expected squared deviation (eq. IPSAvar)
//   k_marg_partial / k_marg_combine   global marginal over locations,
//                    out[j] = sum_k rho_k A[k][j], in a fixed order
//
// The column kernels give one wave64 to one column at a time (see
// stream_columns); the bin edges sit once per workgroup in LDS. All HBM
// traffic is one read of P and one write of the outputs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "vup_device.hpp"
#include "vup_fields.hpp"

namespace vup {

// ---------------------------------------------------------------------------
// model at points
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_eval_points(vup_model m, int ndim, long long n,
                                                     const double* __restrict__ x, long long ldx,
                                                     double* __restrict__ y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double p[4] = {0.0, 0.0, 0.0, 0.0};
  for (int d = 0; d < ndim; ++d) p[d] = x[i * ldx + d];
  y[i] = model_at(m.kind, ndim, m.theta, p);
}

hipError_t launch_eval_points(const vup_model& m, int ndim, int64_t n, const double* x,
                              int64_t ldx, double* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const long long blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_eval_points, dim3((unsigned)blocks), dim3(256), 0, s, m, ndim,
                     (long long)n, x, (long long)ldx, y);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// column streaming shared by the column kernels
//
// A column is handled by a group of LPC lanes: LPC = 16 (four columns per
// wave, one per DPP row) when B <= 1024, else LPC = 64. Lane r of a group
// holds, for round i, the four bins RS i + 4 r .. + 3 (RS = 4 LPC bins per
// round) in one float4, zero beyond B, so a round is one coalesced read of
// 16 LPC bytes per column. Each wave walks its own sequence of column slots
// (no workgroup barrier in the loop) and loads the next slot's columns while
// it works on the current ones. Sums within a group use DPP row operations
// (LPC = 16) or the whole-wave reduction (LPC = 64), in a fixed order.
// ---------------------------------------------------------------------------
template <int LPC, int MV, bool VEC>
__device__ __forceinline__ void load_col(const float* __restrict__ P, long long k, long long K,
                                         int B, float4 (&v)[MV]) {
  const int r = threadIdx.x & (LPC - 1);
  const float* col = P + k * (long long)B;
  const bool live = k < K;
#pragma unroll
  for (int i = 0; i < MV; ++i) {
    const int b = 4 * LPC * i + 4 * r;
    if constexpr (VEC) {
      v[i] = live && b < B ? *reinterpret_cast<const float4*>(col + b)
                           : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      v[i].x = live && b < B ? col[b] : 0.f;
      v[i].y = live && b + 1 < B ? col[b + 1] : 0.f;
      v[i].z = live && b + 2 < B ? col[b + 2] : 0.f;
      v[i].w = live && b + 3 < B ? col[b + 3] : 0.f;
    }
  }
}

// body(k, live, v): k = this group's column, live = k < K (uniform in the
// group); every lane of the wave calls body for every slot
template <int LPC, int MV, bool VEC, class Body>
__device__ __forceinline__ void stream_columns(const float* __restrict__ P, long long K, int B,
                                               Body&& body) {
  constexpr int G = 64 / LPC;
  const int waves = blockDim.x >> 6;
  const long long step = (long long)gridDim.x * waves * G;
  const int g = (threadIdx.x & 63) / LPC;
  long long base = ((long long)blockIdx.x * waves + (threadIdx.x >> 6)) * G;
  float4 cur[MV];
  if (base < K) load_col<LPC, MV, VEC>(P, base + g, K, B, cur);
  while (base < K) {
    const long long nb = base + step;
    float4 nxt[MV];
    if (nb < K) {
      load_col<LPC, MV, VEC>(P, nb + g, K, B, nxt);
    } else {
#pragma unroll
      for (int i = 0; i < MV; ++i) nxt[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    body(base + g, base + g < K, cur);
#pragma unroll
    for (int i = 0; i < MV; ++i) cur[i] = nxt[i];
    base = nb;
  }
}

__device__ __forceinline__ double shfl_f64(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __shfl((int)(b & 0xFFFFFFFF), src, 64);
  const int hi = __shfl((int)(b >> 32), src, 64);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// value of the previous lane of the group (0 for the group's first lane)
template <int LPC>
__device__ __forceinline__ double grp_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __shfl_up((int)(b & 0xFFFFFFFF), 1, LPC);
  const int hi = __shfl_up((int)(b >> 32), 1, LPC);
  const double p = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  return (threadIdx.x & (LPC - 1)) == 0 ? 0.0 : p;
}

// inclusive scan within the group
template <int LPC>
__device__ __forceinline__ double grp_scan(double v) {
  if constexpr (LPC == 16) return row_scan(v);
  else return wave_scan(v);
}

// the group's last lane's value, given to every lane of the group
template <int LPC>
__device__ __forceinline__ double grp_last(double v) {
  if constexpr (LPC == 16) return shfl_f64(v, (threadIdx.x & 63) | 15);
  else return lane_value(v, 63);
}

template <int LPC>
__device__ __forceinline__ double grp_sum(double v) {
  if constexpr (LPC == 16) return grp_last<16>(row_scan(v));
  else return wave_sum(v);
}

__device__ __forceinline__ float f4(const float4& v, int j) {
  return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}

// LDS writes of a wave made visible to the wave's other lanes
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Column CDF in registers, one round at a time. col_scan gives each lane the
// inclusive group scan of its four-bin sums per round and returns the column
// total T; round_cdf then yields c[j] = C_{b+j} for the lane's bins b + j and
// c[4] = C_{b+4}. The end value c[4] is taken from the scan itself, so it
// equals the next lane's c[0] (and, for the column's last bins, T) bit for
// bit: the lanes' intervals (c[0], c[4]] tile (0, T] with no gap or overlap.
template <int LPC, int MV>
__device__ __forceinline__ double col_scan(const float4 (&v)[MV], int B, double (&incl)[MV]) {
  double T = 0.0;
#pragma unroll
  for (int i = 0; i < MV; ++i) {
    incl[i] = 0.0;
    if (4 * LPC * i < B) {
      const double s = (((double)v[i].x + (double)v[i].y) + (double)v[i].z) + (double)v[i].w;
      incl[i] = grp_scan<LPC>(s);
      T += grp_last<LPC>(incl[i]);
    }
  }
  return T;
}

// `base` is the mass of the earlier rounds, advanced exactly as col_scan
// accumulated T
template <int LPC>
__device__ __forceinline__ void round_cdf(const float4& v, double incl, double& base,
                                          double (&c)[5]) {
  c[0] = base + grp_prev<LPC>(incl);
  c[1] = c[0] + (double)v.x;
  c[2] = c[1] + (double)v.y;
  c[3] = c[2] + (double)v.z;
  c[4] = base + incl;
  base += grp_last<LPC>(incl);
}

// edges, bin centres and (for the matrix) reciprocal bin widths, once per
// workgroup
__device__ __forceinline__ void stage_tables(const double* __restrict__ edges, int B, double* E,
                                             double* cen, double* invw) {
  if (E)
    for (int b = threadIdx.x; b <= B; b += blockDim.x) E[b] = edges[b];
  if (cen)
    for (int b = threadIdx.x; b < B; b += blockDim.x) cen[b] = 0.5 * (edges[b] + edges[b + 1]);
  if (invw)
    for (int b = threadIdx.x; b < B; b += blockDim.x) invw[b] = 1.0 / (edges[b + 1] - edges[b]);
  __syncthreads();
}

// p ln p for one FP32 probability: FP32 base-2 logarithm of the FP32 value
// (relative error a few 2^-24), scaled and accumulated in FP64. Values below
// the smallest normal FP32 number contribute less than 1e-36 and are skipped.
__device__ __forceinline__ double p_log2_p(float p) {
  return p >= 1.17549435e-38f ? (double)p * (double)__log2f(p) : 0.0;
}

// ---------------------------------------------------------------------------
// coarse-grained statistics of vup_ipsa: binned mean, two-pass variance and
// entropy, FP64 sums (Sec. 5.2)
// ---------------------------------------------------------------------------
struct StatArgs {
  const float* P;
  const double* edges;
  long long K;
  int B;
  double* mean_hist;
  double* var;
  double* entropy;
};

template <int LPC, int MV, bool VEC>
__global__ __launch_bounds__(256) void k_ipsa(StatArgs a) {
  extern __shared__ double lds[];
  double* cen = lds;
  const int B = a.B;
  const int r = threadIdx.x & (LPC - 1);
  stage_tables(a.edges, B, nullptr, cen, nullptr);
  stream_columns<LPC, MV, VEC>(a.P, a.K, B, [&](long long k, bool live, const float4 (&v)[MV]) {
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < MV; ++i) {
      const int b = 4 * LPC * i + 4 * r;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (b + j < B) m += (double)f4(v[i], j) * cen[b + j];
    }
    m = grp_sum<LPC>(m);
    double var = 0.0, h = 0.0;
#pragma unroll
    for (int i = 0; i < MV; ++i) {
      const int b = 4 * LPC * i + 4 * r;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (b + j < B) {
          const float p = f4(v[i], j);
          const double dc = cen[b + j] - m;
          var += (double)p * (dc * dc);
          h += p_log2_p(p);
        }
      }
    }
    var = grp_sum<LPC>(var);
    h = grp_sum<LPC>(h);
    if (live && r == 0) {
      if (a.mean_hist) a.mean_hist[k] = m;
      if (a.var) a.var[k] = var;
      if (a.entropy) a.entropy[k] = -0.69314718055994530942 * h;
    }
  });
}

// ---------------------------------------------------------------------------
// IPSA probability matrix
// ---------------------------------------------------------------------------
struct MatrixArgs {
  const float* P;       // [K][B]
  const double* edges;  // [B+1]
  const double* y_ref;  // [K]
  long long K;
  int B;
  double dy_lo, dy_width;
  int J;       // target cells
  float* Q;    // [K][J]
  double* lost;
};

// number of edges e_0..e_B that are <= t (0 for NaN t)
__device__ __forceinline__ int count_le(const double* E, int B, double t) {
  int lo = 0, hi = B + 1;  // answer in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (E[mid] <= t) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// piecewise-linear CDF at t, given cnt = count_le(t)
__device__ __forceinline__ double cdf_at(const double* E, const double* invw, const double* C, int B,
                                         double T, int cnt, double t) {
  if (cnt == 0) return 0.0;
  if (cnt > B) return T;
  const int b = cnt - 1;
  const double frac = (t - E[b]) * invw[b];
  return C[b] + (C[b + 1] - C[b]) * frac;
}

// target grid point d_j = d_lo + j*h (one multiply, one add, no contraction),
// moved into output coordinates by y
__device__ __forceinline__ double target_point(double dlo, double h, int j, double y) {
  return __dadd_rn(__dadd_rn(dlo, __dmul_rn((double)j, h)), y);
}

// number of edges <= t from a guess: exact whatever the guess (monotone
// edges), a step or two when the guess comes from near-uniform edges
__device__ __forceinline__ int count_le_from(const double* E, int B, double t, int cnt) {
  while (cnt <= B && E[cnt] <= t) ++cnt;
  while (cnt > 0 && !(E[cnt - 1] <= t)) --cnt;
  return cnt;
}

// The matrix gives a column a whole wave. The J + 1 grid points d_j + y are
// taken round-robin (lane l of round r has point 64 r + l), so the lanes of a
// round look up adjacent bins (no LDS bank conflicts); Q_j = F(j+1) - F(j)
// comes from the neighbouring lane. With near-uniform edges (each within half
// an average bin width of its uniform position) a point's bin is guessed
// arithmetically and corrected exactly; otherwise it is found by bisection.
template <int LPC, int MV, bool VEC>
__global__ __launch_bounds__(256) void k_ipsa_matrix(MatrixArgs a) {
  // launched with LPC = 64 only (one column per wave); the launch table
  // instantiates the other widths, which do nothing
  if constexpr (LPC != 64) {
    return;
  } else {
  constexpr int G = 1;
  extern __shared__ double lds[];
  __shared__ int s_nonuniform;
  const int B = a.B;
  double* E = lds;
  double* invw = lds + (B + 1);
  const int lane = threadIdx.x & 63;
  const int r = lane & (LPC - 1);
  const int g = lane / LPC;
  double* C = lds + (2 * B + 1) + ((threadIdx.x >> 6) * G + g) * (B + 1);
  if (threadIdx.x == 0) s_nonuniform = 0;
  stage_tables(a.edges, B, E, nullptr, invw);
  // near-uniform edges?
  const double e0 = E[0], wbar = (E[B] - E[0]) / B;
  for (int b = threadIdx.x; b <= B; b += blockDim.x)
    if (!(fabs(E[b] - (e0 + b * wbar)) <= 0.5 * wbar)) atomicOr(&s_nonuniform, 1);
  __syncthreads();
  const bool uniform = s_nonuniform == 0;
  const double scale = 1.0 / wbar;
  stream_columns<LPC, MV, VEC>(a.P, a.K, B, [&](long long k, bool live, const float4 (&v)[MV]) {
    double incl[MV];
    const double T = col_scan<LPC, MV>(v, B, incl);
    double base = 0.0;
#pragma unroll
    for (int i = 0; i < MV; ++i) {
      if (4 * LPC * i < B) {
        double c[5];
        round_cdf<LPC>(v[i], incl[i], base, c);
        const int b = 4 * LPC * i + 4 * r;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (b + j < B) C[b + j] = c[j];
      }
    }
    if (r == 0) C[B] = T;
    wave_lds_sync();
    float* q = a.Q + k * (long long)a.J;
    const bool fin = isfinite(T);
    if (live && !fin) {
      for (int j = lane; j < a.J; j += 64) q[j] = __builtin_nanf("");
      if (lane == 0 && a.lost) a.lost[k] = __builtin_nan("");
    } else if (live) {
      const double y = a.y_ref[k];
      const int J = a.J;
      double last = 0.0, F_first = 0.0, F_end = 0.0;
      for (int p0 = 0; p0 <= J; p0 += 64) {
        const int p = p0 + lane;
        double F = 0.0;
        if (p <= J) {
          const double t = target_point(a.dy_lo, a.dy_width, p, y);
          int cnt;
          if (uniform) {
            const double gd = fmin(fmax(floor((t - e0) * scale), -1.0), (double)B);
            cnt = count_le_from(E, B, t, (int)gd + 1);
          } else {
            cnt = count_le(E, B, t);
          }
          F = cdf_at(E, invw, C, B, T, cnt, t);
        }
        double Fprev = grp_prev<64>(F);
        if (lane == 0) Fprev = last;
        if (p >= 1 && p <= J) q[p - 1] = (float)(F - Fprev);
        last = lane_value(F, 63);
        if (p0 == 0) F_first = lane_value(F, 0);
        if (p0 == (J / 64) * 64) F_end = lane_value(F, J - p0);
      }
      if (lane == 0 && a.lost) a.lost[k] = F_first + (T - F_end);
    }
    wave_lds_sync();  // C is rewritten for the next column
  });
  }
}

// ---------------------------------------------------------------------------
// field lines
// ---------------------------------------------------------------------------
struct FieldArgs {
  const float* P;
  const double* edges;
  const double* y_ref;
  long long K;
  int B;
  int nq;
  double level[kMaxLevels];
  double* y_mode;
  double* p_max;
  double* quant;  // [K][nq]
  double* dev;
  double* delta2;
};

template <int LPC, int MV, bool VEC>
__global__ __launch_bounds__(256) void k_ipsa_fields(FieldArgs a) {
  extern __shared__ double lds[];
  const int B = a.B;
  double* E = lds;
  double* cen = lds + (B + 1);
  double* lev = lds + (2 * B + 1);
  const int lane = threadIdx.x & 63;
  const int r = lane & (LPC - 1);
  const int g = lane / LPC;
  const double nan = __builtin_nan("");
  if (threadIdx.x < kMaxLevels) lev[threadIdx.x] = a.level[threadIdx.x];
  stage_tables(a.edges, B, E, cen, nullptr);
  stream_columns<LPC, MV, VEC>(a.P, a.K, B, [&](long long k, bool live, const float4 (&v)[MV]) {
    const double y = (live && a.y_ref) ? a.y_ref[k] : 0.0;
    double incl[MV];
    const double T = col_scan<LPC, MV>(v, B, incl);
    const bool finite = isfinite(T);
    const bool positive = finite && T > 0.0;
    float vmax = -__builtin_inff();
    int imax = B;
    double s1 = 0.0, s2 = 0.0;
    double base = 0.0;
    unsigned found = 0u;  // levels answered so far (uniform in the group)
#pragma unroll
    for (int i = 0; i < MV; ++i) {
      if (4 * LPC * i < B) {
        const int b = 4 * LPC * i + 4 * r;
        double c[5];
        round_cdf<LPC>(v[i], incl[i], base, c);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (b + j < B) {
            const float p = f4(v[i], j);
            if (p > vmax) {
              vmax = p;
              imax = b + j;
            }
            const double t = cen[b + j] - y;
            const double pt = (double)p * t;
            s1 += pt;
            s2 += pt * t;
          }
        }
        if (a.quant) {
#pragma unroll 1
          for (int q = 0; q < a.nq; ++q) {
            {
              const double target = lev[q] * T;
              const bool want = positive && !(found & (1u << q));
              const bool mine = want && b < B && c[0] < target && target <= c[4];
              const unsigned long long mask = __ballot(mine);
              // this group's bits of the ballot
              unsigned long long gm = mask;
              if constexpr (LPC < 64) gm = (mask >> (g * LPC)) & ((1ull << LPC) - 1);
              if (gm != 0ull) {
                found |= 1u << q;
                if (live && r == __ffsll((long long)gm) - 1) {
                  // first of the lane's bins whose upper CDF value reaches the
                  // level (selects only: no register array indexed at run time)
                  const int jj = c[1] >= target ? 0 : c[2] >= target ? 1 : c[3] >= target ? 2 : 3;
                  const double cj = jj == 0 ? c[0] : jj == 1 ? c[1] : jj == 2 ? c[2] : c[3];
                  const double pb = (double)f4(v[i], jj);
                  double* out = a.quant + k * (long long)a.nq + q;
                  if (pb > 0.0) {
                    const double frac = fmin(fmax((target - cj) / pb, 0.0), 1.0);
                    *out = E[b + jj] + frac * (E[b + jj + 1] - E[b + jj]);
                  } else {
                    // reached only when rounding puts the level an ulp past
                    // the end of the last positive bin before an empty
                    // stretch: answer that bin's right edge
                    int jb = -1;
#pragma unroll
                    for (int t2 = 0; t2 < 4; ++t2)
                      if (t2 <= jj && f4(v[i], t2) > 0.0f) jb = t2;
                    *out = jb >= 0 ? E[b + jb + 1] : E[b];
                  }
                }
              }
            }
          }
        }
      }
    }
    // first maximum over the group: larger value wins, equal values keep the lower bin
    for (int o = LPC / 2; o >= 1; o >>= 1) {
      const float ov = __shfl_xor(vmax, o, 64);
      const int oi = __shfl_xor(imax, o, 64);
      if (ov > vmax || (ov == vmax && oi < imax)) {
        vmax = ov;
        imax = oi;
      }
    }
    const double S1 = grp_sum<LPC>(s1);
    const double S2 = grp_sum<LPC>(s2);
    if (live && r == 0) {
      if (a.p_max) a.p_max[k] = finite ? (double)vmax : nan;
      if (a.y_mode) a.y_mode[k] = positive ? cen[imax] : nan;
      if (a.dev) a.dev[k] = finite ? S1 : nan;
      if (a.delta2) a.delta2[k] = finite ? 0.5 * S2 : nan;
      if (a.quant)
        for (int q = 0; q < a.nq; ++q)
          if (!(found & (1u << q))) a.quant[k * (long long)a.nq + q] = nan;
    }
  });
}

// ---------------------------------------------------------------------------
// launch configuration of the column kernels
// ---------------------------------------------------------------------------
template <typename F>
static hipError_t allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// lanes per column (the statistics and field lines; the matrix always gives a
// column a whole wave, whose lanes then share the target cells) and rounds
// per column, rounded up to the instantiated sizes
static int col_lpc(int B) { return B <= 1024 ? 16 : 64; }
static int col_rounds(int B, int lpc) {
  const int rs = 4 * lpc;
  const int r = (B + rs - 1) / rs;
  return r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : r <= 8 ? 8 : 16;
}

// waves per workgroup: 4 unless the per-wave LDS does not fit 64 KiB
static int col_waves(size_t fixed, size_t per_wave) {
  int w = 4;
  while (w > 1 && fixed + per_wave * w > 65536) --w;
  return w;
}

static unsigned col_grid(long long K, int lpc, int waves) {
  const long long per_block = (long long)waves * (64 / lpc);
  const long long need = (K + per_block - 1) / per_block;
  return (unsigned)(need < 2048 ? need : 2048);
}

#define VUP_COL_CASE(NAME, LPC, MV)                        \
  case (LPC == 16 ? 0 : 100) + MV * 2: kern = NAME<LPC, MV, false>; break; \
  case (LPC == 16 ? 0 : 100) + MV * 2 + 1: kern = NAME<LPC, MV, true>; break;

#define VUP_COL_KERNEL_TABLE(NAME, ARGS)                                                        \
  static hipError_t launch_##NAME(const ARGS& a, int lpc, bool vec, int waves, size_t bytes,      \
                                  hipStream_t s) {                                                \
    void (*kern)(ARGS) = nullptr;                                                                 \
    switch ((lpc == 16 ? 0 : 100) + col_rounds(a.B, lpc) * 2 + (vec ? 1 : 0)) {                   \
      VUP_COL_CASE(NAME, 16, 1)                                                                   \
      VUP_COL_CASE(NAME, 16, 2)                                                                   \
      VUP_COL_CASE(NAME, 16, 4)                                                                   \
      VUP_COL_CASE(NAME, 16, 8)                                                                   \
      VUP_COL_CASE(NAME, 16, 16)                                                                  \
      VUP_COL_CASE(NAME, 64, 1)                                                                   \
      VUP_COL_CASE(NAME, 64, 2)                                                                   \
      VUP_COL_CASE(NAME, 64, 4)                                                                   \
      VUP_COL_CASE(NAME, 64, 8)                                                                   \
      VUP_COL_CASE(NAME, 64, 16)                                                                  \
      default: return hipErrorInvalidValue;                                                       \
    }                                                                                             \
    hipError_t e = allow_lds(kern, bytes);                                                        \
    if (e != hipSuccess) return e;                                                                \
    hipLaunchKernelGGL(kern, dim3(col_grid(a.K, lpc, waves)), dim3(64 * waves), bytes, s, a);     \
    return hipGetLastError();                                                                     \
  }

VUP_COL_KERNEL_TABLE(k_ipsa, StatArgs)
VUP_COL_KERNEL_TABLE(k_ipsa_matrix, MatrixArgs)
VUP_COL_KERNEL_TABLE(k_ipsa_fields, FieldArgs)
#undef VUP_COL_KERNEL_TABLE
#undef VUP_COL_CASE

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

hipError_t launch_ipsa_stats(const double* edges, int B, int64_t K, const float* P,
                             double* mean_hist, double* var, double* entropy, hipStream_t s) {
  if (K == 0) return hipSuccess;
  StatArgs a{P, edges, (long long)K, B, mean_hist, var, entropy};
  const size_t bytes = (size_t)B * sizeof(double);
  return launch_k_ipsa(a, col_lpc(B), B % 4 == 0 && aligned16(P), 4, bytes, s);
}

hipError_t launch_ipsa_matrix(const double* edges, int B, int64_t K, const float* P,
                              const double* y_ref, double dy_lo, double dy_width, int n_dy,
                              float* Q, double* lost, hipStream_t s) {
  if (K == 0) return hipSuccess;
  MatrixArgs a{};
  a.P = P;
  a.edges = edges;
  a.y_ref = y_ref;
  a.K = K;
  a.B = B;
  a.dy_lo = dy_lo;
  a.dy_width = dy_width;
  a.J = n_dy;
  const int lpc = 64;
  a.Q = Q;
  a.lost = lost;
  const size_t fixed = (size_t)(2 * B + 1) * sizeof(double);
  const size_t per_wave = (size_t)(64 / lpc) * (B + 1) * sizeof(double);
  const int waves = col_waves(fixed, per_wave);
  return launch_k_ipsa_matrix(a, lpc, B % 4 == 0 && aligned16(P), waves, fixed + per_wave * waves,
                              s);
}

hipError_t launch_ipsa_fields(const double* edges, int B, int64_t K, const float* P,
                              const double* y_ref, int n_levels, const double* levels,
                              double* y_mode, double* p_max, double* quant, double* dev,
                              double* delta2, hipStream_t s) {
  if (K == 0) return hipSuccess;
  FieldArgs a{};
  a.P = P;
  a.edges = edges;
  a.y_ref = y_ref;
  a.K = K;
  a.B = B;
  a.nq = quant ? n_levels : 0;
  for (int q = 0; q < n_levels && q < kMaxLevels; ++q) a.level[q] = levels[q];
  a.y_mode = y_mode;
  a.p_max = p_max;
  a.quant = quant;
  a.dev = dev;
  a.delta2 = delta2;
  const size_t bytes = (size_t)(2 * B + 1 + kMaxLevels) * sizeof(double);
  return launch_k_ipsa_fields(a, col_lpc(B), B % 4 == 0 && aligned16(P), 4, bytes, s);
}

// ---------------------------------------------------------------------------
// marginal over locations
// ---------------------------------------------------------------------------
constexpr int kMargCols = 256;  // columns per workgroup of the partial sums

int marginal_chunks(int64_t K, int n) {
  if (K <= 0 || n <= 0) return 0;
  const long long tiles = (n + kMargCols - 1) / kMargCols;
  long long c = (2048 + tiles - 1) / tiles;     // about 2048 workgroups in all
  const long long max_by_rows = (K + 7) / 8;   // at least 8 rows per chunk
  if (c > max_by_rows) c = max_by_rows;
  if (c > 65535) c = 65535;
  return (int)(c < 1 ? 1 : c);
}

size_t marginal_workspace_bytes(int64_t K, int n) {
  return (size_t)marginal_chunks(K, n) * (size_t)(n > 0 ? n : 0) * sizeof(double);
}

// part[chunk][j] = sum over the chunk's rows r, in order, of w_r A[r][j]
__global__ __launch_bounds__(256) void k_marg_partial(const float* __restrict__ A, long long K,
                                                      int n, const double* __restrict__ rho,
                                                      double w_uniform, long long rows,
                                                      double* __restrict__ part) {
  const int j = blockIdx.x * kMargCols + threadIdx.x;
  if (j >= n) return;
  const long long r0 = (long long)blockIdx.y * rows;
  const long long r1 = min(K, r0 + rows);
  double acc = 0.0;
  long long r = r0;
  for (; r + 8 <= r1; r += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = A[(r + u) * n + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (rho ? rho[r + u] : w_uniform) * (double)v[u];
  }
  for (; r < r1; ++r) acc += (rho ? rho[r] : w_uniform) * (double)A[r * n + j];
  part[(long long)blockIdx.y * n + j] = acc;
}

// out[j] = sum over chunks of part[chunk][j]: one wave per column, lanes take
// chunks lane, lane + 64, ... and the wave sum fixes the order
__global__ __launch_bounds__(64) void k_marg_combine(const double* __restrict__ part, int chunks,
                                                     int n, double* __restrict__ out) {
  const int j = blockIdx.x;
  double s = 0.0;
#pragma unroll 8
  for (int c = threadIdx.x; c < chunks; c += 64) s += part[(long long)c * n + j];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[j] = s;
}

hipError_t launch_marginalize(int64_t K, int n, const float* A, const double* rho, void* ws,
                              double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int chunks = marginal_chunks(K, n);
  double* part = static_cast<double*>(ws);
  if (chunks > 0) {
    const long long rows = (K + chunks - 1) / chunks;
    const unsigned tiles = (unsigned)((n + kMargCols - 1) / kMargCols);
    hipLaunchKernelGGL(k_marg_partial, dim3(tiles, (unsigned)chunks), dim3(kMargCols), 0, s, A,
                       (long long)K, n, rho, 1.0 / (double)K, rows, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_marg_combine, dim3((unsigned)n), dim3(64), 0, s, part, chunks, n, out);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// marginal without a caller workspace: the partial sums live in a file-scope
// device array of kStaticMarginalBytes, one copy per GPU for the life of the
// process. Host code never passes the array's name to a kernel (on the host
// it is a stand-in, not a device address); it passes the address
// hipGetSymbolAddress returns for the current device, looked up on the first
// call on that device and kept. Every partial sum is written before it is
// read, so nothing needs clearing between calls; calls that overlap on one
// GPU share the array and race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double g_marginal_scratch[kStaticMarginalBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static hipError_t marginal_scratch_for_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_marginal_scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_marginalize_static(int64_t K, int n, const float* A, const double* rho,
                                     double* out, hipStream_t s) {
  if (marginal_workspace_bytes(K, n) > kStaticMarginalBytes) return hipErrorInvalidValue;
  void* part = nullptr;
  const hipError_t e = marginal_scratch_for_current_device(&part);
  if (e != hipSuccess) return e;
  return launch_marginalize(K, n, A, rho, part, out, s);
}

}  // namespace vup
