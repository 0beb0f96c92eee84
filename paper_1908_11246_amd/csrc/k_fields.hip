// Sensitivity views of the propagated output matrix (Sec. 5.2) and the model
// at the input pdfs' maxima (Sec. 5.3):
//   k_eval_points    y_i = M(x_i) at caller-given points, FP64
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
// The column kernels give one wave64 to one column at a time. Lane l owns the
// bins [l*m, l*m + m), m = ceil(B/64): it reads them (coalesced across the
// wave), keeps their running sum, and after an exclusive scan of the lane
// totals writes C_b = sum_{b'<b} P_b' (FP64) into the wave's LDS slice. The
// bin edges sit once per workgroup in LDS. All HBM traffic is one read of P
// and one write of the outputs.
#include <hip/hip_runtime.h>

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
// shared pieces of the column kernels
// ---------------------------------------------------------------------------
struct ColArgs {
  const double* edges;  // [B+1]
  const float* P;       // [K][B]
  const double* y_ref;  // [K]
  long long K;
  int B;
  int m;       // bins per lane, ceil(B/64)
  int waves;   // columns in flight per workgroup (one per wave)
  int c_off;   // doubles from the start of LDS to the first wave's CDF
};

struct MatrixArgs {
  ColArgs c;
  double dy_lo, dy_width;
  int J;       // target cells
  int mt;      // target cells per lane, ceil(J/64)
  float* Q;    // [K][J]
  double* lost;
};

struct FieldArgs {
  ColArgs c;
  int nq;
  double level[kMaxLevels];
  double* y_mode;
  double* p_max;
  double* quant;  // [K][nq]
  double* dev;
  double* delta2;
};

__device__ __forceinline__ double shfl_up1(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __shfl_up((int)(b & 0xFFFFFFFF), 1, 64);
  const int hi = __shfl_up((int)(b >> 32), 1, 64);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// copy the edges into LDS (whole workgroup)
__device__ __forceinline__ void stage_edges(const ColArgs& a, double* E) {
  for (int b = threadIdx.x; b <= a.B; b += blockDim.x) E[b] = a.edges[b];
}

// FP64 CDF of one column into C[0..B]; returns T = C[B] (uniform). `visit`
// sees every (bin, P value) the lane owns, in increasing bin order.
template <class Visit>
__device__ __forceinline__ double build_cdf(const ColArgs& a, long long k, double* C, Visit&& visit) {
  const int lane = threadIdx.x & 63;
  const int b0 = lane * a.m;
  const float* col = a.P + k * (long long)a.B;
  double run = 0.0;
  for (int i = 0; i < a.m; ++i) {
    const int b = b0 + i;
    if (b < a.B) {
      const float p = col[b];
      C[b] = run;
      run += (double)p;
      visit(b, p);
    }
  }
  const double incl = wave_scan(run);
  double off = shfl_up1(incl);
  if (lane == 0) off = 0.0;
  const double T = lane_value(incl, 63);
  for (int i = 0; i < a.m; ++i) {
    const int b = b0 + i;
    if (b < a.B) C[b] = off + C[b];
  }
  if (lane == 0) C[a.B] = T;
  return T;
}

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
__device__ __forceinline__ double cdf_at(const double* E, const double* C, int B, double T, int cnt,
                                         double t) {
  if (cnt == 0) return 0.0;
  if (cnt > B) return T;
  const int b = cnt - 1;
  const double frac = (t - E[b]) / (E[b + 1] - E[b]);
  return C[b] + (C[b + 1] - C[b]) * frac;
}

// target grid point d_j = d_lo + j*h (one multiply, one add, no contraction),
// moved into output coordinates by y
__device__ __forceinline__ double target_point(double dlo, double h, int j, double y) {
  return __dadd_rn(__dadd_rn(dlo, __dmul_rn((double)j, h)), y);
}

// ---------------------------------------------------------------------------
// IPSA probability matrix
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ipsa_matrix(MatrixArgs a) {
  extern __shared__ double lds[];
  double* E = lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* C = lds + a.c.c_off + wave * (a.c.B + 1);
  const int B = a.c.B;
  stage_edges(a.c, E);
  const long long per_iter = (long long)gridDim.x * a.c.waves;
  for (long long base = (long long)blockIdx.x * a.c.waves; base < a.c.K; base += per_iter) {
    __syncthreads();  // edges staged / previous column's CDF no longer read
    const long long k = base + wave;
    const bool active = wave < a.c.waves && k < a.c.K;
    double T = 0.0;
    if (active) T = build_cdf(a.c, k, C, [](int, float) {});
    __syncthreads();
    if (!active) continue;
    const int j0 = lane * a.mt;
    const int j1 = min(a.J, j0 + a.mt);
    float* q = a.Q + k * (long long)a.J;
    const int last = (a.J - 1) / a.mt;  // lane owning the last target cell
    if (!isfinite(T)) {
      for (int j = j0; j < j1; ++j) q[j] = __builtin_nanf("");
      if (lane == 0 && a.lost) a.lost[k] = __builtin_nan("");
      continue;
    }
    const double y = a.c.y_ref[k];
    double F_first = 0.0, F_end = 0.0;
    if (j0 < j1) {
      double t = target_point(a.dy_lo, a.dy_width, j0, y);
      int cnt = count_le(E, B, t);
      double F = cdf_at(E, C, B, T, cnt, t);
      F_first = F;
      for (int j = j0; j < j1; ++j) {
        t = target_point(a.dy_lo, a.dy_width, j + 1, y);
        while (cnt <= B && E[cnt] <= t) ++cnt;
        const double Fn = cdf_at(E, C, B, T, cnt, t);
        q[j] = (float)(Fn - F);
        F = Fn;
      }
      F_end = F;
    }
    const double lo_part = lane_value(F_first, 0);
    const double hi_part = lane_value(F_end, last);
    if (lane == 0 && a.lost) a.lost[k] = lo_part + (T - hi_part);
  }
}

// ---------------------------------------------------------------------------
// field lines
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ipsa_fields(FieldArgs a) {
  extern __shared__ double lds[];
  double* E = lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* C = lds + a.c.c_off + wave * (a.c.B + 1);
  const int B = a.c.B;
  const double nan = __builtin_nan("");
  stage_edges(a.c, E);
  const long long per_iter = (long long)gridDim.x * a.c.waves;
  for (long long base = (long long)blockIdx.x * a.c.waves; base < a.c.K; base += per_iter) {
    __syncthreads();
    const long long k = base + wave;
    const bool active = wave < a.c.waves && k < a.c.K;
    const double y = (active && a.c.y_ref) ? a.c.y_ref[k] : 0.0;
    float vmax = -__builtin_inff();
    int imax = B;
    double s1 = 0.0, s2 = 0.0;
    double T = 0.0;
    if (active) {
      T = build_cdf(a.c, k, C, [&](int b, float p) {
        if (p > vmax) {
          vmax = p;
          imax = b;
        }
        const double t = 0.5 * (E[b] + E[b + 1]) - y;
        const double pt = (double)p * t;
        s1 += pt;
        s2 += pt * t;
      });
    }
    __syncthreads();
    if (!active) continue;
    // first maximum over the wave: larger value wins, equal values keep the lower bin
    for (int o = 32; o >= 1; o >>= 1) {
      const float ov = __shfl_xor(vmax, o, 64);
      const int oi = __shfl_xor(imax, o, 64);
      if (ov > vmax || (ov == vmax && oi < imax)) {
        vmax = ov;
        imax = oi;
      }
    }
    const double S1 = wave_sum(s1);
    const double S2 = wave_sum(s2);
    const bool finite = isfinite(T);
    const bool positive = finite && T > 0.0;
    if (lane == 0) {
      if (a.p_max) a.p_max[k] = finite ? (double)vmax : nan;
      if (a.y_mode) a.y_mode[k] = positive ? 0.5 * (E[imax] + E[imax + 1]) : nan;
      if (a.dev) a.dev[k] = finite ? S1 : nan;
      if (a.delta2) a.delta2[k] = finite ? 0.5 * S2 : nan;
    }
    if (!a.quant) continue;
    const int b0 = lane * a.c.m;
    const int b1 = min(B, b0 + a.c.m);
    const float* col = a.c.P + k * (long long)B;
#pragma unroll
    for (int q = 0; q < kMaxLevels; ++q) {
      if (q < a.nq) {
        const double target = a.level[q] * T;
        const bool mine = positive && b0 < b1 && C[b0] < target && target <= C[b1];
        const unsigned long long mask = __ballot(mine);
        double* out = a.quant + k * (long long)a.nq + q;
        if (mask == 0ull) {
          if (lane == 0) *out = nan;
        } else if (lane == __ffsll((long long)mask) - 1) {
          int b = b0;
          while (b < b1 - 1 && C[b + 1] < target) ++b;
          const double pb = (double)col[b];
          if (pb > 0.0) {
            const double frac = fmin(fmax((target - C[b]) / pb, 0.0), 1.0);
            *out = E[b] + frac * (E[b + 1] - E[b]);
          } else {
            // reached only when rounding puts the level an ulp past the end
            // of the last positive bin before an empty stretch: answer that
            // bin's right edge
            int bb = b;
            while (bb > b0 && col[bb] == 0.0f) --bb;
            *out = col[bb] > 0.0f ? E[bb + 1] : E[b0];
          }
        }
      }
    }
  }
}

// LDS layout: edges, then one CDF per wave; as many waves as fit in 64 KiB
// (at least one, with the limit raised above 64 KiB when B needs it)
static void col_layout(int B, int* waves, int* c_off, size_t* bytes) {
  const size_t per = (size_t)(B + 1) * sizeof(double);
  int w = kWaves;
  while (w > 1 && per * (1 + w) > 65536) --w;
  *waves = w;
  *c_off = B + 1;
  *bytes = per * (1 + w);
}

template <typename F>
static hipError_t allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static ColArgs col_args(const double* edges, int B, int64_t K, const float* P, const double* y_ref,
                        size_t* bytes) {
  ColArgs c{};
  c.edges = edges;
  c.P = P;
  c.y_ref = y_ref;
  c.K = K;
  c.B = B;
  c.m = (B + 63) / 64;
  col_layout(B, &c.waves, &c.c_off, bytes);
  return c;
}

static unsigned col_blocks(const ColArgs& c) {
  const long long need = (c.K + c.waves - 1) / c.waves;
  return (unsigned)(need < 4096 ? need : 4096);
}

hipError_t launch_ipsa_matrix(const double* edges, int B, int64_t K, const float* P,
                              const double* y_ref, double dy_lo, double dy_width, int n_dy,
                              float* Q, double* lost, hipStream_t s) {
  if (K == 0) return hipSuccess;
  MatrixArgs a{};
  size_t bytes = 0;
  a.c = col_args(edges, B, K, P, y_ref, &bytes);
  a.dy_lo = dy_lo;
  a.dy_width = dy_width;
  a.J = n_dy;
  a.mt = (n_dy + 63) / 64;
  a.Q = Q;
  a.lost = lost;
  hipError_t e = allow_lds(k_ipsa_matrix, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ipsa_matrix, dim3(col_blocks(a.c)), dim3(kThreads), bytes, s, a);
  return hipGetLastError();
}

hipError_t launch_ipsa_fields(const double* edges, int B, int64_t K, const float* P,
                              const double* y_ref, int n_levels, const double* levels,
                              double* y_mode, double* p_max, double* quant, double* dev,
                              double* delta2, hipStream_t s) {
  if (K == 0) return hipSuccess;
  FieldArgs a{};
  size_t bytes = 0;
  a.c = col_args(edges, B, K, P, y_ref, &bytes);
  a.nq = quant ? n_levels : 0;
  for (int q = 0; q < n_levels && q < kMaxLevels; ++q) a.level[q] = levels[q];
  a.y_mode = y_mode;
  a.p_max = p_max;
  a.quant = quant;
  a.dev = dev;
  a.delta2 = delta2;
  hipError_t e = allow_lds(k_ipsa_fields, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ipsa_fields, dim3(col_blocks(a.c)), dim3(kThreads), bytes, s, a);
  return hipGetLastError();
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

}  // namespace vup
