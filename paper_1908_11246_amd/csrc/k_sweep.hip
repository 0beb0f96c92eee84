// Window sweeps over the shared model matrix: propagation (eq. VUP), exact-f
// moments, and the adjoint sweep of the IPSA sensitivities.
//
// One workgroup (256 threads, 4 waves) handles one distribution k and loops
// over its mixture components. For each component:
//   1. the truncation window is computed per axis (FP64, exact op order) and
//      the per-axis Gaussian factors g_d(j) are tabulated in LDS (FP32);
//   2. cell form: the window is swept as rows (all axes but the fastest) x
//      strips of SW consecutive cells of the fastest axis, aligned to SW in
//      the padded bin map. A thread keeps its strip's factors in registers and
//      walks rows; the row factor (product of the slower axes' factors) and
//      the row's bin-map offset come from a row table in LDS. Per cell the
//      density is one FP32 multiply;
//      run form (FP32 propagation and the adjoint): each row of the window is
//      a sequence of runs of equal bin, and the density is separable, so a
//      run's sums are differences of prefix sums of the fastest-axis factors;
//   3. propagation accumulates into the bins' LDS slots as 32-bit fixed-point
//      integers (LDS float atomics are two orders of magnitude slower than
//      integer ones on gfx950), split into magnitude classes with one
//      histogram and one scale each so that tail cells keep a fine quantum
//      (see the fixed-point notes below). Integer sums are exact, so results
//      do not depend on scheduling. Moments and the adjoint keep per-thread
//      sums reduced in a fixed order.
// The input probability matrix is never materialised.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "vup_device.hpp"
#include "vup_internal.hpp"

namespace vup {

struct SweepArgs {
  GridDev g;
  DistsDev d;
  int B;
  const uint16_t* __restrict__ binmap;
  const float* __restrict__ f32;
  const double* __restrict__ edges;
  unsigned long long* counters;
  SweepLayout L;
  long long kpx;  // distributions per XCD slot (block -> k mapping)
  // run-length form of the model matrix (propagation, FP32)
  const uint32_t* __restrict__ runs;
  const int* __restrict__ rowptr;
  const uint16_t* __restrict__ runidx;
  long long ncells;
  int allow_runs;
  // propagate
  float* P;
  double* Z;
  // moments
  double* mean;
  double* var;
  double* delta2;
  vup_model model;
  int has_model;
  // backward
  const float* Pin;
  const double* mean_hist;
  const double* g_var;
  const double* g_ent;
  double* g_mu;
  double* g_sigma;
  double* g_weight;
};

// element i < 4 of a small array of the kernel arguments, by selects rather
// than an indexed load (a runtime index would copy the array to private memory)
template <typename T>
__device__ __forceinline__ T pick4(const T (&v)[4], int i) {
  return i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
}

// per-component window state, identical in every thread of the workgroup
struct Win {
  int lo[4];
  int W[4];
  long long R;  // rows
  bool bad;
  bool empty;
};

// Window of component kc. Lanes 0..3 of wave 0 compute one axis each (FP64,
// the exact formula of axis_window, and the axis's scale exponent) into LDS
// (`wsh`, 16 ints); every thread then reads the result. Contains two
// workgroup barriers.
__device__ __forceinline__ Win make_win(const SweepArgs& a, long long kc, int* wsh) {
  const int D = a.g.ndim;
  __syncthreads();  // earlier readers of wsh are done
  if (threadIdx.x < 4) {
    const int d = threadIdx.x;
    int jlo = 0, jhi = 0, flags = 0, m = 0;
    if (d < D) {
      const double mu = a.d.mu[kc * D + d], sg = a.d.sigma[kc * D + d];
      const bool ok = axis_window(a.g.lo[d], a.g.hi[d], a.g.n[d], mu, sg, a.d.ns, jlo, jhi);
      flags = (ok ? 0 : 1) | (jhi < jlo ? 2 : 0);
      // a window of several cells holds only cells within n_sigma sigma of the
      // mean, so m = 0 there unless n_sigma reaches about 5.27 (axis_scale_exp)
      if (ok && jhi >= jlo && (jhi == jlo || a.d.ns >= 5.25))
        m = axis_scale_exp(a.g.lo[d], a.g.hi[d], a.g.n[d], jlo, jhi, mu, 1.0 / sg);
    }
    wsh[d] = jlo;
    wsh[4 + d] = jhi - jlo + 1;
    wsh[8 + d] = flags;
    wsh[12 + d] = m;
  }
  __syncthreads();
  // the values are uniform: keep them in scalar registers
  Win w;
  w.R = 1;
  const int flags = __builtin_amdgcn_readfirstlane(wsh[8] | wsh[9] | wsh[10] | wsh[11]);
  w.bad = (flags & 1) != 0;
  w.empty = (flags & 2) != 0;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    w.lo[d] = __builtin_amdgcn_readfirstlane(wsh[d]);
    w.W[d] = __builtin_amdgcn_readfirstlane(wsh[4 + d]);
    if (d + 1 < D) w.R *= (w.W[d] > 0 ? w.W[d] : 0);
  }
  return w;
}

// scale exponent of axis d of the current window (make_win leaves it in LDS
// after the window ints; one uniform LDS read where a table needs it)
__device__ __forceinline__ int win_m(const SweepArgs& a, const float* smem, int d) {
  return __builtin_amdgcn_readfirstlane(
      reinterpret_cast<const int*>(smem + a.L.red_off + 80)[12 + d]);
}

// fastest-axis window bounds (avoids dynamic indexing of the Win arrays)
__device__ __forceinline__ void last_axis(const Win& w, int D, int& lo, int& W) {
  lo = w.lo[0];
  W = w.W[0];
#pragma unroll
  for (int d = 1; d < 4; ++d)
    if (d == D - 1) {
      lo = w.lo[d];
      W = w.W[d];
    }
}

// block -> distribution: consecutive blocks are spread over the 8 XCDs, so a
// contiguous range of distributions (overlapping windows) shares one L2.
__device__ __forceinline__ long long block_k(const SweepArgs& a) {
  const long long b = blockIdx.x;
  return (b & 7) * a.kpx + (b >> 3);
}

// strip width minimising the sweep time estimate of one component: passes
// over the rows times (cells of a strip + a per-row cost of three cells'
// worth, the measured best of the values tried)
__device__ __forceinline__ int choose_sw(int loL, int WL, long long R, int maxsw) {
  int best = 4;
  long long bestc = 0x7fffffffffffffffll;
  for (int sw = 4; sw <= maxsw; sw *= 2) {
    const int ns = (loL + WL - 1) / sw - loL / sw + 1;
    const int cols = ns < kThreads ? ns : kThreads;
    const int P0 = kThreads / cols;
    const long long ncg = (ns + kThreads - 1) / kThreads;
    const long long c = ((R + P0 - 1) / P0) * ncg * (sw + 3);
    if (c < bestc) {
      bestc = c;
      best = sw;
    }
  }
  return best;
}

// Build per-axis factor tables for the window of component kc. Outer axes
// d < D-1: tab_d[i] = g_d(lo_d + i), i < W_d. Fastest axis: tab_L[jj] for
// jj < ns*sw, cell colbase + jj, zero outside the window.
__device__ __forceinline__ void build_tables(const SweepArgs& a, float* smem, const Win& w,
                                             long long kc, int sw, int colbase, int ns) {
  const int D = a.g.ndim;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d + 1 < D) {
      float* tab = smem + a.L.tab_off[d];
      const double mu = a.d.mu[kc * D + d], rsig = 1.0 / a.d.sigma[kc * D + d];
      const double off = scale_log(win_m(a, smem, d));
      for (int i = threadIdx.x; i < w.W[d]; i += kThreads) {
        const double x = cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], w.lo[d] + i);
        tab[i] = gauss_factor_r(x, mu, rsig, off);
      }
    }
  }
  const int L = D - 1;
  int loL, WL;
  last_axis(w, D, loL, WL);
  float* tab = smem + pick4(a.L.tab_off, L);
  const double mu = a.d.mu[kc * D + L], rsig = 1.0 / a.d.sigma[kc * D + L];
  const double off = scale_log(win_m(a, smem, L));
  for (int jj = threadIdx.x; jj < ns * sw; jj += kThreads) {
    const int j = colbase + jj;
    float v = 0.0f;
    if (j >= loL && j < loL + WL) {
      const double x = cell_centre(pick4(a.g.lo, L), pick4(a.g.hi, L), pick4(a.g.n, L), j);
      v = gauss_factor_r(x, mu, rsig, off);
    }
    tab[jj] = v;
  }
}

// Row table for rows [r0, r0 + rc): row factor (product of the slower axes'
// factors) and element offset of the row in the padded bin map. With
// `trow`, also the standardised coordinates t_d of the slower axes.
__device__ __forceinline__ void build_rows(const SweepArgs& a, float* smem, const Win& w,
                                           long long r0, int rc, long long kc, bool trow) {
  const int D = a.g.ndim;
  float2* rt = reinterpret_cast<float2*>(smem + a.L.row_off);
  float4* tt = trow ? reinterpret_cast<float4*>(smem + a.L.trow_off) : nullptr;
  for (int r = threadIdx.x; r < rc; r += kThreads) {
    int t = (int)r0 + r;
    float go = 1.0f;
    int off = 0;  // the padded bin map has fewer than 2^31 elements
    float tv[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int d = 2; d >= 0; --d) {
      if (d <= D - 2) {
        const int i = d == 0 ? t : t % w.W[d];
        if (d > 0) t /= w.W[d];
        go *= smem[a.L.tab_off[d] + i];
        off += (w.lo[d] + i) * (int)a.g.rowstride[d];
        if (trow) {
          const double x = cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], w.lo[d] + i);
          tv[d] = (float)((x - a.d.mu[kc * D + d]) / a.d.sigma[kc * D + d]);
        }
      }
    }
    rt[r] = make_float2(go, __int_as_float(off));
    if (trow) tt[r] = make_float4(tv[0], tv[1], tv[2], 0.0f);
  }
}

template <int SW>
struct MapVec {
  uint32_t v[SW / 2];
};

template <int SW>
__device__ __forceinline__ MapVec<SW> load_map(const uint16_t* __restrict__ p) {
  MapVec<SW> m;
  if constexpr (SW == 4) {
    const uint2 q = *reinterpret_cast<const uint2*>(p);
    m.v[0] = q.x;
    m.v[1] = q.y;
  } else {
#pragma unroll
    for (int i = 0; i < SW / 8; ++i) {
      const uint4 q = reinterpret_cast<const uint4*>(p)[i];
      m.v[4 * i + 0] = q.x;
      m.v[4 * i + 1] = q.y;
      m.v[4 * i + 2] = q.z;
      m.v[4 * i + 3] = q.w;
    }
  }
  return m;
}

template <int SW>
__device__ __forceinline__ uint32_t map_at(const MapVec<SW>& m, int j) {
  return (j & 1) ? (m.v[j >> 1] >> 16) : (m.v[j >> 1] & 0xFFFFu);
}

// ===========================================================================
// propagation
// ===========================================================================
// ---------------------------------------------------------------------------
// Fixed-point histogram accumulation.
// Densities are accumulated as 32-bit fixed-point integers with integer LDS
// atomics: exact, independent of scheduling, and not limited by the rate of
// LDS float atomics. A component's scale is K / (qfac * bound of its mass),
// K = 2^32 - 2^20 - (cells), qfac >= 1 the largest relative increase of a
// density by the precision's rounding, so no total can overflow; a cell adds
// floor(w * scale + u) with a fixed dither u in (0, 1), so rounding is unbiased
// on average and cells below one quantum still count.
// Cell form: the LDS holds NC copies of the histogram interleaved by bin (bin
// b, copy c at word b NC + c); the cells of strip s (of SW fastest-axis cells)
// in window row r go to copy (s + r cols) mod NC, cols being the strips a
// workgroup walks side by side, so the NC lanes next to each other use NC
// different copies and a wave's random bin addresses spread over the banks.
// Each copy has its own scale from its exact mass, a cyclic convolution of the
// strip masses by residue mod NC with the row-factor sums by residue (which
// factor over the axes), so its quantum is about 1/NC of the component's. The
// dither is a 16-row by SW-column ordered pattern, u = j/SW + (r mod 16 +
// 1/2) / (16 SW), whose 16 SW values over a block are all distinct, so in a
// smooth region the rounding bias averages to at most 1/(32 SW) quantum.
// Run form: three classes by the row factor (>= 2^-4, >= 2^-8, smaller), one
// stacked histogram each, and a per-thread dither (see below).
// ---------------------------------------------------------------------------
constexpr float kClassT1 = 0.0625f;      // 2^-4
constexpr float kClassT2 = 0.00390625f;  // 2^-8

__device__ __forceinline__ int mag_class(float g) {
  return g >= kClassT1 ? 0 : (g >= kClassT2 ? 1 : 2);
}

template <int PREC>
__host__ __device__ constexpr double prec_qfac() {
  return PREC == VUP_BF16 ? 1.0 + 1.0 / 256 : PREC == VUP_BF16X2 ? 1.0 + 1.0 / 65536
         : PREC == VUP_FP8E4M3 ? 1.125 : 1.0 + 1.0 / 1048576;
}

// the model matrix's run form is used for this propagation (FP32 densities):
// forced by the sweep mode, or chosen when runs along the fastest axis are at
// least kRunMinLength cells long on average
__device__ __forceinline__ bool runs_chosen(const SweepArgs& a) {
  if (!a.allow_runs) return false;
  const unsigned long long mode = a.counters[kCntMode];
  const unsigned long long nruns = a.counters[kCntRuns];
  return nruns > 0 && (mode == VUP_SWEEP_RUNS ||
                       (mode == VUP_SWEEP_AUTO && (long long)nruns * kRunMinLength <= a.ncells));
}

// Row factor sum bound of the window: product over the slower axes of their
// factor table sums (FP64).
__device__ __forceinline__ double row_mass(const SweepArgs& a, const float* smem, const Win& w,
                                           double* red) {
  const int D = a.g.ndim;
  double Zrows = 1.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d + 1 < D) {
      double zp = 0.0;
      for (int i = threadIdx.x; i < w.W[d]; i += kThreads) zp += (double)smem[a.L.tab_off[d] + i];
      Zrows *= block_sum(zp, red);
    }
  }
  return Zrows;
}

// Factor tables of the cell-form propagation: every axis' factors from the
// FP64 exponential, each rounded once to FP32. Outer axes d < D-1:
// tab_d[i] = g_d(lo_d + i), i < W_d. Fastest axis: tab_L[jj] for jj < ns*sw,
// cell colbase + jj, zero outside the window.
// exp(a) for a <= 0 in FP64 with few registers: a = n ln2 + r, |r| <= ln2/2,
// ln 2 split in a head and a tail (Cody and Waite's argument reduction), and
// exp(r) by its Taylor series to degree 11 (truncation below 3e-13 relative),
// so the FP32 rounding of the result is the correctly rounded value except
// within about 2^-40 of a rounding tie.
__device__ __forceinline__ double exp_nonpos(double a) {
  if (a < -745.0) return 0.0;
  const double n = rint(a * 1.4426950408889634);     // a / ln 2
  double r = fma(-n, 0.6931471805599453, a);          // ln 2, head
  r = fma(-n, 2.3190468138462996e-17, r);             // ln 2, tail
  double p = 1.0 / 39916800.0;                        // 1/11!
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)n);
}

// scaled by 2^m as gauss_factor_r, off = scale_log(m) (axis_scale_exp keeps
// the argument <= 0)
__device__ __forceinline__ float gauss_factor_exact(double x, double mu, double rsig,
                                                    double off) {
  const double t = (x - mu) * rsig;
  return (float)exp_nonpos(fma(-0.5, t * t, off));
}

__device__ __forceinline__ void build_tables_exact(const SweepArgs& a, float* smem, const Win& w,
                                                   long long kc, int sw, int colbase, int ns) {
  const int D = a.g.ndim;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d + 1 < D) {
      float* tab = smem + a.L.tab_off[d];
      const double mu = a.d.mu[kc * D + d], rsig = 1.0 / a.d.sigma[kc * D + d];
      const double off = scale_log(win_m(a, smem, d));
      for (int i = threadIdx.x; i < w.W[d]; i += kThreads)
        tab[i] = gauss_factor_exact(cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], w.lo[d] + i), mu,
                                    rsig, off);
    }
  }
  const int L = D - 1;
  int loL, WL;
  last_axis(w, D, loL, WL);
  float* tab = smem + pick4(a.L.tab_off, L);
  const double mu = a.d.mu[kc * D + L], rsig = 1.0 / a.d.sigma[kc * D + L];
  const double off = scale_log(win_m(a, smem, L));
  for (int jj = threadIdx.x; jj < ns * sw; jj += kThreads) {
    const int j = colbase + jj;
    float v = 0.0f;
    if (j >= loL && j < loL + WL)
      v = gauss_factor_exact(cell_centre(pick4(a.g.lo, L), pick4(a.g.hi, L), pick4(a.g.n, L), j),
                             mu, rsig, off);
    tab[jj] = v;
  }
}

// sum over the axes of component kc of their scale exponents m
// (axis_scale_exp): the factor tables' products, and the masses summed from
// them, are 2^sum times the densities'
__device__ __forceinline__ int win_scale_exp(const SweepArgs& a, const float* smem) {
  int s = 0;
  for (int d = 0; d < a.g.ndim; ++d) s += win_m(a, smem, d);
  return s;
}

// per-copy scales of the cell form, shared by all threads (LDS)
struct PropScales {
  double scale[16];    // fixed-point units per unit of density, per copy
  double unscale[16];  // 1 / scale (0 for a copy without cells)
  int mexp;            // win_scale_exp of the component
  float scalef[16];    // scale rounded to FP32
};
constexpr int kPropScalesFloats = (int)(sizeof(PropScales) / sizeof(float));
constexpr int kPropScaleScratch = 16 + 16 + 256 + 16;  // doubles: A, G, partials, S

// Exact mass of each histogram copy of component kc (the copy of strip s in
// window row r is (s + r cols) mod nc) and its scale K / (qfac mass). With A[a]
// the factor mass of the strips s = a (mod nc) and S[b] the row-factor mass of
// the rows r = b (mod nc), copy c holds the sum over a + b cols = c (mod nc) of
// A[a] S[b]. Rows are flat indices over the slower axes (axis 0 slowest), so
// with x the last slower axis (W_x cells), row r = o W_x + i_x and
// S[b] = sum over the outer rows o of go(o) G[(b - o W_x) mod nc], G[e] the
// sum of axis x's factors at i_x = e (mod nc). FP64, in a fixed order. The
// row table's LDS serves as scratch (it is rebuilt after this).
template <int PREC>
__device__ __forceinline__ void prop_scales(const SweepArgs& a, float* smem, const Win& w,
                                            long long kc, int ns, int sw, int cols,
                                            PropScales* ps) {
  static_assert(kThreads == 256, "256 partial sums");
  const int D = a.g.ndim;
  const int nc = a.L.cpw;
  const int t = threadIdx.x;
  double* scr = reinterpret_cast<double*>(smem + a.L.row_off);
  double* A = scr;           // [16] strip masses by residue
  double* G = scr + 16;      // [16] axis x's factor sums by residue
  double* part = scr + 32;   // [256] partial row sums
  double* S = scr + 288;     // [16] row-factor masses by residue
  const float* tabL = smem + pick4(a.L.tab_off, D - 1);
  const int Wx = D > 1 ? pick4(w.W, D - 2) : 1;
  if (t < nc) {
    double sa = 0.0;
    for (int st = t; st < ns; st += nc)
      for (int j = 0; j < sw; ++j) sa += (double)tabL[st * sw + j];
    A[t] = sa;
    double sg = 0.0;
    if (D > 1) {
      const float* tx = smem + pick4(a.L.tab_off, D - 2);
      for (int i = t; i < Wx; i += nc) sg += (double)tx[i];
    } else {
      sg = t == 0 ? 1.0 : 0.0;  // one row, r = 0, of factor 1
    }
    G[t] = sg;
  }
  __syncthreads();
  // thread t: residue b = t mod nc, outer rows o = t / nc + k (256 / nc)
  // outer rows (window rows number below 2^31): 4-D walks (i0, i1) with a
  // carry instead of dividing
  const int outer = D > 1 ? (int)(w.R / Wx) : 1;
  const int b = t & (nc - 1), per = kThreads / nc;
  double sp = 0.0;
  const int W1 = D == 4 ? w.W[1] : 1;
  int o = t / nc;
  int i0 = o / W1, i1 = o - i0 * W1;
  const int s0 = per / W1, s1 = per - s0 * W1;  // the step per in (i0, i1)
  for (; o < outer; o += per) {
    double go = 1.0;
    if (D >= 3) go = (double)smem[a.L.tab_off[0] + i0];
    if (D == 4) go *= (double)smem[a.L.tab_off[1] + i1];
    sp += go * G[(int)(((unsigned)b - (unsigned)o * (unsigned)Wx) & (unsigned)(nc - 1))];
    i1 += s1;
    i0 += s0;
    if (i1 >= W1) {
      i1 -= W1;
      ++i0;
    }
  }
  part[t] = sp;
  __syncthreads();
  if (t < nc) {
    double sb = 0.0;
    for (int k = t; k < kThreads; k += nc) sb += part[k];
    S[t] = sb;
  }
  __syncthreads();
  const double cells = (double)w.R * (double)(ns * sw);
  double K = 4294967296.0 - 1048576.0 - cells;
  if (PREC == VUP_FP8E4M3) K *= 0.5;  // subnormal rounding can more than double tiny values
  // U[d] = sum of S[b] over b cols = d (mod nc); copy c holds
  // sum over a of A[a] U[(c - a) mod nc]
  double* U = part;  // the partials are consumed
  if (t < nc) {
    double u = 0.0;
    for (int bb = 0; bb < nc; ++bb)
      if (((bb * cols) & (nc - 1)) == t) u += S[bb];
    U[t] = u;
  }
  __syncthreads();
  if (t < nc) {
    double m = 0.0;
    for (int aa = 0; aa < nc; ++aa) m += A[aa] * U[(t - aa) & (nc - 1)];
    const double sc = m > 0.0 ? K / (prec_qfac<PREC>() * m) : 0.0;
    ps->scale[t] = sc;
    ps->unscale[t] = sc > 0.0 ? 1.0 / sc : 0.0;
    ps->scalef[t] = (float)sc;
  }
  if (t == 0) ps->mexp = win_scale_exp(a, smem);
  __syncthreads();
}

// Window row r of the cell form as mixed-radix digits over the slower axes
// (axis 0 slowest, axis D-2 the least significant digit). A thread starts at
// its first row with one division per axis and then steps by kThreads rows
// with carries, so the row table is built without dividing.
struct RowIt {
  int i[3];
};

__device__ __forceinline__ void rowit_init(RowIt& it, long long r, const Win& w, int D) {
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    it.i[d] = 0;
    if (d <= D - 2) {
      if (d > 0) {
        it.i[d] = (int)(r % w.W[d]);
        r /= w.W[d];
      } else {
        it.i[d] = (int)r;
      }
    }
  }
}

// digits of the step kThreads (uniform)
__device__ __forceinline__ RowIt rowit_step_digits(const Win& w, int D) {
  RowIt s;
  long long r = kThreads;
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    s.i[d] = 0;
    if (d <= D - 2) {
      if (d > 0) {
        s.i[d] = (int)(r % w.W[d]);
        r /= w.W[d];
      } else {
        s.i[d] = (int)r;
      }
    }
  }
  return s;
}

__device__ __forceinline__ void rowit_step(RowIt& it, const RowIt& s, const Win& w, int D) {
  int carry = 0;
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    if (d <= D - 2) {
      it.i[d] += s.i[d] + carry;
      carry = 0;
      if (d > 0 && it.i[d] >= w.W[d]) {  // i + step + carry < 2 W: one wrap at most
        it.i[d] -= w.W[d];
        carry = 1;
      }
    }
  }
}

// Row table of the cell form for rows [r0, r0 + rc): (go, map offset), with
// the row factor go the product of the slower axes' factors taken in FP64 and
// rounded once. Thread t holds the digits of row r0 + t and advances them by
// kThreads per row it builds (chunks are multiples of kThreads rows).
__device__ __forceinline__ void build_rows_prop(const SweepArgs& a, float* smem, const Win& w,
                                                int rc, RowIt& it, const RowIt& step) {
  const int D = a.g.ndim;
  float2* rt = reinterpret_cast<float2*>(smem + a.L.row_off);
  for (int r = threadIdx.x; r < rc; r += kThreads) {
    double go = 1.0;
    int off = 0;  // the padded bin map has fewer than 2^31 elements
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d <= D - 2) {
        go *= (double)smem[a.L.tab_off[d] + it.i[d]];
        off += (w.lo[d] + it.i[d]) * (int)a.g.rowstride[d];
      }
    }
    rt[r] = make_float2((float)go, __int_as_float(off));
    rowit_step(it, step, w, D);
  }
}

template <int SW, int PREC>
__device__ __forceinline__ void prop_rows(const SweepArgs& a, float* smem, int r0, int rc,
                                          int colbase, int ns, const PropScales* ps) {
  const int cols = ns < kThreads ? ns : kThreads;
  const int P0 = kThreads / cols;
  const int col = threadIdx.x % cols;
  const int ph = threadIdx.x / cols;
  if (ph >= P0) return;
  const float2* rt = reinterpret_cast<const float2*>(smem + a.L.row_off);
  const int cm = a.L.cpw - 1;     // copies - 1 (a power of two minus one)
  // byte address of (bin, copy): hist + (4 bin) << cshift + 4 copy
  const uint32_t cmul = 1u << a.L.cshift;
  const uint32_t hist = lds_addr(smem + a.L.hist_off);
  const float* tabL = smem + pick4(a.L.tab_off, a.g.ndim - 1);
  for (int s = col; s < ns; s += cols) {
    float gl[SW];
#pragma unroll
    for (int j = 0; j < SW; ++j) gl[j] = tabL[s * SW + j];
    const uint16_t* mbase = a.binmap + colbase + s * SW;
    struct Row {
      float2 e;
      float sc;  // scale of the strip-row's copy
      MapVec<SW> mv;
    };
    // the copy of strip s in window row r0 + r: (s + (r0 + r) cols) mod nc
    auto copy_of = [&](int r) {
      return (int)(((unsigned)(r0 + r) * (unsigned)cols + (unsigned)s) & (unsigned)cm);
    };
    auto load = [&](int r, Row& x) {
      x.e = rt[r];
      x.sc = ps->scalef[copy_of(r)];
      x.mv = load_map<SW>(mbase + (unsigned)__float_as_int(x.e.y));
    };
    auto accumulate = [&](int r, const Row& x) {
      // this strip-row's copy and its scale; the ordered dither's row part
      const uint32_t hb = hist + 4 * copy_of(r);
      const float sc = x.sc;
      const float ub = ((float)(r & 15) + 0.5f) * (1.0f / (16.0f * (float)SW));
      float gos = 0.0f, qs = 0.0f, gq = 0.0f;
      if constexpr (PREC == VUP_FP32) {
        gos = x.e.x * sc;
      } else {
        // E4M3 rounds 448 w: the row factor carries the 448
        qs = sc * (PREC == VUP_FP8E4M3 ? (1.0f / 448.0f) : 1.0f);
        gq = PREC == VUP_FP8E4M3 ? x.e.x * 448.0f : x.e.x;
      }
#pragma unroll
      for (int j = 0; j < SW; j += 2) {
        const float u0 = (float)j * (1.0f / (float)SW) + ub;
        const float u1 = (float)(j + 1) * (1.0f / (float)SW) + ub;
        float v0, v1;
        if constexpr (PREC == VUP_FP32) {
          v0 = fmaf(gos, gl[j], u0);
          v1 = fmaf(gos, gl[j + 1], u1);
        } else {
          float q0, q1;
          quantize2<PREC>(gq * gl[j], gq * gl[j + 1], q0, q1);
          v0 = fmaf(q0, qs, u0);
          v1 = fmaf(q1, qs, u1);
        }
        // codes j (low half) and j + 1 (high half) of one packed word
        const uint32_t pk = x.mv.v[j >> 1];
        vup_lds_u32* s0 = (vup_lds_u32*)(uintptr_t)mad_lo16(pk, cmul, hb);
        vup_lds_u32* s1 = (vup_lds_u32*)(uintptr_t)mad_hi16(pk, cmul, hb);
        __hip_atomic_fetch_add(s0, (uint32_t)v0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(s1, (uint32_t)v1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    };
    // rows two at a time in ping-pong buffers: one row's bin codes are in
    // flight while the other row is accumulated
    int r = ph;
    if (r >= rc) continue;
    Row ra, rb;
    load(r, ra);
    for (;;) {
      const int r2 = r + P0;
      if (r2 < rc) load(r2, rb);
      accumulate(r, ra);
      if (r2 >= rc) break;
      r = r2 + P0;
      if (r < rc) load(r, ra);
      accumulate(r2, rb);
      if (r >= rc) break;
    }
  }
}

// Unscale the interleaved histogram copies of component kc (bin b, copy c at
// word b nc + c), normalise by the sum over all slots (cells without a bin
// included) and add the weighted column into Pk. The reported normaliser is
// the mass of the densities: the tables' mass times 2^-*mexp.
__device__ __forceinline__ void finish_cells(const SweepArgs& a, const uint32_t* hist, int nc,
                                             const double* unscale, double* red, long long kc,
                                             const int* mexp, float* Pk, bool written) {
  const int B = a.B;
  auto slot = [&](int b) {
    double v = 0.0;
    const uint32_t* h = hist + (size_t)b * nc;
    if (nc >= 4) {
      for (int c = 0; c < nc; c += 4) {
        const uint4 q = *reinterpret_cast<const uint4*>(h + c);
        v += (double)q.x * unscale[c] + (double)q.y * unscale[c + 1] +
             (double)q.z * unscale[c + 2] + (double)q.w * unscale[c + 3];
      }
    } else {
      for (int c = 0; c < nc; ++c) v += (double)h[c] * unscale[c];
    }
    return v;
  };
  const double wk = (a.d.C > 1) ? a.d.weight[kc] : 1.0;
  if (B + 1 <= 2 * kThreads) {
    const int b0 = threadIdx.x, b1 = threadIdx.x + kThreads;
    const double v0 = b0 <= B ? slot(b0) : 0.0;
    const double v1 = b1 <= B ? slot(b1) : 0.0;
    const double Zc = block_sum(v0 + v1, red);
    if (a.Z && threadIdx.x == 0) a.Z[kc] = ldexp(Zc, -*mexp);
    const double f = wk / Zc;
    if (b0 < B) Pk[b0] = (float)((written ? (double)Pk[b0] : 0.0) + v0 * f);
    if (b1 < B) Pk[b1] = (float)((written ? (double)Pk[b1] : 0.0) + v1 * f);
    return;
  }
  double zpart = 0.0;
  for (int b = threadIdx.x; b <= B; b += kThreads) zpart += slot(b);
  const double Zc = block_sum(zpart, red);
  if (a.Z && threadIdx.x == 0) a.Z[kc] = ldexp(Zc, -*mexp);
  const double f = wk / Zc;
  for (int b = threadIdx.x; b < B; b += kThreads) {
    const double prev = written ? (double)Pk[b] : 0.0;
    Pk[b] = (float)(prev + slot(b) * f);
  }
}

// Run form: unscale the class histograms of component kc, normalise by the
// sum over all slots (cells without a bin included) and add the weighted
// column into Pk. Histogram copy i of class cl sits at hist + (cl * cpc + i) *
// stride.
__device__ __forceinline__ void finish_component(const SweepArgs& a, const uint32_t* hist, int ncls,
                                                 int cpc, const double* unscale, double* red,
                                                 long long kc, const int* mexp, float* Pk,
                                                 bool written) {
  const int B = a.B;
  const int stride = a.L.hist_stride;
  auto slot = [&](int b) {
    double v = 0.0;
    for (int cl = 0; cl < ncls; ++cl) {
      uint64_t cnt = 0;
      for (int cp = 0; cp < cpc; ++cp) cnt += hist[(cl * cpc + cp) * stride + b];
      v += (double)cnt * unscale[cl];
    }
    return v;
  };
  const double wk = (a.d.C > 1) ? a.d.weight[kc] : 1.0;
  if (B + 1 <= 2 * kThreads) {
    // at most two slots per thread: keep them in registers
    const int b0 = threadIdx.x, b1 = threadIdx.x + kThreads;
    const double v0 = b0 <= B ? slot(b0) : 0.0;
    const double v1 = b1 <= B ? slot(b1) : 0.0;
    const double Zc = block_sum(v0 + v1, red);
    if (a.Z && threadIdx.x == 0) a.Z[kc] = ldexp(Zc, -*mexp);
    const double f = wk / Zc;
    if (b0 < B) Pk[b0] = (float)((written ? (double)Pk[b0] : 0.0) + v0 * f);
    if (b1 < B) Pk[b1] = (float)((written ? (double)Pk[b1] : 0.0) + v1 * f);
    return;
  }
  double zpart = 0.0;
  for (int b = threadIdx.x; b <= B; b += kThreads) zpart += slot(b);
  const double Zc = block_sum(zpart, red);
  if (a.Z && threadIdx.x == 0) a.Z[kc] = ldexp(Zc, -*mexp);
  const double f = wk / Zc;
  for (int b = threadIdx.x; b < B; b += kThreads) {
    const double prev = written ? (double)Pk[b] : 0.0;
    Pk[b] = (float)(prev + slot(b) * f);
  }
}

// column of distribution k after all components: NaN for an invalid
// parameter, zeros when every window is empty; counted
__device__ __forceinline__ void finish_column(const SweepArgs& a, float* Pk, bool anybad,
                                              bool written) {
  if (anybad || !written)
    for (int b = threadIdx.x; b < a.B; b += kThreads) Pk[b] = anybad ? __builtin_nanf("") : 0.0f;
  if (threadIdx.x == 0) {
    if (anybad) atomicAdd(a.counters + kCntBadParam, 1ull);
    else if (!written) atomicAdd(a.counters + kCntEmpty, 1ull);
  }
}

// four waves per SIMD: the occupancy the cell form's LDS allows (about 40 KB
// per workgroup), so the kernel is held to 128 VGPRs
template <int PREC>
__global__ __launch_bounds__(kThreads, 4) void k_propagate(SweepArgs a) {
  extern __shared__ float smem[];
  if (PREC == VUP_FP32 && runs_chosen(a)) return;  // k_propagate_runs does the work
  const long long k = block_k(a);
  if (k >= a.d.K) return;
  const int D = a.g.ndim;
  const int nc = a.L.cpw;
  double* red = reinterpret_cast<double*>(smem + a.L.red_off);
  PropScales* ps = reinterpret_cast<PropScales*>(smem + a.L.red_off + 96);
  const uint32_t* hist = reinterpret_cast<const uint32_t*>(smem + a.L.hist_off);
  float* Pk = a.P + k * (long long)a.B;
  bool anybad = false;
  bool written = false;  // row k holds a partial mixture
  for (int c = 0; c < a.d.C; ++c) {
    const long long kc = k * a.d.C + c;
    const Win w = make_win(a, kc, reinterpret_cast<int*>(smem + a.L.red_off + 80));
    if (w.bad) {
      anybad = true;
      if (a.Z && threadIdx.x == 0) a.Z[kc] = __builtin_nan("");
      continue;
    }
    if (w.empty) {
      if (a.Z && threadIdx.x == 0) a.Z[kc] = 0.0;
      continue;
    }
    int loL, WL;
    last_axis(w, D, loL, WL);
    const int sw = choose_sw(loL, WL, w.R, kMaxSW);
    const int colbase = (loL / sw) * sw;
    const int ns = (loL + WL - 1) / sw - loL / sw + 1;
    __syncthreads();  // LDS reuse across components
    build_tables_exact(a, smem, w, kc, sw, colbase, ns);
    {
      uint4* h4 = reinterpret_cast<uint4*>(smem + a.L.hist_off);
      for (int i = threadIdx.x; i < a.L.hist_stride / 4; i += kThreads)
        h4[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    prop_scales<PREC>(a, smem, w, kc, ns, sw, ns < kThreads ? ns : kThreads, ps);
    const int rr = a.L.rrows;
    RowIt it;
    rowit_init(it, threadIdx.x, w, D);
    const RowIt step = rowit_step_digits(w, D);
    for (long long r0 = 0; r0 < w.R; r0 += rr) {
      const int rc = (int)((w.R - r0) < rr ? (w.R - r0) : rr);
      __syncthreads();
      build_rows_prop(a, smem, w, rc, it, step);
      __syncthreads();
      switch (sw) {
        case 4: prop_rows<4, PREC>(a, smem, (int)r0, rc, colbase, ns, ps); break;
        case 8: prop_rows<8, PREC>(a, smem, (int)r0, rc, colbase, ns, ps); break;
        default: prop_rows<16, PREC>(a, smem, (int)r0, rc, colbase, ns, ps); break;
      }
    }
    __syncthreads();
    finish_cells(a, hist, nc, ps->unscale, red, kc, &ps->mexp, Pk, written);
    written = true;
  }
  finish_column(a, Pk, anybad, written);
}

// ---------------------------------------------------------------------------
// Run form (FP32 densities). Along the fastest axis a row of the model matrix
// is a sequence of runs of equal bin, and the density is separable, so the
// mass of the window part [s, e) of a run is go * (G[e] - G[s]), with G the
// FP64 prefix sums of the fastest-axis factors over the window. One integer
// atomic then carries a whole run instead of one cell. The fixed point has
// three classes by row factor (as above) and no column classes: a class-r
// scale is K / (rowbound[r] * G[W]), since the runs of a row telescope to
// G[W]. The dither is per thread, u = (t + 1/2)/256.
// G covers the whole fastest axis (flat outside the window), so no run needs
// clipping. A 16-lane group walks one row: lane l takes runs l, l+16, ... of
// the row's window segment, so record loads are coalesced. A run ends where
// the next begins; lane l takes that record from lane l+1 (a DPP rotate
// within the 16-lane row; lane 15 from lane 0's record of the next step).
// The four groups of a wave walk rows a quarter of the row chunk apart, so
// their atomics rarely meet in a bank.
// ---------------------------------------------------------------------------
struct RunRow {
  double rs;  // row factor x class scale
  int ra;     // first run of the row's window segment (index into the run records)
  uint32_t meta;  // runs in the segment | byte offset of the class histogram << 16
};

struct RunScales {
  double srow[3];
  double unscale[3];
  int mexp;  // win_scale_exp of the component
};

constexpr int kRunGroup = 16;  // lanes per row: one DPP row
// the same for the adjoint's run form (32-byte rows): about 30 KB of LDS per
// workgroup at 1024-cell rows, five workgroups per CU, matched by holding the
// 2-D kernel to 96 VGPRs (five waves per SIMD)
constexpr int kBwdRowChunk = 256;

// G[c] = sum of the fastest-axis factors of the window columns below c, FP64,
// for every column c = 0 .. n (0 up to loL, the window total from hiL + 1 on).
// Thread t sums a contiguous slice of the window; slice totals are scanned.
__device__ __forceinline__ void build_prefix_runs(const SweepArgs& a, float* smem, long long kc,
                                                  int loL, int WL, double off, double* red) {
  const int D = a.g.ndim;
  const int L = D - 1;
  const int nL = pick4(a.g.n, L);
  double* G = reinterpret_cast<double*>(smem + a.L.g_off);
  const double mu = a.d.mu[kc * D + L], rsig = 1.0 / a.d.sigma[kc * D + L];
  const int per = (WL + kThreads - 1) / kThreads;
  const int j0 = min((int)threadIdx.x * per, WL);
  const int j1 = min(j0 + per, WL);
  double* Gw = G + loL;  // Gw[j + 1] = sum over window columns loL .. loL + j
  double sum = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double x = cell_centre(pick4(a.g.lo, L), pick4(a.g.hi, L), nL, loL + j);
    const double g = (double)gauss_factor_r(x, mu, rsig, off);
    Gw[j + 1] = g;
    sum += g;
  }
  // inclusive scan of the slice sums within the wave, then across waves
  const int lane = threadIdx.x & 63;
  const double incl = wave_scan(sum);
  if (lane == 63) red[threadIdx.x >> 6] = incl;
  __syncthreads();
  double run = incl - sum;
  for (int wv = 0; wv < (int)(threadIdx.x >> 6); ++wv) run += red[wv];
  for (int j = j0; j < j1; ++j) {
    run += Gw[j + 1];
    Gw[j + 1] = run;
  }
  const double total = red[0] + red[1] + red[2] + red[3];
  static_assert(kWaves == 4, "scan of four waves");
  for (int c = threadIdx.x; c <= loL; c += kThreads) G[c] = 0.0;
  for (int c = loL + WL + 1 + threadIdx.x; c <= nL; c += kThreads) G[c] = total;
  __syncthreads();
}

// Row table of the run form for rows [r0, r0 + rc) of the window.
__device__ __forceinline__ void build_rows_runs(const SweepArgs& a, float* smem, const Win& w,
                                                long long r0, int rc, const RunScales* ps,
                                                int loL, int hiL) {
  const int D = a.g.ndim;
  RunRow* rt = reinterpret_cast<RunRow*>(smem + a.L.row_off);
  const int hstrideb = a.L.hist_stride * 4;
  for (int r = threadIdx.x; r < rc; r += kThreads) {
    int t = (int)r0 + r;  // window rows and grid rows number below 2^31
    float go = 1.0f;
    int gr = 0;  // grid row (flat index over the slower axes)
    int mul = 1;
#pragma unroll
    for (int d = 2; d >= 0; --d) {
      if (d <= D - 2) {
        // axis 0 is the slowest: what is left of t is its index
        const int i = d == 0 ? t : t % w.W[d];
        if (d > 0) t /= w.W[d];
        go *= smem[a.L.tab_off[d] + i];
        gr += (w.lo[d] + i) * mul;
        mul *= a.g.n[d];
      }
    }
    const int off = gr * a.g.pitch;
    const int base = a.rowptr[gr];
    const int ra = base + (int)a.runidx[off + loL];
    const int rb = base + (int)a.runidx[off + hiL] + 1;
    const int cls = mag_class(go);
    RunRow e;
    e.rs = (double)go * ps->srow[cls];
    e.ra = ra;
    e.meta = (uint32_t)(rb - ra) | ((uint32_t)(cls * hstrideb) << 16);
    rt[r] = e;
  }
}

// FP64 load from an LDS byte address (lds_addr of the prefix sums plus
// 8 column, formed by mad_lo16 from a run record in one VALU op)
typedef const __attribute__((address_space(3))) double lds_f64;
__device__ __forceinline__ double lds_load_f64(uint32_t byte_addr) {
  return *(lds_f64*)(size_t)byte_addr;
}

// value of lane (l + 1) mod 16 within each 16-lane row (DPP row rotate)
__device__ __forceinline__ uint32_t next_lane(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x12F /* row_ror:15 */, 0xF, 0xF, false);
}

__device__ __forceinline__ void prop_runs(const SweepArgs& a, float* smem, int rc) {
  const int l = threadIdx.x & (kRunGroup - 1);
  const int gi = (threadIdx.x >> 4) & 3;  // group within the wave
  const int wv = threadIdx.x >> 6;
  const RunRow* rt = reinterpret_cast<const RunRow*>(smem + a.L.row_off);
  char* hbase = reinterpret_cast<char*>(smem + a.L.hist_off);
  const uint32_t gaddr = lds_addr(smem + a.L.g_off);  // FP64 prefix sums G
  const double u = ((double)threadIdx.x + 0.5) * (1.0 / kThreads);
  const int bl = (rc + 3) >> 2;
  const int rend = min((gi + 1) * bl, rc);
  for (int r = gi * bl + wv; r < rend; r += kWaves) {
    const RunRow row = rt[r];
    const int cnt = (int)(row.meta & 0xFFFFu);
    char* lh = hbase + (row.meta >> 16);
    const uint32_t* rp = a.runs + row.ra;
    // One run: this lane's record c; the run after it starts at lane l+1's
    // record (dc = c rotated down one lane) or, for lane 15, at lane 0's
    // record of the next step (dn). G is flat outside the window, so the
    // part of a run inside the window is G[next start] - G[start] without
    // clamping. `left` = runs of the row from this lane's current one on.
    auto step = [&](uint32_t c, uint32_t dc, uint32_t dn, int left) {
      const uint32_t nx = (l == kRunGroup - 1) ? dn : dc;
      if (left > 0) {
        const double v =
            fma(lds_load_f64(mad_lo16_k<8>(nx, gaddr)) - lds_load_f64(mad_lo16_k<8>(c, gaddr)),
                row.rs, u);
        uint32_t* slot = reinterpret_cast<uint32_t*>(lh + (c >> 16));
        __hip_atomic_fetch_add(slot, (uint32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    };
    // four runs per lane per pass: the four record loads are in flight
    // together (a step no lane of the wave needs is branched over). Records
    // past the segment (at most 79) are read but unused; the run buffer is
    // padded for them.
    uint32_t cur = rp[l];
    uint32_t dcur = next_lane(cur);
    for (int q0 = l; q0 - l < cnt; q0 += 4 * kRunGroup) {
      const uint32_t* p = rp + q0;
      const uint32_t r1 = p[kRunGroup];
      const uint32_t r2 = p[2 * kRunGroup];
      const uint32_t r3 = p[3 * kRunGroup];
      const uint32_t r4 = p[4 * kRunGroup];
      const uint32_t d1 = next_lane(r1), d2 = next_lane(r2);
      const uint32_t d3 = next_lane(r3), d4 = next_lane(r4);
      const int left = cnt - q0;
      step(cur, dcur, d1, left);
      step(r1, d1, d2, left - kRunGroup);
      step(r2, d2, d3, left - 2 * kRunGroup);
      step(r3, d3, d4, left - 3 * kRunGroup);
      cur = r4;
      dcur = d4;
    }
  }
}

// RR: rows per row-table pass (the layout's rrows). Seven waves per SIMD: at
// eight the 64-VGPR budget spilled a few per-thread addresses of the finish,
// and their scratch writes doubled the kernel's HBM write traffic (138 MB per
// launch at grid1024 against the 67 MB of P) for no gain in time
template <int RR>
__global__ __launch_bounds__(kThreads, 7) void k_propagate_runs(SweepArgs a) {
  extern __shared__ float smem[];
  if (!runs_chosen(a)) return;  // k_propagate does the work
  const long long k = block_k(a);
  if (k >= a.d.K) return;
  const int D = a.g.ndim;
  double* red = reinterpret_cast<double*>(smem + a.L.red_off);
  RunScales* ps = reinterpret_cast<RunScales*>(red + 16);
  const uint32_t* hist = reinterpret_cast<const uint32_t*>(smem + a.L.hist_off);
  float* Pk = a.P + k * (long long)a.B;
  bool anybad = false;
  bool written = false;
  for (int c = 0; c < a.d.C; ++c) {
    const long long kc = k * a.d.C + c;
    const Win w = make_win(a, kc, reinterpret_cast<int*>(smem + a.L.red_off + 80));
    if (w.bad) {
      anybad = true;
      if (a.Z && threadIdx.x == 0) a.Z[kc] = __builtin_nan("");
      continue;
    }
    if (w.empty) {
      if (a.Z && threadIdx.x == 0) a.Z[kc] = 0.0;
      continue;
    }
    int loL, WL;
    last_axis(w, D, loL, WL);
    __syncthreads();  // LDS reuse across components
    // factor tables of the slower axes
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d + 1 < D) {
        float* tab = smem + a.L.tab_off[d];
        const double mu = a.d.mu[kc * D + d], rsig = 1.0 / a.d.sigma[kc * D + d];
        const double off = scale_log(win_m(a, smem, d));
        for (int i = threadIdx.x; i < w.W[d]; i += kThreads)
          tab[i] = gauss_factor_r(cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], w.lo[d] + i), mu,
                                  rsig, off);
      }
    }
    for (int i = threadIdx.x; i < 3 * a.L.hist_stride; i += kThreads) smem[a.L.hist_off + i] = 0.0f;
    build_prefix_runs(a, smem, kc, loL, WL, scale_log(win_m(a, smem, D - 1)), red);
    const double Zrows = row_mass(a, smem, w, red);
    if (threadIdx.x == 0) {
      const double colmass = reinterpret_cast<const double*>(smem + a.L.g_off)[loL + WL];
      const double R = (double)w.R;
      const double K = 4294967296.0 - 1048576.0 - R * (double)WL;
      const double rowbound[3] = {Zrows, fmin(Zrows, R * (double)kClassT1),
                                  fmin(Zrows, R * (double)kClassT2)};
      for (int r = 0; r < 3; ++r) {
        ps->srow[r] = K / (prec_qfac<VUP_FP32>() * rowbound[r] * colmass);
        ps->unscale[r] = 1.0 / ps->srow[r];
      }
      ps->mexp = win_scale_exp(a, smem);
    }
    for (long long r0 = 0; r0 < w.R; r0 += RR) {
      const int rc = (int)((w.R - r0) < RR ? (w.R - r0) : RR);
      __syncthreads();
      build_rows_runs(a, smem, w, r0, rc, ps, loL, loL + WL - 1);
      __syncthreads();
      prop_runs(a, smem, rc);
    }
    __syncthreads();
    finish_component(a, hist, 3, 1, ps->unscale, red, kc, &ps->mexp, Pk, written);
    written = true;
  }
  finish_column(a, Pk, anybad, written);
}

// ===========================================================================
// exact-f moments: shifted FP32 strip sums, FP64 accumulation
// ===========================================================================
// A thread walks the rows of its strip two at a time (ping-pong buffers): the
// loads of one row are in flight while the other row is summed.
template <int SW>
struct MomRow {
  float4 f[SW / 4];
  float go;
};

template <int SW>
__device__ __forceinline__ void mom_load(const SweepArgs& a, const float2* rt, const float* fbase,
                                         int r, MomRow<SW>& m) {
  const float2 e = rt[r];
  m.go = e.x;
  const float4* p = reinterpret_cast<const float4*>(fbase + (unsigned)__float_as_int(e.y));
#pragma unroll
  for (int q = 0; q < SW / 4; ++q) m.f[q] = p[q];
}

// One row of a thread's 8-cell strip. The FP32 model copy is anchored: the
// strip's first cell holds f_0 and the others d_j = f_j - f_0. Each cell's
// shifted value v_j = f_j - shift = d_j + (f_0 - shift) is formed before it is
// weighted, so the sums hold only terms of the size of f - shift: expanding
// (d_j + delta)^2 instead would add terms of the size of d_j and delta that
// cancel, and lose their FP32 rounding error against the variance whenever the
// anchor's value lies far from the window's (a strip that meets the window in
// a few cells of a steep, coarsely sampled axis).
template <int SW>
__device__ __forceinline__ void mom_sum(const MomRow<SW>& m, const float* gl, float shift,
                                        float& B1, float& B2) {
  static_assert(SW == 8, "strips of eight cells, one anchor each");
  const float dl = m.f[0].x - shift;
  float a1 = 0.0f, a2 = 0.0f;
#pragma unroll
  for (int q = 0; q < SW / 4; ++q) {
    const float fj[4] = {m.f[q].x, m.f[q].y, m.f[q].z, m.f[q].w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float v = (q == 0 && e == 0) ? dl : fj[e] + dl;
      const float t = gl[4 * q + e] * v;
      a1 += t;
      a2 = fmaf(t, v, a2);
    }
  }
  B1 = fmaf(m.go, a1, B1);
  B2 = fmaf(m.go, a2, B2);
}

template <int SW>
__device__ __forceinline__ void mom_rows(const SweepArgs& a, const float* smem, int rc,
                                         int colbase, int ns, float shift, double& A1,
                                         double& A2) {
  const int cols = ns < kThreads ? ns : kThreads;
  const int P0 = kThreads / cols;
  const int col = threadIdx.x % cols;
  const int ph = threadIdx.x / cols;
  if (ph >= P0) return;
  const float2* rt = reinterpret_cast<const float2*>(smem + a.L.row_off);
  const float* tabL = smem + pick4(a.L.tab_off, a.g.ndim - 1);
  for (int s = col; s < ns; s += cols) {
    float gl[SW];
#pragma unroll
    for (int j = 0; j < SW; ++j) gl[j] = tabL[s * SW + j];
    const float* fbase = a.f32 + colbase + s * SW;
    int r = ph;
    if (r >= rc) continue;
    MomRow<SW> ma, mb;
    mom_load<SW>(a, rt, fbase, r, ma);
    // row sums times the row factor gather in FP32 over at most eight rows,
    // then in FP64
    float B1 = 0.0f, B2 = 0.0f;
    int pairs = 0;
    for (;;) {
      const int rb = r + P0;
      if (rb < rc) mom_load<SW>(a, rt, fbase, rb, mb);
      mom_sum<SW>(ma, gl, shift, B1, B2);
      if (rb >= rc) break;
      r = rb + P0;
      if (r < rc) mom_load<SW>(a, rt, fbase, r, ma);
      mom_sum<SW>(mb, gl, shift, B1, B2);
      if (r >= rc) break;
      if (++pairs == 4) {
        A1 += (double)B1;
        A2 += (double)B2;
        B1 = B2 = 0.0f;
        pairs = 0;
      }
    }
    A1 += (double)B1;
    A2 += (double)B2;
  }
}

__global__ __launch_bounds__(kThreads) void k_moments(SweepArgs a) {
  extern __shared__ float smem[];
  const long long k = block_k(a);
  if (k >= a.d.K) return;
  const int D = a.g.ndim;
  double* red = reinterpret_cast<double*>(smem + a.L.red_off);
  double Ec[VUP_MAX_COMP], Vc[VUP_MAX_COMP], pcs[VUP_MAX_COMP];
  bool used[VUP_MAX_COMP];
  bool anybad = false;
  for (int c = 0; c < a.d.C; ++c) {
    const long long kc = k * a.d.C + c;
    const Win w = make_win(a, kc, reinterpret_cast<int*>(smem + a.L.red_off + 80));
    used[c] = false;
    pcs[c] = (a.d.C > 1) ? a.d.weight[kc] : 1.0;
    if (w.bad) {
      anybad = true;
      continue;
    }
    if (w.empty) continue;
    used[c] = true;
    int loL, WL;
    last_axis(w, D, loL, WL);
    const int sw = 8;  // the anchored model copy has one anchor per 8 columns
    const int colbase = (loL / sw) * sw;
    const int ns = (loL + WL - 1) / sw - loL / sw + 1;
    // shift: model value at the window's centre cell (anchor plus offset)
    const int ccol = loL + WL / 2;
    long long cidx = ccol;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (d + 1 < D) cidx += (long long)(w.lo[d] + w.W[d] / 2) * a.g.rowstride[d];
    const long long aidx = cidx - (ccol & 7);
    const float shift = (ccol & 7) ? a.f32[aidx] + a.f32[cidx] : a.f32[aidx];
    __syncthreads();
    build_tables(a, smem, w, kc, sw, colbase, ns);
    double A1 = 0.0, A2 = 0.0;
    // row tables with the incremental digits (no division per row); chunks
    // of kRowChunk rows, a multiple of the workgroup size
    static_assert(kRowChunk % kThreads == 0, "row chunks of whole workgroup steps");
    RowIt it;
    rowit_init(it, threadIdx.x, w, D);
    const RowIt step = rowit_step_digits(w, D);
    for (long long r0 = 0; r0 < w.R; r0 += kRowChunk) {
      const int rc = (int)((w.R - r0) < kRowChunk ? (w.R - r0) : kRowChunk);
      __syncthreads();
      build_rows_prop(a, smem, w, rc, it, step);
      __syncthreads();
      mom_rows<8>(a, smem, rc, colbase, ns, shift, A1, A2);
    }
    // normaliser: product of the per-axis factor sums (separable density)
    double Z = 1.0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      if (d < D) {
        double zp = 0.0;
        const int cnt = (d + 1 < D) ? w.W[d] : ns * sw;
        for (int i = threadIdx.x; i < cnt; i += kThreads) zp += (double)smem[a.L.tab_off[d] + i];
        Z *= block_sum(zp, red);
      }
    }
    const double s1 = block_sum(A1, red) / Z;
    const double s2 = block_sum(A2, red) / Z;
    Ec[c] = (double)shift + s1;
    // a one-cell window is a point mass: variance 0 exactly (the anchored
    // sums would leave a rounding residue of the cell's offset squared)
    Vc[c] = (w.R == 1 && WL == 1) ? 0.0 : s2 - s1 * s1;
  }
  if (threadIdx.x != 0) return;
  double E = 0.0, wsum = 0.0;
  for (int c = 0; c < a.d.C; ++c)
    if (used[c]) {
      E += pcs[c] * Ec[c];
      wsum += pcs[c];
    }
  double V = 0.0;
  for (int c = 0; c < a.d.C; ++c)
    if (used[c]) V += pcs[c] * (Vc[c] + (Ec[c] - E) * (Ec[c] - E));
  const bool nan = anybad || wsum == 0.0;
  a.mean[k] = nan ? __builtin_nan("") : E;
  a.var[k] = nan ? __builtin_nan("") : V;
  if (a.delta2) {
    double d2 = __builtin_nan("");
    if (!nan && a.has_model && a.d.C == 1) {
      double x[4];
      for (int d = 0; d < D; ++d) x[d] = a.d.mu[k * D + d];
      const double fm = model_at(a.model.kind, D, a.model.theta, x);
      d2 = 0.5 * (V + (E - fm) * (E - fm));
    }
    a.delta2[k] = d2;
  }
}

// ===========================================================================
// adjoint sweep for the IPSA sensitivities
// ===========================================================================
// per-thread adjoint accumulators: sum w v, and sum w v t_d, sum w v t_d^2 for
// the fastest axis (L) and the slower axes (o[d], d < L)
template <int NO>  // number of slower axes
struct BwdAcc {
  double a0, l1, l2;
  double o1[NO > 0 ? NO : 1], o2[NO > 0 ? NO : 1];
};

template <int SW, int NO>
__device__ __forceinline__ void bwd_rows(const SweepArgs& a, const float* smem, int rc,
                                         int colbase, int ns, double muL, double sgL,
                                         BwdAcc<NO>& acc) {
  const int D = a.g.ndim;
  const int L = D - 1;
  const int cols = ns < kThreads ? ns : kThreads;
  const int P0 = kThreads / cols;
  const int col = threadIdx.x % cols;
  const int ph = threadIdx.x / cols;
  if (ph >= P0) return;
  const float2* rt = reinterpret_cast<const float2*>(smem + a.L.row_off);
  const float4* tt = reinterpret_cast<const float4*>(smem + a.L.trow_off);
  const char* vt = reinterpret_cast<const char*>(smem + a.L.hist_off);
  const float* tabL = smem + pick4(a.L.tab_off, L);
  for (int s = col; s < ns; s += cols) {
    float gl[SW], g1[SW], g2[SW];
    const float* tab1 = smem + a.L.g_off;
    const float* tab2 = tab1 + pick4(a.L.cap, L);
#pragma unroll
    for (int j = 0; j < SW; ++j) {
      gl[j] = tabL[s * SW + j];
      g1[j] = tab1[s * SW + j];
      g2[j] = tab2[s * SW + j];
    }
    const uint16_t* mbase = a.binmap + colbase + s * SW;
    // one row: the sums of the strip's cells weighted by the bin's v, then the
    // row factor (and the slower axes' t) applied in FP64
    auto row_sum = [&](int r, const MapVec<SW>& mv) {
      float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
#pragma unroll
      for (int j = 0; j < SW; ++j) {
        const float vb = *reinterpret_cast<const float*>(vt + map_at<SW>(mv, j));
        a0 = fmaf(gl[j], vb, a0);
        a1 = fmaf(g1[j], vb, a1);
        a2 = fmaf(g2[j], vb, a2);
      }
      const double go = (double)rt[r].x;
      const double c0 = go * (double)a0;
      acc.a0 += c0;
      acc.l1 += go * (double)a1;
      acc.l2 += go * (double)a2;
      if constexpr (NO > 0) {
        const float4 tv = tt[r];
        const float tr[3] = {tv.x, tv.y, tv.z};
#pragma unroll
        for (int d = 0; d < NO; ++d) {
          const double td = (double)tr[d];
          acc.o1[d] += c0 * td;
          acc.o2[d] += c0 * td * td;
        }
      }
    };
    // rows two at a time in ping-pong buffers: one row's bin codes are in
    // flight while the other row is summed
    int r = ph;
    if (r >= rc) continue;
    MapVec<SW> ma = load_map<SW>(mbase + (unsigned)__float_as_int(rt[r].y)), mb;
    for (;;) {
      const int rb = r + P0;
      if (rb < rc) mb = load_map<SW>(mbase + (unsigned)__float_as_int(rt[rb].y));
      row_sum(r, ma);
      if (rb >= rc) break;
      r = rb + P0;
      if (r < rc) ma = load_map<SW>(mbase + (unsigned)__float_as_int(rt[r].y));
      row_sum(rb, mb);
      if (r >= rc) break;
    }
  }
}

// LDS table of the adjoint weights of distribution k's bins (the table is FP32,
// so ln P_b is taken in FP32; P_b itself is FP32):
// S = sum_b P_b (c_b - E); v_b = gv((c_b - E)^2 - 2 c_b S) - ge(ln P_b + 1);
// vref = sum_b P_b v_b is subtracted from the table (covariances are shift
// invariant) and returned, to be added back for the weight gradient. Cells
// without a bin do not enter Var or H: their slot B holds -vref (v = 0).
__device__ __forceinline__ double build_vtable(const SweepArgs& a, float* vt, long long k,
                                               double* red) {
  const int B = a.B;
  const float* Pk = a.Pin + k * (long long)B;
  const double gv = a.g_var ? a.g_var[k] : 0.0;
  const double ge = a.g_ent ? a.g_ent[k] : 0.0;
  const double E = a.mean_hist[k];
  double sp = 0.0;
  for (int b = threadIdx.x; b < B; b += kThreads) {
    const double cb = 0.5 * (a.edges[b] + a.edges[b + 1]);
    sp += (double)Pk[b] * (cb - E);
  }
  const double S = block_sum(sp, red);
  double vp = 0.0;
  for (int b = threadIdx.x; b < B; b += kThreads) {
    const double cb = 0.5 * (a.edges[b] + a.edges[b + 1]);
    const double pb = (double)Pk[b];
    double v = gv * ((cb - E) * (cb - E) - 2.0 * cb * S);
    if (pb > 0.0) v -= ge * ((double)logf((float)pb) + 1.0);
    vp += pb * v;
  }
  const double vref = block_sum(vp, red);
  for (int b = threadIdx.x; b <= B; b += kThreads) {
    double v = 0.0;
    if (b < B) {
      const double cb = 0.5 * (a.edges[b] + a.edges[b + 1]);
      const double pb = (double)Pk[b];
      v = gv * ((cb - E) * (cb - E) - 2.0 * cb * S);
      if (pb > 0.0) v -= ge * ((double)logf((float)pb) + 1.0);
    }
    vt[b] = (float)(v - vref);
  }
  return vref;
}

// Gradients of component kc from the normalised sweep sums: A0 = E[v],
// l1, l2 = E[v t], E[v t^2] along the fastest axis, t1[d], t2[d] the same for
// the slower axes, m1[d], m2[d] = E[t], E[t^2] per axis (covariances, since
// the weight table is centred), scaled by the mixture weight pc. An axis
// whose window is one cell has a constant t, so its covariances, and the
// derivatives, are exactly 0 (the component's output does not depend on its
// mean or deviation along that axis within the window): written as 0 rather
// than as the rounding residue of two equal sums times t / sigma, which for a
// pdf much narrower than a cell is large.
__device__ __forceinline__ void write_grads(const SweepArgs& a, const Win& w, long long kc,
                                            double pc, double A0, double l1, double l2,
                                            const double* t1, const double* t2,
                                            const double* m1, const double* m2, double vref) {
  if (threadIdx.x != 0) return;
  const int D = a.g.ndim;
  const int L = D - 1;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (d < D) {
      const double sg = a.d.sigma[kc * D + d];
      const double s1 = (d == L) ? l1 : t1[d < 3 ? d : 0];
      const double s2 = (d == L) ? l2 : t2[d < 3 ? d : 0];
      const bool one = w.W[d] == 1;
      a.g_mu[kc * D + d] = one ? 0.0 : pc * (s1 - m1[d] * A0) / sg;
      a.g_sigma[kc * D + d] = one ? 0.0 : pc * (s2 - m2[d] * A0) / sg;
    }
  }
  if (a.g_weight) a.g_weight[kc] = A0 + vref;
}

// NO = ndim - 1 slower axes (a compile-time count keeps the accumulators of
// absent axes out of the registers)
template <int NO>
__global__ __launch_bounds__(kThreads) void k_backward(SweepArgs a) {
  extern __shared__ float smem[];
  if (runs_chosen(a)) return;  // k_backward_runs does the work
  const long long k = block_k(a);
  if (k >= a.d.K) return;
  const int D = a.g.ndim;
  double* red = reinterpret_cast<double*>(smem + a.L.red_off);
  float* vt = smem + a.L.hist_off;
  const double vref = build_vtable(a, vt, k, red);
  for (int c = 0; c < a.d.C; ++c) {
    const long long kc = k * a.d.C + c;
    const Win w = make_win(a, kc, reinterpret_cast<int*>(smem + a.L.red_off + 80));
    const double pc = (a.d.C > 1) ? a.d.weight[kc] : 1.0;
    if (w.bad || w.empty) {
      if (threadIdx.x == 0) {
        const double val = w.bad ? __builtin_nan("") : 0.0;
        for (int d = 0; d < D; ++d) {
          a.g_mu[kc * D + d] = val;
          a.g_sigma[kc * D + d] = val;
        }
        if (a.g_weight) a.g_weight[kc] = val;
      }
      continue;
    }
    const int L = D - 1;
    int loL, WL;
    last_axis(w, D, loL, WL);
    const int sw = choose_sw(loL, WL, w.R, 8);
    const int colbase = (loL / sw) * sw;
    const int ns = (loL + WL - 1) / sw - loL / sw + 1;
    __syncthreads();
    build_tables(a, smem, w, kc, sw, colbase, ns);
    {
      float* tab1 = smem + a.L.g_off;
      float* tab2 = tab1 + pick4(a.L.cap, L);
      const double muL = a.d.mu[kc * D + L], rsg = 1.0 / a.d.sigma[kc * D + L];
      for (int jj = threadIdx.x; jj < ns * sw; jj += kThreads) {
        const double t = (cell_centre(pick4(a.g.lo, L), pick4(a.g.hi, L), pick4(a.g.n, L), colbase + jj) - muL) * rsg;
        const double g = (double)smem[pick4(a.L.tab_off, L) + jj];
        tab1[jj] = (float)(g * t);
        tab2[jj] = (float)(g * t * t);
      }
    }
    BwdAcc<NO> acc;
    acc.a0 = acc.l1 = acc.l2 = 0.0;
#pragma unroll
    for (int i = 0; i < (NO > 0 ? NO : 1); ++i) acc.o1[i] = acc.o2[i] = 0.0;
    const double muL = a.d.mu[kc * D + L];
    const double sgL = a.d.sigma[kc * D + L];
    for (long long r0 = 0; r0 < w.R; r0 += kRowChunk) {
      const int rc = (int)((w.R - r0) < kRowChunk ? (w.R - r0) : kRowChunk);
      __syncthreads();
      build_rows(a, smem, w, r0, rc, kc, true);
      __syncthreads();
      switch (sw) {
        case 4: bwd_rows<4, NO>(a, smem, rc, colbase, ns, muL, sgL, acc); break;
        default: bwd_rows<8, NO>(a, smem, rc, colbase, ns, muL, sgL, acc); break;
      }
    }
    // per-axis normalisers and score means from the factor tables (FP64)
    double Z = 1.0, m1[4], m2[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      m1[d] = m2[d] = 0.0;
      if (d < D) {
        const int cnt = (d + 1 < D) ? w.W[d] : ns * sw;
        const int first = (d + 1 < D) ? w.lo[d] : colbase;
        const double mu = a.d.mu[kc * D + d], sg = a.d.sigma[kc * D + d];
        double z0 = 0.0, z1 = 0.0, z2 = 0.0;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
          const double g = (double)smem[a.L.tab_off[d] + i];
          const double t = (cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], first + i) - mu) / sg;
          z0 += g;
          z1 += g * t;
          z2 += g * t * t;
        }
        const double Zd = block_sum(z0, red);
        m1[d] = block_sum(z1, red) / Zd;
        m2[d] = block_sum(z2, red) / Zd;
        Z *= Zd;
      }
    }
    const double A0 = block_sum(acc.a0, red) / Z;
    double t1[4], t2[4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      t1[d] = d < NO ? block_sum(acc.o1[d < NO ? d : 0], red) / Z : 0.0;
      t2[d] = d < NO ? block_sum(acc.o2[d < NO ? d : 0], red) / Z : 0.0;
    }
    t1[3] = 0.0;
    t2[3] = 0.0;
    const double l1 = block_sum(acc.l1, red) / Z;
    const double l2 = block_sum(acc.l2, red) / Z;
    write_grads(a, w, kc, pc, A0, l1, l2, t1, t2, m1, m2, vref);
  }
}

// ---------------------------------------------------------------------------
// Adjoint sweep, run form. With the run form of the model matrix and the
// separable density, the three fastest-axis sums the adjoint needs over a run
// [s, e) are differences of prefix sums over the axis: G0 of g, G1 of g t and
// G2 of g t^2 (t = (x - mu)/sigma), summed in FP64 and held in LDS as FP32
// (flat outside the window) at offset 0, one 16-byte entry per column. A run
// costs two 16-byte LDS reads, the bin's weight and three FMAs; there are no
// atomics: each lane keeps its own sums, applied per row with the row factor
// (and the slower axes' t). Rows, lanes and the DPP hand-over of run ends are
// as in the run-form propagation.
// ---------------------------------------------------------------------------
struct BwdRunRow {
  float go;    // row factor
  float t[3];  // standardised coordinates of the slower axes
  int ra;      // first run of the row's window segment
  int cnt;     // runs in the segment
  int pad[2];
};

typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(3))) f32x4v lds_f4;
__device__ __forceinline__ f32x4v lds_load_f4(uint32_t byte_addr) {
  return *(lds_f4*)(size_t)byte_addr;
}

// G3[c] = (G0, G1, G2, -) for c = 0 .. n (sums over the window columns below
// c); the FP64 window totals go to tot[0..2].
__device__ __forceinline__ void build_prefix_bwd(const SweepArgs& a, float* smem, long long kc,
                                                 int loL, int WL, double off, double* red,
                                                 double* tot) {
  const int D = a.g.ndim;
  const int L = D - 1;
  const int nL = pick4(a.g.n, L);
  const double lo = pick4(a.g.lo, L), hi = pick4(a.g.hi, L);
  float4* G3 = reinterpret_cast<float4*>(smem);
  const double mu = a.d.mu[kc * D + L], rsig = 1.0 / a.d.sigma[kc * D + L];
  const int per = (WL + kThreads - 1) / kThreads;
  const int j0 = min((int)threadIdx.x * per, WL);
  const int j1 = min(j0 + per, WL);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double t = (cell_centre(lo, hi, nL, loL + j) - mu) * rsig;
    const float gf = gauss_factor_r(cell_centre(lo, hi, nL, loL + j), mu, rsig, off);
    const double g = (double)gf;
    s0 += g;
    s1 += g * t;
    s2 += g * t * t;
    G3[loL + j + 1].w = gf;  // the factor, until the sums overwrite the entry
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double i0 = wave_scan(s0), i1 = wave_scan(s1), i2 = wave_scan(s2);
  if (lane == 63) {
    red[wv] = i0;
    red[4 + wv] = i1;
    red[8 + wv] = i2;
  }
  __syncthreads();
  double r0 = i0 - s0, r1 = i1 - s1, r2 = i2 - s2;
  for (int w = 0; w < wv; ++w) {
    r0 += red[w];
    r1 += red[4 + w];
    r2 += red[8 + w];
  }
  for (int j = j0; j < j1; ++j) {
    const double t = (cell_centre(lo, hi, nL, loL + j) - mu) * rsig;
    const double g = (double)G3[loL + j + 1].w;
    r0 += g;
    r1 += g * t;
    r2 += g * t * t;
    G3[loL + j + 1] = make_float4((float)r0, (float)r1, (float)r2, 0.0f);
  }
  const double T0 = (red[0] + red[1]) + (red[2] + red[3]);
  const double T1 = (red[4] + red[5]) + (red[6] + red[7]);
  const double T2 = (red[8] + red[9]) + (red[10] + red[11]);
  for (int c = threadIdx.x; c <= loL; c += kThreads) G3[c] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int c = loL + WL + 1 + threadIdx.x; c <= nL; c += kThreads)
    G3[c] = make_float4((float)T0, (float)T1, (float)T2, 0.0f);
  if (threadIdx.x == 0) {
    tot[0] = T0;
    tot[1] = T1;
    tot[2] = T2;
  }
  __syncthreads();
}

// row table of the adjoint run form for rows [r0, r0 + rc) of the window
__device__ __forceinline__ void build_rows_bwd_runs(const SweepArgs& a, float* smem, const Win& w,
                                                    long long r0, int rc, long long kc, int loL,
                                                    int hiL) {
  const int D = a.g.ndim;
  BwdRunRow* rt = reinterpret_cast<BwdRunRow*>(smem + a.L.row_off);
  double rsig[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) rsig[d] = d + 1 < D ? 1.0 / a.d.sigma[kc * D + d] : 0.0;
  for (int r = threadIdx.x; r < rc; r += kThreads) {
    int t = (int)r0 + r;
    float go = 1.0f;
    float tv[3] = {0.0f, 0.0f, 0.0f};
    int gr = 0, mul = 1;
#pragma unroll
    for (int d = 2; d >= 0; --d) {
      if (d <= D - 2) {
        const int i = d == 0 ? t : t % w.W[d];
        if (d > 0) t /= w.W[d];
        go *= smem[a.L.tab_off[d] + i];
        gr += (w.lo[d] + i) * mul;
        mul *= a.g.n[d];
        const double x = cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], w.lo[d] + i);
        tv[d] = (float)((x - a.d.mu[kc * D + d]) * rsig[d]);
      }
    }
    const int off = gr * a.g.pitch;
    const int base = a.rowptr[gr];
    BwdRunRow e;
    e.go = go;
    e.t[0] = tv[0];
    e.t[1] = tv[1];
    e.t[2] = tv[2];
    e.ra = base + (int)a.runidx[off + loL];
    e.cnt = base + (int)a.runidx[off + hiL] + 1 - e.ra;
    e.pad[0] = e.pad[1] = 0;
    rt[r] = e;
  }
}

template <int NO>
__device__ __forceinline__ void bwd_runs(const SweepArgs& a, float* smem, int rc,
                                         BwdAcc<NO>& acc) {
  const int l = threadIdx.x & (kRunGroup - 1);
  const int gi = (threadIdx.x >> 4) & 3;
  const int wv = threadIdx.x >> 6;
  const BwdRunRow* rt = reinterpret_cast<const BwdRunRow*>(smem + a.L.row_off);
  const char* vt = reinterpret_cast<const char*>(smem + a.L.hist_off);
  const uint32_t gaddr = lds_addr(smem);  // G3 (16-byte entries per column)
  struct {
    float a0, l1, l2, o1[NO > 0 ? NO : 1], o2[NO > 0 ? NO : 1];
  } b = {};
  int nrow = 0;
  auto flush = [&]() {
    acc.a0 += (double)b.a0;
    acc.l1 += (double)b.l1;
    acc.l2 += (double)b.l2;
#pragma unroll
    for (int d = 0; d < NO; ++d) {
      acc.o1[d] += (double)b.o1[d];
      acc.o2[d] += (double)b.o2[d];
    }
    b = {};
  };
  // the four groups of a wave take adjacent rows (similar run counts; there
  // are no atomics to spread over banks here)
  for (int r = 4 * wv + gi; r < rc; r += 4 * kWaves) {
    const BwdRunRow row = rt[r];
    const int cnt = row.cnt;
    const uint32_t* rp = a.runs + row.ra;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    auto step = [&](uint32_t c, uint32_t dc, uint32_t dn, int left) {
      const uint32_t nx = (l == kRunGroup - 1) ? dn : dc;
      if (left > 0) {
        const f32x4v gs = lds_load_f4(mad_lo16_k<16>(c, gaddr));
        const f32x4v ge = lds_load_f4(mad_lo16_k<16>(nx, gaddr));
        const float vb = *reinterpret_cast<const float*>(vt + (c >> 16));
        a0 = fmaf(vb, ge.x - gs.x, a0);
        a1 = fmaf(vb, ge.y - gs.y, a1);
        a2 = fmaf(vb, ge.z - gs.z, a2);
      }
    };
    uint32_t cur = rp[l];
    uint32_t dcur = next_lane(cur);
    for (int q0 = l; q0 - l < cnt; q0 += 4 * kRunGroup) {
      const uint32_t* p = rp + q0;
      const uint32_t r1 = p[kRunGroup];
      const uint32_t r2 = p[2 * kRunGroup];
      const uint32_t r3 = p[3 * kRunGroup];
      const uint32_t r4 = p[4 * kRunGroup];
      const uint32_t d1 = next_lane(r1), d2 = next_lane(r2);
      const uint32_t d3 = next_lane(r3), d4 = next_lane(r4);
      const int left = cnt - q0;
      step(cur, dcur, d1, left);
      step(r1, d1, d2, left - kRunGroup);
      step(r2, d2, d3, left - 2 * kRunGroup);
      step(r3, d3, d4, left - 3 * kRunGroup);
      cur = r4;
      dcur = d4;
    }
    // per-row sums times the row factor (and the slower axes' t), gathered
    // in FP32 over at most eight rows, then in FP64
    const float c0 = row.go * a0;
    b.a0 += c0;
    b.l1 = fmaf(row.go, a1, b.l1);
    b.l2 = fmaf(row.go, a2, b.l2);
    if constexpr (NO > 0) {
#pragma unroll
      for (int d = 0; d < NO; ++d) {
        const float ct = c0 * row.t[d];
        b.o1[d] += ct;
        b.o2[d] = fmaf(ct, row.t[d], b.o2[d]);
      }
    }
    if (++nrow == 8) {
      flush();
      nrow = 0;
    }
  }
  flush();
}

template <int NO>
__global__ __launch_bounds__(kThreads, NO <= 1 ? 5 : 1) void k_backward_runs(SweepArgs a) {
  extern __shared__ float smem[];
  if (!runs_chosen(a)) return;  // k_backward does the work
  const long long k = block_k(a);
  if (k >= a.d.K) return;
  const int D = a.g.ndim;
  const int L = D - 1;
  double* red = reinterpret_cast<double*>(smem + a.L.red_off);
  double* tot = red + 16;  // FP64 window totals of G0, G1, G2
  float* vt = smem + a.L.hist_off;
  const double vref = build_vtable(a, vt, k, red);
  for (int c = 0; c < a.d.C; ++c) {
    const long long kc = k * a.d.C + c;
    const Win w = make_win(a, kc, reinterpret_cast<int*>(smem + a.L.red_off + 80));
    const double pc = (a.d.C > 1) ? a.d.weight[kc] : 1.0;
    if (w.bad || w.empty) {
      if (threadIdx.x == 0) {
        const double val = w.bad ? __builtin_nan("") : 0.0;
        for (int d = 0; d < D; ++d) {
          a.g_mu[kc * D + d] = val;
          a.g_sigma[kc * D + d] = val;
        }
        if (a.g_weight) a.g_weight[kc] = val;
      }
      continue;
    }
    int loL, WL;
    last_axis(w, D, loL, WL);
    __syncthreads();  // LDS reuse across components
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d + 1 < D) {
        float* tab = smem + a.L.tab_off[d];
        const double mu = a.d.mu[kc * D + d], rsig = 1.0 / a.d.sigma[kc * D + d];
        const double off = scale_log(win_m(a, smem, d));
        for (int i = threadIdx.x; i < w.W[d]; i += kThreads)
          tab[i] = gauss_factor_r(cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], w.lo[d] + i), mu,
                                  rsig, off);
      }
    }
    build_prefix_bwd(a, smem, kc, loL, WL, scale_log(win_m(a, smem, D - 1)), red, tot);
    BwdAcc<NO> acc;
    acc.a0 = acc.l1 = acc.l2 = 0.0;
#pragma unroll
    for (int i = 0; i < (NO > 0 ? NO : 1); ++i) acc.o1[i] = acc.o2[i] = 0.0;
    for (long long r0 = 0; r0 < w.R; r0 += kBwdRowChunk) {
      const int rc = (int)((w.R - r0) < kBwdRowChunk ? (w.R - r0) : kBwdRowChunk);
      __syncthreads();
      build_rows_bwd_runs(a, smem, w, r0, rc, kc, loL, loL + WL - 1);
      __syncthreads();
      bwd_runs<NO>(a, smem, rc, acc);
    }
    // per-axis normalisers and score means: the fastest axis from the FP64
    // totals, the slower axes from their factor tables
    const double T0 = tot[0], T1 = tot[1], T2 = tot[2];
    double Z = T0, m1[4], m2[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      m1[d] = m2[d] = 0.0;
      if (d + 1 < D) {
        const double mu = a.d.mu[kc * D + d], rsg = 1.0 / a.d.sigma[kc * D + d];
        double z0 = 0.0, z1 = 0.0, z2 = 0.0;
        for (int i = threadIdx.x; i < w.W[d]; i += kThreads) {
          const double g = (double)smem[a.L.tab_off[d] + i];
          const double t = (cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], w.lo[d] + i) - mu) * rsg;
          z0 += g;
          z1 += g * t;
          z2 += g * t * t;
        }
        const double Zd = block_sum(z0, red);
        m1[d] = block_sum(z1, red) / Zd;
        m2[d] = block_sum(z2, red) / Zd;
        Z *= Zd;
      } else if (d == L) {
        m1[d] = T1 / T0;
        m2[d] = T2 / T0;
      }
    }
    const double A0 = block_sum(acc.a0, red) / Z;
    double t1[4], t2[4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      t1[d] = d < NO ? block_sum(acc.o1[d < NO ? d : 0], red) / Z : 0.0;
      t2[d] = d < NO ? block_sum(acc.o2[d < NO ? d : 0], red) / Z : 0.0;
    }
    t1[3] = 0.0;
    t2[3] = 0.0;
    const double l1 = block_sum(acc.l1, red) / Z;
    const double l2 = block_sum(acc.l2, red) / Z;
    write_grads(a, w, kc, pc, A0, l1, l2, t1, t2, m1, m2, vref);
  }
}

// ===========================================================================
// host side
// ===========================================================================
static int round_up(int x, int m) { return (x + m - 1) / m * m; }

bool sweep_layout(const vup_grid& g, int B, SweepKind kind, SweepLayout* out, int run_rows) {
  SweepLayout L{};
  L.rrows = run_rows > 0 ? run_rows : kRunRowChunk;
  const int D = g.ndim;
  int off = 0;
  for (int d = 0; d < 4; ++d) {
    L.tab_off[d] = -1;
    L.cap[d] = 0;
  }
  // the run form starts with the FP64 prefix sums G[0..n] of the fastest
  // axis (at offset 0, so a column times 8 is its byte address)
  L.g_off = -1;
  if (kind == kSweepRuns) {
    L.g_off = 0;
    off = round_up(2 * (g.n[D - 1] + 1), 4);
  } else if (kind == kSweepBwdRuns) {
    // (G0, G1, G2, -) FP32 per column, 16 bytes
    L.g_off = 0;
    off = 4 * (g.n[D - 1] + 1);
  }
  const bool runform = kind == kSweepRuns || kind == kSweepBwdRuns;
  // factor tables: every axis for the cell sweeps; the run forms keep the
  // slower axes only
  const int ntab = runform ? D - 1 : D;
  for (int d = 0; d < ntab; ++d) {
    const int cap = (d + 1 < D) ? g.n[d] : g.n[d] + 64;
    L.cap[d] = round_up(cap, 4);
    L.tab_off[d] = off;
    off += L.cap[d];
  }
  off = round_up(off, 4);
  L.row_off = off;
  if (kind == kSweepPropagate) L.rrows = kPropRowChunk;
  // (the cell form's row table, 2 floats per row, is also the scratch of its
  // per-copy scales: kPropScaleScratch doubles)
  off += kind == kSweepRuns ? 4 * L.rrows
         : kind == kSweepPropagate ? round_up(std::max(2 * L.rrows, 2 * kPropScaleScratch), 4)
         : kind == kSweepBwdRuns ? 8 * kBwdRowChunk : 2 * kRowChunk;
  L.trow_off = -1;
  if (kind == kSweepBackward) {
    L.trow_off = off;
    off += 4 * kRowChunk;
  }
  L.hist_off = off;
  L.hist_stride = 0;
  L.cpw = 0;
  L.ncls = 1;
  if (kind == kSweepPropagate) {
    // NC histogram copies interleaved by bin: the most (up to 16) that keep a
    // workgroup within about 40 KB of LDS (four workgroups per CU), else the
    // most that fit at all; hist_stride holds the words to clear (NC (B + 1)
    // rounded up to a multiple of four, for 16-byte stores)
    const int budget = 40 * 1024 / 4 - 96 - kPropScalesFloats;
    int nc = 16;
    while (nc > 1 && off + round_up(nc * (B + 1), 4) > budget) nc /= 2;
    while (nc > 1 && off + round_up(nc * (B + 1), 4) > 160 * 1024 / 4 - 96 - kPropScalesFloats)
      nc /= 2;
    L.ncls = 1;
    L.cpw = nc;
    L.cshift = 0;
    while ((1 << L.cshift) < nc) ++L.cshift;
    L.hist_stride = round_up(nc * (B + 1), 4);
    off += L.hist_stride;
  } else if (kind == kSweepRuns) {
    // three row classes, one copy each
    const int stride = round_up(B + 1, 32) + 1;
    L.hist_stride = stride;
    L.ncls = 3;
    L.cpw = 1;
    off += 3 * stride;
  } else if (kind == kSweepBwdRuns) {
    off += round_up(B + 1, 4);  // weight table
  } else if (kind == kSweepBackward) {
    off += round_up(B + 1, 4);
    // fastest-axis factor times t and times t^2 (t = (x - mu)/sigma)
    L.g_off = off;
    off += 2 * L.cap[D - 1];
  }
  off = round_up(off, 4);
  L.red_off = off;
  off += 96;  // 16 doubles of reduction scratch, per-component scales, window ints
  if (kind == kSweepPropagate) off += round_up(kPropScalesFloats, 4);  // per-copy scales
  L.bytes = (size_t)off * 4;
  *out = L;
  return L.bytes <= 160 * 1024;
}

GridDev make_grid_dev(const vup_mm& mm) {
  GridDev g{};
  g.ndim = mm.grid.ndim;
  for (int d = 0; d < 4; ++d) {
    g.n[d] = d < g.ndim ? mm.grid.n[d] : 1;
    g.lo[d] = mm.grid.lo[d];
    g.hi[d] = mm.grid.hi[d];
    g.rowstride[d] = 0;
  }
  g.pitch = mm.pitch;
  // element stride of axis d (< ndim-1) in the padded map: product of the
  // later non-fastest axes times the pitch
  long long s = mm.pitch;
  for (int d = g.ndim - 2; d >= 0; --d) {
    g.rowstride[d] = s;
    s *= g.n[d];
  }
  return g;
}

DistsDev make_dists_dev(const vup_dists& d) {
  DistsDev r;
  r.K = d.K;
  r.C = d.ncomp;
  r.ns = d.n_sigma;
  r.mu = d.mu;
  r.sigma = d.sigma;
  r.weight = d.weight;
  return r;
}

// run records hold 16-bit columns and are addressed with 32-bit offsets; the
// run form's LDS (prefix sums of a whole fastest axis) must fit in 64 KiB
bool runs_allowed(const vup_mm& mm) {
  SweepLayout L;
  return mm.grid.n[mm.grid.ndim - 1] <= 65534 && mm.N < (1ll << 30) &&
         sweep_layout(mm.grid, mm.B, kSweepRuns, &L) && L.bytes <= 64 * 1024;
}

static SweepArgs base_args(const vup_mm& mm, const vup_dists& d, SweepKind kind) {
  SweepArgs a{};
  a.g = make_grid_dev(mm);
  a.d = make_dists_dev(d);
  a.B = mm.B;
  const char* ws = static_cast<const char*>(mm.ws);
  a.binmap = reinterpret_cast<const uint16_t*>(ws + mm.off_binmap);
  a.f32 = reinterpret_cast<const float*>(ws + mm.off_f32);
  a.edges = reinterpret_cast<const double*>(ws + mm.off_edges);
  a.counters = reinterpret_cast<unsigned long long*>(static_cast<char*>(mm.ws) + mm.off_counters);
  sweep_layout(mm.grid, mm.B, kind, &a.L);
  a.kpx = (d.K + 7) / 8;
  a.runs = reinterpret_cast<const uint32_t*>(ws + mm.off_runs);
  a.rowptr = reinterpret_cast<const int*>(ws + mm.off_rowptr);
  a.runidx = reinterpret_cast<const uint16_t*>(ws + mm.off_runidx);
  a.ncells = mm.N;
  a.allow_runs = runs_allowed(mm);
  return a;
}

static dim3 sweep_grid(const vup_dists& d) { return dim3((unsigned)(8 * ((d.K + 7) / 8))); }

// dynamic LDS above 64 KiB must be enabled per kernel
template <typename F>
static hipError_t allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_propagate(const vup_mm& mm, const vup_dists& d, int prec, float* P, double* Z,
                            hipStream_t s) {
  if (d.K == 0) return hipSuccess;
  SweepArgs a = base_args(mm, d, kSweepPropagate);
  a.P = P;
  a.Z = Z;
  const dim3 grid = sweep_grid(d), block(kThreads);
  hipError_t e = hipSuccess;
  if (prec == VUP_FP32 && a.allow_runs && mm.sweep != VUP_SWEEP_CELLS) {
    // the run form returns at once unless the device-side mode and run
    // statistics select it; the cell form below then returns at once
    SweepArgs ar = a;
    // with fewer distributions than the GPU holds workgroups, occupancy does
    // not matter and the larger row table saves passes
    const long long nwg = 8 * ((d.K + 7) / 8);
    if (nwg <= 2048 && sweep_layout(mm.grid, mm.B, kSweepRuns, &ar.L, 2 * kRunRowChunk) &&
        ar.L.bytes <= 64 * 1024) {
      hipLaunchKernelGGL(k_propagate_runs<2 * kRunRowChunk>, grid, block, ar.L.bytes, s, ar);
    } else {
      sweep_layout(mm.grid, mm.B, kSweepRuns, &ar.L);
      hipLaunchKernelGGL(k_propagate_runs<kRunRowChunk>, grid, block, ar.L.bytes, s, ar);
    }
    e = hipGetLastError();
    if (e != hipSuccess || mm.sweep == VUP_SWEEP_RUNS) return e;
  }
  switch (prec) {
    case VUP_BF16: e = allow_lds(k_propagate<VUP_BF16>, a.L.bytes); break;
    case VUP_BF16X2: e = allow_lds(k_propagate<VUP_BF16X2>, a.L.bytes); break;
    case VUP_FP8E4M3: e = allow_lds(k_propagate<VUP_FP8E4M3>, a.L.bytes); break;
    default: e = allow_lds(k_propagate<VUP_FP32>, a.L.bytes); break;
  }
  if (e != hipSuccess) return e;
  switch (prec) {
    case VUP_BF16: hipLaunchKernelGGL(k_propagate<VUP_BF16>, grid, block, a.L.bytes, s, a); break;
    case VUP_BF16X2:
      hipLaunchKernelGGL(k_propagate<VUP_BF16X2>, grid, block, a.L.bytes, s, a);
      break;
    case VUP_FP8E4M3:
      hipLaunchKernelGGL(k_propagate<VUP_FP8E4M3>, grid, block, a.L.bytes, s, a);
      break;
    default: hipLaunchKernelGGL(k_propagate<VUP_FP32>, grid, block, a.L.bytes, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_moments(const vup_mm& mm, const vup_dists& d, const vup_model* model,
                          double* mean, double* var, double* delta2, hipStream_t s) {
  if (d.K == 0) return hipSuccess;
  SweepArgs a = base_args(mm, d, kSweepMoments);
  a.mean = mean;
  a.var = var;
  a.delta2 = delta2;
  a.has_model = model != nullptr;
  if (model) a.model = *model;
  const hipError_t e = allow_lds(k_moments, a.L.bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_moments, sweep_grid(d), dim3(kThreads), a.L.bytes, s, a);
  return hipGetLastError();
}

hipError_t launch_backward(const vup_mm& mm, const vup_dists& d, const float* P,
                           const double* mean_hist, const double* g_var, const double* g_ent,
                           double* g_mu, double* g_sigma, double* g_weight, hipStream_t s) {
  if (d.K == 0) return hipSuccess;
  SweepArgs a = base_args(mm, d, kSweepBackward);
  a.Pin = P;
  a.mean_hist = mean_hist;
  a.g_var = g_var;
  a.g_ent = g_ent;
  a.g_mu = g_mu;
  a.g_sigma = g_sigma;
  a.g_weight = g_weight;
  const int D = mm.grid.ndim;
  hipError_t e = hipSuccess;
  // the run form, when the model matrix uses it and its LDS fits in 64 KiB
  SweepArgs ar = a;
  a.allow_runs = a.allow_runs && sweep_layout(mm.grid, mm.B, kSweepBwdRuns, &ar.L) &&
                 ar.L.bytes <= 64 * 1024;
  ar.allow_runs = a.allow_runs;
  if (a.allow_runs && mm.sweep != VUP_SWEEP_CELLS) {
    const dim3 grid = sweep_grid(d), block(kThreads);
    switch (D) {
      case 1: hipLaunchKernelGGL(k_backward_runs<0>, grid, block, ar.L.bytes, s, ar); break;
      case 2: hipLaunchKernelGGL(k_backward_runs<1>, grid, block, ar.L.bytes, s, ar); break;
      case 3: hipLaunchKernelGGL(k_backward_runs<2>, grid, block, ar.L.bytes, s, ar); break;
      default: hipLaunchKernelGGL(k_backward_runs<3>, grid, block, ar.L.bytes, s, ar); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess || mm.sweep == VUP_SWEEP_RUNS) return e;
  }
  switch (D) {
    case 1: e = allow_lds(k_backward<0>, a.L.bytes); break;
    case 2: e = allow_lds(k_backward<1>, a.L.bytes); break;
    case 3: e = allow_lds(k_backward<2>, a.L.bytes); break;
    default: e = allow_lds(k_backward<3>, a.L.bytes); break;
  }
  if (e != hipSuccess) return e;
  switch (D) {
    case 1: hipLaunchKernelGGL(k_backward<0>, sweep_grid(d), dim3(kThreads), a.L.bytes, s, a); break;
    case 2: hipLaunchKernelGGL(k_backward<1>, sweep_grid(d), dim3(kThreads), a.L.bytes, s, a); break;
    case 3: hipLaunchKernelGGL(k_backward<2>, sweep_grid(d), dim3(kThreads), a.L.bytes, s, a); break;
    default: hipLaunchKernelGGL(k_backward<3>, sweep_grid(d), dim3(kThreads), a.L.bytes, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace vup
