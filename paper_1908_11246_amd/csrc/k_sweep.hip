// Window sweeps over the shared model matrix: propagation (eq. VUP), exact-f
// moments, and the adjoint sweep of the IPSA sensitivities.
//
// One workgroup (256 threads, 4 waves) handles one distribution k and loops
// over its mixture components. For each component:
//   1. the truncation window is computed per axis (FP64, exact op order) and
//      the per-axis Gaussian factors g_d(j) are tabulated in LDS (FP32). The
//      fastest-axis table is zero-padded to whole strips;
//   2. the window is swept as rows (all axes but the fastest) x strips of SW
//      consecutive cells of the fastest axis, aligned to SW in the padded bin
//      map. A thread keeps its strip's factors in registers and walks rows; the
//      row factor (product of the slower axes' factors) and the row's bin-map
//      offset come from a row table in LDS;
//   3. per cell the density is one FP32 multiply (row factor x fastest-axis
//      factor); it is accumulated into the bin's LDS slot as a 32-bit
//      fixed-point integer (LDS float atomics are two orders of magnitude
//      slower than integer ones on gfx950). Cells are split into magnitude
//      classes with one histogram and one scale each, so tail cells keep a
//      fine quantum (see the fixed-point notes below). Integer sums are exact,
//      so results do not depend on scheduling.
// The input probability matrix is never materialised.
#include <hip/hip_runtime.h>

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

// per-component window state, identical in every thread of the workgroup
struct Win {
  int lo[4];
  int W[4];
  long long R;  // rows
  bool bad;
  bool empty;
};

__device__ __forceinline__ Win make_win(const SweepArgs& a, long long kc) {
  Win w;
  w.bad = false;
  w.empty = false;
  w.R = 1;
  const int D = a.g.ndim;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    w.lo[d] = 0;
    w.W[d] = 1;
    if (d < D) {
      int jlo, jhi;
      const bool ok = axis_window(a.g.lo[d], a.g.hi[d], a.g.n[d], a.d.mu[kc * D + d],
                                  a.d.sigma[kc * D + d], a.d.ns, jlo, jhi);
      if (!ok) w.bad = true;
      if (jhi < jlo) w.empty = true;
      w.lo[d] = jlo;
      w.W[d] = jhi - jlo + 1;
      if (d + 1 < D) w.R *= (w.W[d] > 0 ? w.W[d] : 0);
    }
  }
  return w;
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

// strip width minimising the sweep time estimate of one component
__device__ __forceinline__ int choose_sw(int loL, int WL, long long R, int maxsw) {
  int best = 4;
  long long bestc = 0x7fffffffffffffffll;
  for (int sw = 4; sw <= maxsw; sw *= 2) {
    const int ns = (loL + WL - 1) / sw - loL / sw + 1;
    const int cols = ns < kThreads ? ns : kThreads;
    const int P0 = kThreads / cols;
    const long long ncg = (ns + kThreads - 1) / kThreads;
    const long long c = ((R + P0 - 1) / P0) * ncg * (sw + 6);
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
      const double mu = a.d.mu[kc * D + d], sg = a.d.sigma[kc * D + d];
      for (int i = threadIdx.x; i < w.W[d]; i += kThreads) {
        const double x = cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], w.lo[d] + i);
        tab[i] = gauss_factor(x, mu, sg);
      }
    }
  }
  const int L = D - 1;
  int loL, WL;
  last_axis(w, D, loL, WL);
  float* tab = smem + a.L.tab_off[L];
  const double mu = a.d.mu[kc * D + L], sg = a.d.sigma[kc * D + L];
  for (int jj = threadIdx.x; jj < ns * sw; jj += kThreads) {
    const int j = colbase + jj;
    float v = 0.0f;
    if (j >= loL && j < loL + WL) {
      const double x = cell_centre(a.g.lo[L], a.g.hi[L], a.g.n[L], j);
      v = gauss_factor(x, mu, sg);
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
    long long t = r0 + r;
    float go = 1.0f;
    long long off = 0;
    float tv[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int d = 2; d >= 0; --d) {
      if (d <= D - 2) {
        const int i = (int)(t % w.W[d]);
        t /= w.W[d];
        go *= smem[a.L.tab_off[d] + i];
        off += (long long)(w.lo[d] + i) * a.g.rowstride[d];
        if (trow) {
          const double x = cell_centre(a.g.lo[d], a.g.hi[d], a.g.n[d], w.lo[d] + i);
          tv[d] = (float)((x - a.d.mu[kc * D + d]) / a.d.sigma[kc * D + d]);
        }
      }
    }
    rt[r] = make_float2(go, __int_as_float((int)off));
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
// Sum of the tabulated per-axis factors of the current window, multiplied
// over the axes (FP64): the total weight of the separable truncated density.
__device__ __forceinline__ double table_mass(const SweepArgs& a, const float* smem, const Win& w,
                                             int ns, int sw, double* red) {
  const int D = a.g.ndim;
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
  return Z;
}

// ---------------------------------------------------------------------------
// Fixed-point histogram accumulation.
// The density of a cell is the product go * gl of its row factor and its
// fastest-axis factor. Cells are split into 3 x 3 magnitude classes by the row
// factor (go >= 2^-4, >= 2^-8, smaller) and by the largest factor of their
// strip; every class has its own LDS histogram and its own scale
//     scale[rc][cc] = K / (qfac * rowbound[rc] * colmass[cc]),
// where colmass is the exact factor sum of the strips in class cc, rowbound an
// upper bound of the row factors' sum in class rc, qfac >= 1 the largest
// relative increase of a density by the precision's rounding, and
// K = 2^32 - 2^20 - (cells). A cell adds floor(w * scale + u) with a fixed
// dither u = (j + 1/2)/SW that depends only on its position j in the strip, so
// no class total can exceed 2^32: nothing overflows, tail cells keep a fine
// quantum, and rounding is unbiased on average. Integer adds are exact, so
// the result does not depend on scheduling.
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

// per-component scales shared by all threads (LDS): srow[3], scol[3], inv[9]
struct PropScales {
  float srow[3];
  float scol[3];
  double unscale[9];  // 1 / scale of each class (FP64)
  int peak;           // run form: index of the largest fastest-axis factor
};

template <int PREC>
__device__ __forceinline__ void prop_scales(const SweepArgs& a, float* smem, const Win& w, int ns,
                                            int sw, double* red, PropScales* ps, bool runmode) {
  const int D = a.g.ndim;
  const float* tabL = smem + a.L.tab_off[D - 1];
  double cm[3] = {0.0, 0.0, 0.0};
  if (!runmode) {
    // column classes: by the largest factor of each strip
    for (int st = threadIdx.x; st < ns; st += kThreads) {
      float gmax = 0.0f;
      double sum = 0.0;
      for (int j = 0; j < sw; ++j) {
        const float g = tabL[st * sw + j];
        gmax = fmaxf(gmax, g);
        sum += (double)g;
      }
      const int cc = mag_class(gmax);
      cm[0] += cc == 0 ? sum : 0.0;
      cm[1] += cc == 1 ? sum : 0.0;
      cm[2] += cc == 2 ? sum : 0.0;
    }
  } else {
    // runs are classed by their largest factor, so a class-c run holds only
    // columns below the class ceiling: bound by the sum of all such columns
    for (int j = threadIdx.x; j < ns * sw; j += kThreads) {
      const float g = tabL[j];
      cm[0] += (double)g;
      cm[1] += g < kClassT1 ? (double)g : 0.0;
      cm[2] += g < kClassT2 ? (double)g : 0.0;
    }
  }
  double colmass[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) colmass[c] = block_sum(cm[c], red);
  // row factor sum bound per class: total row mass, and rows * class ceiling
  double Zrows = 1.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d + 1 < D) {
      double zp = 0.0;
      for (int i = threadIdx.x; i < w.W[d]; i += kThreads) zp += (double)smem[a.L.tab_off[d] + i];
      Zrows *= block_sum(zp, red);
    }
  }
  const double R = (double)w.R;
  const double cells = R * (double)(ns * sw);
  double K = 4294967296.0 - 1048576.0 - cells;
  if (PREC == VUP_FP8E4M3) K *= 0.5;  // subnormal rounding of tiny values
  if (threadIdx.x == 0) {
    if (a.L.ncls > 1) {
      const double rowbound[3] = {Zrows, fmin(Zrows, R * (double)kClassT1),
                                  fmin(Zrows, R * (double)kClassT2)};
      for (int r = 0; r < 3; ++r) ps->srow[r] = (float)(K / (prec_qfac<PREC>() * rowbound[r]));
      for (int c = 0; c < 3; ++c) ps->scol[c] = colmass[c] > 0.0 ? (float)(1.0 / colmass[c]) : 0.0f;
    } else {
      // a single class: one scale for the whole window
      const double cmass = colmass[0] + colmass[1] + colmass[2];
      for (int r = 0; r < 3; ++r) ps->srow[r] = (float)(K / (prec_qfac<PREC>() * Zrows));
      for (int c = 0; c < 3; ++c) ps->scol[c] = (float)(1.0 / cmass);
    }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        ps->unscale[r * 3 + c] =
            ps->scol[c] > 0.0f ? 1.0 / ((double)ps->srow[r] * (double)ps->scol[c]) : 0.0;
  }
}

// Row table of the propagation: (go, go * srow[class], map offset, class).
__device__ __forceinline__ void build_rows_prop(const SweepArgs& a, float* smem, const Win& w,
                                                long long r0, int rc, const PropScales* ps) {
  const int D = a.g.ndim;
  float4* rt = reinterpret_cast<float4*>(smem + a.L.row_off);
  for (int r = threadIdx.x; r < rc; r += kThreads) {
    long long t = r0 + r;
    float go = 1.0f;
    long long off = 0;
#pragma unroll
    for (int d = 2; d >= 0; --d) {
      if (d <= D - 2) {
        const int i = (int)(t % w.W[d]);
        t /= w.W[d];
        go *= smem[a.L.tab_off[d] + i];
        off += (long long)(w.lo[d] + i) * a.g.rowstride[d];
      }
    }
    const int cls = a.L.ncls > 1 ? mag_class(go) : 0;
    rt[r] = make_float4(go, go * ps->srow[cls], __int_as_float((int)off), __int_as_float(cls));
  }
}

template <int SW, int PREC>
__device__ __forceinline__ void prop_rows(const SweepArgs& a, float* smem, int rc, int colbase,
                                          int ns, const PropScales* ps) {
  const int cols = ns < kThreads ? ns : kThreads;
  const int P0 = kThreads / cols;
  const int col = threadIdx.x % cols;
  const int ph = threadIdx.x / cols;
  if (ph >= P0) return;
  const float4* rt = reinterpret_cast<const float4*>(smem + a.L.row_off);
  const int cpc = a.L.cpw;  // copies per class
  const int strideb = a.L.hist_stride * 4;
  // byte offset between row classes (3 column classes x cpc copies each)
  const int rcstep = 3 * cpc * strideb;
  char* hbase = reinterpret_cast<char*>(smem + a.L.hist_off) + (ph & (cpc - 1)) * strideb;
  const float* tabL = smem + a.L.tab_off[a.g.ndim - 1];
  for (int s = col; s < ns; s += cols) {
    float gl[SW];
    float gmax = 0.0f;
#pragma unroll
    for (int j = 0; j < SW; ++j) {
      gl[j] = tabL[s * SW + j];
      gmax = fmaxf(gmax, gl[j]);
    }
    const int cc = a.L.ncls > 1 ? mag_class(gmax) : 0;
    const float scol = ps->scol[cc];
    char* lh = hbase + cc * cpc * strideb;
    const int mcol = colbase + s * SW;
    int r = ph;
    if (r >= rc) continue;
    float4 cur = rt[r];
    MapVec<SW> mv = load_map<SW>(a.binmap + (long long)__float_as_int(cur.z) + mcol);
    for (; r < rc; r += P0) {
      const int rn = r + P0;
      float4 nxt = cur;
      MapVec<SW> mn = mv;
      if (rn < rc) {
        nxt = rt[rn];
        mn = load_map<SW>(a.binmap + (long long)__float_as_int(nxt.z) + mcol);
      }
      const int rcl = a.L.ncls > 1 ? __float_as_int(cur.w) : 0;
      char* lr = lh + rcl * rcstep;
      const float gos = cur.y * scol;
      float qs = 0.0f;
      if constexpr (PREC != VUP_FP32) {
        qs = ps->srow[rcl] * scol * (PREC == VUP_FP8E4M3 ? (1.0f / 448.0f) : 1.0f);
      }
#pragma unroll
      for (int j = 0; j < SW; ++j) {
        const float u = ((float)j + 0.5f) * (1.0f / (float)SW);
        float v;
        if constexpr (PREC == VUP_FP32) {
          v = fmaf(gos, gl[j], u);
        } else {
          v = fmaf(quantize<PREC>(cur.x * gl[j]), qs, u);
        }
        uint32_t* slot = reinterpret_cast<uint32_t*>(lr + map_at<SW>(mv, j));
        __hip_atomic_fetch_add(slot, (uint32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      cur = nxt;
      mv = mn;
    }
  }
}

// ---------------------------------------------------------------------------
// Run form (FP32 densities): along the fastest axis the model matrix is a
// sequence of runs of equal bin, and the density is separable, so a run's
// mass is go * (G[e] - G[s]) with G the FP64 prefix sums of the fastest-axis
// factors. Each lane handles one run (16 lanes per row); one integer atomic
// then carries a whole run instead of one cell.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void build_prefix(const SweepArgs& a, float* smem, int len, double* red2,
                                             int* pk) {
  // G[0] = 0, G[j+1] = G[j] + tab_L[j] in FP64; also the index of the
  // largest factor (smallest index among equal maxima)
  const float* tabL = smem + a.L.tab_off[a.g.ndim - 1];
  double* G = reinterpret_cast<double*>(smem + a.L.g_off);
  const int per = (len + kThreads - 1) / kThreads;
  const int j0 = threadIdx.x * per < len ? threadIdx.x * per : len;
  const int j1 = j0 + per < len ? j0 + per : len;
  double sum = 0.0;
  float best = -1.0f;
  int bidx = 0x7fffffff;
  for (int j = j0; j < j1; ++j) {
    const float g = tabL[j];
    sum += (double)g;
    if (g > best) {
      best = g;
      bidx = j;
    }
  }
  red2[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int t = 0; t < kThreads; ++t) {
      const double x = red2[t];
      red2[t] = run;
      run += x;
    }
  }
  __syncthreads();
  double run = red2[threadIdx.x];
  if (threadIdx.x == 0) G[0] = 0.0;
  for (int j = j0; j < j1; ++j) {
    run += (double)tabL[j];
    G[j + 1] = run;
  }
  // argmax: (value, -index) maximum over the block
  for (int o = 32; o > 0; o >>= 1) {
    const float ob = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bidx, o, 64);
    if (ob > best || (ob == best && oi < bidx)) {
      best = ob;
      bidx = oi;
    }
  }
  __syncthreads();
  float* rb = reinterpret_cast<float*>(red2);
  int* ri = reinterpret_cast<int*>(red2) + kWaves;
  if ((threadIdx.x & 63) == 0) {
    rb[threadIdx.x >> 6] = best;
    ri[threadIdx.x >> 6] = bidx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = rb[0];
    int i = ri[0];
    for (int wv = 1; wv < kWaves; ++wv)
      if (rb[wv] > b || (rb[wv] == b && ri[wv] < i)) {
        b = rb[wv];
        i = ri[wv];
      }
    *pk = i;
  }
  __syncthreads();
}

// row table of the run form: (go * srow[class], first run, end run, class)
__device__ __forceinline__ void build_rows_runs(const SweepArgs& a, float* smem, const Win& w,
                                                long long r0, int rc, const PropScales* ps,
                                                int loL, int hiL) {
  const int D = a.g.ndim;
  float4* rt = reinterpret_cast<float4*>(smem + a.L.row_off);
  for (int r = threadIdx.x; r < rc; r += kThreads) {
    long long t = r0 + r;
    float go = 1.0f;
    long long off = 0;
#pragma unroll
    for (int d = 2; d >= 0; --d) {
      if (d <= D - 2) {
        const int i = (int)(t % w.W[d]);
        t /= w.W[d];
        go *= smem[a.L.tab_off[d] + i];
        off += (long long)(w.lo[d] + i) * a.g.rowstride[d];
      }
    }
    const long long gr = off / a.g.pitch;  // grid row
    const int base = a.rowptr[gr];
    const int r_a = base + (int)a.runidx[off + loL];
    const int r_b = base + (int)a.runidx[off + hiL] + 1;
    const int cls = a.L.ncls > 1 ? mag_class(go) : 0;
    rt[r] = make_float4(go * ps->srow[cls], __int_as_float(r_a), __int_as_float(r_b),
                        __int_as_float(cls));
  }
}

// One row per 16-lane group; the row's m runs are split into contiguous
// chunks of ceil(m/16) per lane, whose records (and the next record, for the
// end column) are loaded together before any is used.
__device__ __forceinline__ void prop_runs(const SweepArgs& a, float* smem, int rc, int colbase,
                                          int loL, int hiL, int pk, const PropScales* ps) {
  const int grp = threadIdx.x >> 4;
  const int l = threadIdx.x & 15;
  const float4* rt = reinterpret_cast<const float4*>(smem + a.L.row_off);
  const double* G = reinterpret_cast<const double*>(smem + a.L.g_off);
  const float* tabL = smem + a.L.tab_off[a.g.ndim - 1];
  const int strideb = a.L.hist_stride * 4;
  const int rcstep = 3 * strideb;  // one copy per class in the run form
  char* hbase = reinterpret_cast<char*>(smem + a.L.hist_off);
  const float sc0 = ps->scol[0], sc1 = ps->scol[1], sc2 = ps->scol[2];
  const int hi1 = hiL + 1;
  for (int r = grp; r < rc; r += kThreads / 16) {
    const float4 t = rt[r];
    const int ra = __float_as_int(t.y), rb = __float_as_int(t.z);
    char* lr = hbase + (a.L.ncls > 1 ? __float_as_int(t.w) : 0) * rcstep;
    const int per = (rb - ra + 15) >> 4;
    int q = ra + l * per;
    const int qe = min(q + per, rb);
    while (q < qe) {
      uint32_t rec[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) rec[i] = (q + i <= qe) ? a.runs[q + i] : 0u;
      int s = ((int)(rec[0] & 0xFFFFu) > loL ? (int)(rec[0] & 0xFFFFu) : loL) - colbase;
      double gs = G[s];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (q + i < qe) {
          const int ce = (int)(rec[i + 1] & 0xFFFFu);
          const int e = (ce < hi1 ? ce : hi1) - colbase;
          const double ge = G[e];
          const float val = (float)(ge - gs);
          float gm = fmaxf(tabL[s], tabL[e - 1]);
          if (s <= pk && pk < e) gm = 1.0f;
          const int cc = a.L.ncls > 1 ? mag_class(gm) : 0;
          const float scol = cc == 0 ? sc0 : (cc == 1 ? sc1 : sc2);
          const float u = ((float)(l + 16 * i) + 0.5f) * (1.0f / 128.0f);
          const float v = fmaf(val, t.x * scol, u - floorf(u));
          uint32_t* slot = reinterpret_cast<uint32_t*>(lr + cc * strideb + (rec[i] >> 16));
          __hip_atomic_fetch_add(slot, (uint32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          s = e;
          gs = ge;
        }
      }
      q += 8;
    }
  }
}

template <int PREC>
__global__ __launch_bounds__(kThreads) void k_propagate(SweepArgs a) {
  extern __shared__ float smem[];
  const long long k = block_k(a);
  if (k >= a.d.K) return;
  const int D = a.g.ndim;
  const int B = a.B;
  const int nslots = B + 1;
  const int ncls = a.L.ncls;
  double* red = reinterpret_cast<double*>(smem + a.L.red_off);
  PropScales* ps = reinterpret_cast<PropScales*>(red + 16);
  const uint32_t* hist = reinterpret_cast<const uint32_t*>(smem + a.L.hist_off);
  float* Pk = a.P + k * (long long)B;
  bool anybad = false;
  bool written = false;  // row k holds a partial mixture
  // run form: FP32 densities and a model matrix whose runs along the fastest
  // axis are at least kRunMinLength cells long on average
  bool runmode = false;
  if constexpr (PREC == VUP_FP32) {
    const unsigned long long mode = a.counters[kCntMode];
    const unsigned long long nruns = a.counters[kCntRuns];
    runmode = a.allow_runs && nruns > 0 &&
              (mode == VUP_SWEEP_RUNS ||
               (mode == VUP_SWEEP_AUTO && (long long)nruns * kRunMinLength <= a.ncells));
  }
  // the run form keeps one histogram copy per class (its prefix tables use
  // the space of the others)
  const int cpc = runmode ? 1 : a.L.cpw;
  for (int c = 0; c < a.d.C; ++c) {
    const long long kc = k * a.d.C + c;
    const Win w = make_win(a, kc);
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
    build_tables(a, smem, w, kc, sw, colbase, ns);
    for (int i = threadIdx.x; i < ncls * cpc * a.L.hist_stride; i += kThreads)
      smem[a.L.hist_off + i] = 0.0f;
    __syncthreads();
    prop_scales<PREC>(a, smem, w, ns, sw, red, ps, runmode);
    int pk = 0;
    if (runmode) {
      build_prefix(a, smem, ns * sw, reinterpret_cast<double*>(smem + a.L.scan_off), &ps->peak);
      pk = ps->peak;
    }
    for (long long r0 = 0; r0 < w.R; r0 += kRowChunk) {
      const int rc = (int)((w.R - r0) < kRowChunk ? (w.R - r0) : kRowChunk);
      __syncthreads();
      if (runmode) build_rows_runs(a, smem, w, r0, rc, ps, loL, loL + WL - 1);
      else build_rows_prop(a, smem, w, r0, rc, ps);
      __syncthreads();
      if (runmode) {
        prop_runs(a, smem, rc, colbase, loL, loL + WL - 1, pk, ps);
      } else {
        switch (sw) {
          case 4: prop_rows<4, PREC>(a, smem, rc, colbase, ns, ps); break;
          case 8: prop_rows<8, PREC>(a, smem, rc, colbase, ns, ps); break;
          default: prop_rows<16, PREC>(a, smem, rc, colbase, ns, ps); break;
        }
      }
    }
    __syncthreads();
    // unscale each class, sum its copies; the normaliser is the sum over all
    // slots (cells without a bin included)
    double zpart = 0.0;
    for (int b = threadIdx.x; b < nslots; b += kThreads) {
      double v = 0.0;
      for (int cl = 0; cl < ncls; ++cl) {
        uint64_t cnt = 0;
        for (int cp = 0; cp < cpc; ++cp) cnt += hist[(cl * cpc + cp) * a.L.hist_stride + b];
          v += (double)cnt * ps->unscale[cl];
      }
      zpart += v;
    }
    const double Zc = block_sum(zpart, red);
    if (a.Z && threadIdx.x == 0) a.Z[kc] = Zc;
    const double f = ((a.d.C > 1) ? a.d.weight[kc] : 1.0) / Zc;
    for (int b = threadIdx.x; b < B; b += kThreads) {
      double v = 0.0;
      for (int cl = 0; cl < ncls; ++cl) {
        uint64_t cnt = 0;
        for (int cp = 0; cp < cpc; ++cp) cnt += hist[(cl * cpc + cp) * a.L.hist_stride + b];
        v += (double)cnt * ps->unscale[cl];
      }
      const double prev = written ? (double)Pk[b] : 0.0;
      Pk[b] = (float)(prev + v * f);
    }
    written = true;
  }
  if (anybad || !written)
    for (int b = threadIdx.x; b < B; b += kThreads) Pk[b] = anybad ? __builtin_nanf("") : 0.0f;
  if (threadIdx.x == 0) {
    if (anybad) atomicAdd(a.counters + kCntBadParam, 1ull);
    else if (!written) atomicAdd(a.counters + kCntEmpty, 1ull);
  }
}

// ===========================================================================
// exact-f moments: shifted FP32 strip sums, FP64 accumulation
// ===========================================================================
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
  const float* tabL = smem + a.L.tab_off[a.g.ndim - 1];
  for (int s = col; s < ns; s += cols) {
    float gl[SW];
#pragma unroll
    for (int j = 0; j < SW; ++j) gl[j] = tabL[s * SW + j];
    const int mcol = colbase + s * SW;
    for (int r = ph; r < rc; r += P0) {
      const float2 cur = rt[r];
      const float4* fp =
          reinterpret_cast<const float4*>(a.f32 + (long long)__float_as_int(cur.y) + mcol);
      float a1 = 0.0f, a2 = 0.0f;
#pragma unroll
      for (int q = 0; q < SW / 4; ++q) {
        const float4 fv = fp[q];
        const float fj[4] = {fv.x, fv.y, fv.z, fv.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float dv = fj[e] - shift;
          const float t = gl[4 * q + e] * dv;
          a1 += t;
          a2 = fmaf(t, dv, a2);
        }
      }
      A1 += (double)cur.x * (double)a1;
      A2 += (double)cur.x * (double)a2;
    }
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
    const Win w = make_win(a, kc);
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
    const int sw = choose_sw(loL, WL, w.R, kMaxSW);
    const int colbase = (loL / sw) * sw;
    const int ns = (loL + WL - 1) / sw - loL / sw + 1;
    // shift: model value at the window's centre cell
    long long cidx = loL + WL / 2;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (d + 1 < D) cidx += (long long)(w.lo[d] + w.W[d] / 2) * a.g.rowstride[d];
    const float shift = a.f32[cidx];
    __syncthreads();
    build_tables(a, smem, w, kc, sw, colbase, ns);
    double A1 = 0.0, A2 = 0.0;
    for (long long r0 = 0; r0 < w.R; r0 += kRowChunk) {
      const int rc = (int)((w.R - r0) < kRowChunk ? (w.R - r0) : kRowChunk);
      __syncthreads();
      build_rows(a, smem, w, r0, rc, kc, false);
      __syncthreads();
      switch (sw) {
        case 4: mom_rows<4>(a, smem, rc, colbase, ns, shift, A1, A2); break;
        case 8: mom_rows<8>(a, smem, rc, colbase, ns, shift, A1, A2); break;
        default: mom_rows<16>(a, smem, rc, colbase, ns, shift, A1, A2); break;
      }
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
    Vc[c] = s2 - s1 * s1;
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
struct BwdAcc {
  double a0, l1, l2;
  double o1[3], o2[3];
};

template <int SW>
__device__ __forceinline__ void bwd_rows(const SweepArgs& a, const float* smem, int rc,
                                         int colbase, int ns, double muL, double sgL,
                                         BwdAcc& acc) {
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
  const float* tabL = smem + a.L.tab_off[L];
  for (int s = col; s < ns; s += cols) {
    float gl[SW], g1[SW], g2[SW];
#pragma unroll
    for (int j = 0; j < SW; ++j) {
      gl[j] = tabL[s * SW + j];
      const int jj = colbase + s * SW + j;
      const double t = (cell_centre(a.g.lo[L], a.g.hi[L], a.g.n[L], jj) - muL) / sgL;
      g1[j] = (float)((double)gl[j] * t);
      g2[j] = (float)((double)gl[j] * t * t);
    }
    const int mcol = colbase + s * SW;
    for (int r = ph; r < rc; r += P0) {
      const float2 cur = rt[r];
      const MapVec<SW> mv = load_map<SW>(a.binmap + (long long)__float_as_int(cur.y) + mcol);
      float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
#pragma unroll
      for (int j = 0; j < SW; ++j) {
        const float vb = *reinterpret_cast<const float*>(vt + map_at<SW>(mv, j));
        a0 = fmaf(gl[j], vb, a0);
        a1 = fmaf(g1[j], vb, a1);
        a2 = fmaf(g2[j], vb, a2);
      }
      const double go = (double)cur.x;
      const double c0 = go * (double)a0;
      acc.a0 += c0;
      acc.l1 += go * (double)a1;
      acc.l2 += go * (double)a2;
      if (L > 0) {
        const float4 tv = tt[r];
        const float tr[3] = {tv.x, tv.y, tv.z};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double td = (double)tr[d];
          acc.o1[d] += c0 * td;
          acc.o2[d] += c0 * td * td;
        }
      }
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_backward(SweepArgs a) {
  extern __shared__ float smem[];
  const long long k = block_k(a);
  if (k >= a.d.K) return;
  const int D = a.g.ndim;
  const int B = a.B;
  double* red = reinterpret_cast<double*>(smem + a.L.red_off);
  const float* Pk = a.Pin + k * (long long)B;
  const double gv = a.g_var ? a.g_var[k] : 0.0;
  const double ge = a.g_ent ? a.g_ent[k] : 0.0;
  const double E = a.mean_hist[k];
  // S = sum_b P_b (c_b - E); v_b = gv((c_b - E)^2 - 2 c_b S) - ge(ln P_b + 1);
  // vref = sum_b P_b v_b is subtracted from the table (covariances are
  // shift invariant) and added back for the weight gradient.
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
    if (pb > 0.0) v -= ge * (log(pb) + 1.0);
    vp += pb * v;
  }
  const double vref = block_sum(vp, red);
  float* vt = smem + a.L.hist_off;
  for (int b = threadIdx.x; b <= B; b += kThreads) {
    double v = 0.0;
    if (b < B) {
      const double cb = 0.5 * (a.edges[b] + a.edges[b + 1]);
      const double pb = (double)Pk[b];
      v = gv * ((cb - E) * (cb - E) - 2.0 * cb * S);
      if (pb > 0.0) v -= ge * (log(pb) + 1.0);
    }
    // cells without a bin do not enter Var or H: their v is 0
    vt[b] = (float)(v - vref);
  }
  for (int c = 0; c < a.d.C; ++c) {
    const long long kc = k * a.d.C + c;
    const Win w = make_win(a, kc);
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
    const int sw = choose_sw(loL, WL, w.R, 16);
    const int colbase = (loL / sw) * sw;
    const int ns = (loL + WL - 1) / sw - loL / sw + 1;
    __syncthreads();
    build_tables(a, smem, w, kc, sw, colbase, ns);
    BwdAcc acc;
    acc.a0 = acc.l1 = acc.l2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) acc.o1[i] = acc.o2[i] = 0.0;
    const double muL = a.d.mu[kc * D + L];
    const double sgL = a.d.sigma[kc * D + L];
    for (long long r0 = 0; r0 < w.R; r0 += kRowChunk) {
      const int rc = (int)((w.R - r0) < kRowChunk ? (w.R - r0) : kRowChunk);
      __syncthreads();
      build_rows(a, smem, w, r0, rc, kc, true);
      __syncthreads();
      switch (sw) {
        case 4: bwd_rows<4>(a, smem, rc, colbase, ns, muL, sgL, acc); break;
        case 8: bwd_rows<8>(a, smem, rc, colbase, ns, muL, sgL, acc); break;
        default: bwd_rows<16>(a, smem, rc, colbase, ns, muL, sgL, acc); break;
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
      t1[d] = block_sum(acc.o1[d], red) / Z;
      t2[d] = block_sum(acc.o2[d], red) / Z;
    }
    t1[3] = 0.0;
    t2[3] = 0.0;
    const double l1 = block_sum(acc.l1, red) / Z;
    const double l2 = block_sum(acc.l2, red) / Z;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        if (d < D) {
          const double sg = a.d.sigma[kc * D + d];
          const double s1 = (d == L) ? l1 : t1[d < 3 ? d : 0];
          const double s2 = (d == L) ? l2 : t2[d < 3 ? d : 0];
          a.g_mu[kc * D + d] = pc * (s1 - m1[d] * A0) / sg;
          a.g_sigma[kc * D + d] = pc * (s2 - m2[d] * A0) / sg;
        }
      }
      if (a.g_weight) a.g_weight[kc] = A0 + vref;
    }
  }
}

// ===========================================================================
// host side
// ===========================================================================
static int round_up(int x, int m) { return (x + m - 1) / m * m; }

bool sweep_layout(const vup_grid& g, int B, SweepKind kind, SweepLayout* out) {
  SweepLayout L{};
  const int D = g.ndim;
  int off = 0;
  for (int d = 0; d < 4; ++d) {
    L.tab_off[d] = -1;
    L.cap[d] = 0;
  }
  for (int d = 0; d < D; ++d) {
    const int cap = (d + 1 < D) ? g.n[d] : g.n[d] + 64;
    L.cap[d] = round_up(cap, 4);
    L.tab_off[d] = off;
    off += L.cap[d];
  }
  off = round_up(off, 4);
  L.row_off = off;
  off += (kind == kSweepPropagate ? 4 : 2) * kRowChunk;
  L.trow_off = -1;
  if (kind == kSweepBackward) {
    L.trow_off = off;
    off += 4 * kRowChunk;
  }
  L.g_off = -1;
  L.scan_off = -1;
  L.hist_off = off;
  L.hist_stride = 0;
  L.cpw = 0;
  L.ncls = 1;
  if (kind == kSweepPropagate) {
    // stride = 1 mod 32 so consecutive copies shift banks by one
    const int stride = round_up(B + 1, 32) + 1;
    L.hist_stride = stride;
    // the run form keeps one copy per class and places the FP64 prefix sums
    // of the fastest-axis factors (and their scan scratch) behind it
    const int gfl = 2 * (L.cap[D - 1] + 2) + 2 * kThreads + 2;
    const int budget = 48 * 1024 / 4 - 64;
    const int opts[5][2] = {{9, 2}, {9, 1}, {1, 4}, {1, 2}, {1, 1}};
    auto need = [&](int i) {
      const int h2 = opts[i][0] * opts[i][1] * stride;
      const int h1 = round_up(opts[i][0] * stride, 2) + gfl;
      return h2 > h1 ? h2 : h1;
    };
    int pick = 4;
    for (int i = 0; i < 5; ++i)
      if (off + need(i) <= budget) {
        pick = i;
        break;
      }
    if (pick == 4)  // nothing fits the occupancy budget: take the richest that fits at all
      for (int i = 0; i < 5; ++i)
        if (off + need(i) <= 160 * 1024 / 4 - 64) {
          pick = i;
          break;
        }
    L.ncls = opts[pick][0];
    L.cpw = opts[pick][1];
    L.g_off = off + round_up(L.ncls * stride, 2);
    L.scan_off = L.g_off + 2 * (L.cap[D - 1] + 2);
    off += need(pick);
  } else if (kind == kSweepBackward) {
    off += round_up(B + 1, 4);
  }
  off = round_up(off, 4);
  L.red_off = off;
  off += 64;  // 16 doubles of reduction scratch + per-component scales
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
  a.allow_runs = mm.grid.n[mm.grid.ndim - 1] <= 65534;
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
  const hipError_t e = allow_lds(k_backward, a.L.bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_backward, sweep_grid(d), dim3(kThreads), a.L.bytes, s, a);
  return hipGetLastError();
}

}  // namespace vup
