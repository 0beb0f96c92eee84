// Separable ("banded") form of the propagation for a tensor-product family of
// 2-D Gaussians: distribution k = (mx, my) has mean (mu_x[mx], mu_y[my]) and
// deviations (sigma_x[mx], sigma_y[my]), e.g. measurement locations on a
// subgrid (Sec. 5.3 evaluates one pdf per location l). With the truncated
// per-axis factor matrices A_x[ix][mx], A_y[iy][my] (zero outside each window)
//   P[k][b] = 1/(Zx[mx] Zy[my]) sum_ix A_x[ix][mx] T[ix][b][my],
//   T[ix][b][my] = sum_{iy : bin(ix,iy) = b} A_y[iy][my],
// which is eq. VUP with the input matrix factorised: T is a cheap scatter
// over one axis, and the contraction over the other axis is a dense banded
// matrix product that runs on the matrix cores (MFMA, FP32 in and out).
//   k_axis_factors   A_d, Zd = sum_i A_d[i][m] (FP64), window bounds; each
//                    column scaled by its power of two (axis_scale_exp; the
//                    scale cancels from P)
//   k_sep_z          the normalisers Z[k] = Zx Zy with the scales put back
//   k_axis_prefix    G = prefix sums of A_y along y (FP64)
//   k_sep_runs_tiled T from the model matrix's runs of equal bin along y:
//                    one G difference per run, 32-bin LDS tiles, T written
//                    once (rows up to 4096 cells)
//   k_sep_runs       the same with read-modify-writes of T (rows up to 65534)
//   k_sep_scatter    T cell by cell (longer rows): one wave per (ix, 64 my),
//                    conflict-free LDS accumulation (lane = my), each run of
//                    same-bin cells summed in an FP64 register and rounded
//                    once (a run can span tens of thousands of cells)
//   k_sep_gemm       the banded contraction on the matrix cores, 16x16x4 FP32
//                    MFMA, LDS-staged T blocks, one workgroup per 16 my x 4
//                    bins x 256 mx
//   k_sep_gemm_bf16  the same with BF16 operands (or hi + lo BF16 pairs) on
//                    16x16x32 BF16 MFMA, FP32 accumulation
// Families with fewer than 16 locations along y (e.g. one shared alpha factor,
// M_y = 1) give the contraction too few columns to fill its tiles; they are
// propagated by the general sweep instead (k_sep_expand writes their per-
// distribution parameters into the workspace).
#include <hip/hip_runtime.h>

#include "vup_device.hpp"
#include "vup_internal.hpp"

namespace vup {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct SepArgs {
  int n[2];
  double lo[2], hi[2];
  int M[2];
  double ns;
  const double* mu[2];
  const double* sigma[2];
  int B;
  int pitch;
  const uint16_t* binmap;
  // workspace
  float* A[2];     // A_x: [n_x + 32][ldA0], zero past n_x and past M_x; A_y: [n_y][M_y]
  int ldA0;        // M_x rounded up to a multiple of 256
  __bf16* At[2];   // A_x rounded to BF16, hi and lo = bf16(A - hi), transposed:
                   // [ldA0][ldt], zero past n_x (the BF16 contraction's operands)
  int ldt;         // n_x + 32 rounded up to a multiple of 8
  double* Zd[2];   // [M_d]
  int* win[2];     // [M_d][2]
  float* T;        // [n_x][B][M_y]
  double* G;       // [n_y + 1][M_y] prefix sums of A_y along y (FP64)
  const uint32_t* runs;  // run records of the model matrix (see vup.h)
  const int* rowptr;
  float* P;        // [M_x*M_y][B]
  double* Z;       // [M_x*M_y] or null
  int pvec;        // P rows can be written as float4 (B % 4 == 0, P 16-byte aligned)
};

// one block per (axis, m): column m of A_d, its sum and its window. A_x also
// gets its zero padding (32 rows past n_x, columns up to ldA0), so that the
// contractions read it without bounds checks.
__global__ __launch_bounds__(256) void k_axis_factors(SepArgs a) {
  const int d = blockIdx.y;
  const int m = blockIdx.x;
  const int ld = d == 0 ? a.ldA0 : a.M[1];
  const int n = a.n[d];
  const int rows = d == 0 ? n + 32 : n;
  if (m >= ld) return;
  float* col = a.A[d] + m;
  // axis x also writes its transposed BF16 rows (ldt >= rows entries)
  const int rowsw = d == 0 ? a.ldt : rows;
  __bf16* th = d == 0 ? a.At[0] + (long long)m * a.ldt : nullptr;
  __bf16* tl = d == 0 ? a.At[1] + (long long)m * a.ldt : nullptr;
  if (m >= a.M[d]) {
    for (int i = threadIdx.x; i < rowsw; i += 256) {
      if (i < rows) col[(long long)i * ld] = 0.0f;
      if (d == 0) {
        th[i] = (__bf16)0.0f;
        tl[i] = (__bf16)0.0f;
      }
    }
    return;
  }
  __shared__ double red[kWaves];
  const double mu = a.mu[d][m], sg = a.sigma[d][m];
  int jlo, jhi;
  const bool ok = axis_window(a.lo[d], a.hi[d], n, mu, sg, a.ns, jlo, jhi);
  const int me = (ok && jhi >= jlo) ? axis_scale_exp(a.lo[d], a.hi[d], n, jlo, jhi, mu, 1.0 / sg)
                                     : 0;
  double zp = 0.0;
  for (int i = threadIdx.x; i < rowsw; i += 256) {
    float v = 0.0f;
    if (ok && i < n && i >= jlo && i <= jhi)
      v = gauss_factor(cell_centre(a.lo[d], a.hi[d], n, i), mu, sg, scale_log(me));
    if (i < rows) {
      col[(long long)i * ld] = v;
      zp += (double)v;
    }
    if (d == 0) {
      const __bf16 h = (__bf16)v;
      th[i] = h;
      tl[i] = (__bf16)(v - (float)h);
    }
  }
  const double Z = block_sum(zp, red);
  if (threadIdx.x == 0) {
    a.Zd[d][m] = ok ? Z : __builtin_nan("");
    a.win[d][2 * m] = ok ? jlo : 0;
    a.win[d][2 * m + 1] = ok ? jhi : -1;
  }
}

// T[ix][b][my0 + lane]: one wave, one row ix, 64 consecutive my (lane = my).
// The row's bin codes are read 64 at a time (coalesced) and broadcast with
// readlane; all lanes work on the same cell, so the branch on the bin is
// uniform. Consecutive cells of one bin are summed in a register and the bin's
// LDS slot is updated once per run (slots never collide: lane = my).
__global__ __launch_bounds__(64) void k_sep_scatter(SepArgs a) {
  extern __shared__ float trow[];  // [B][64]
  const int ix = blockIdx.x;
  const int my0 = blockIdx.y * 64;
  const int lane = threadIdx.x;
  const int my = my0 + lane;
  const int B = a.B;
  for (int i = lane; i < B * 64; i += 64) trow[i] = 0.0f;
  // union of the windows of this tile's my (empty windows are (0, -1))
  int lo = 0x7fffffff, hi = -1;
  if (my < a.M[1]) {
    const int l = a.win[1][2 * my], h = a.win[1][2 * my + 1];
    if (h >= l) {
      lo = l;
      hi = h;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  __syncthreads();
  const uint16_t* row = a.binmap + (long long)ix * a.pitch;
  const int My = a.M[1];
  const float* Ay = a.A[1] + (my < My ? my : 0);
  const int none = 4 * B;
  int cur = none;
  double acc = 0.0;
  for (int iy0 = lo; iy0 <= hi; iy0 += 64) {
    const int mine = (iy0 + lane <= hi) ? (int)row[iy0 + lane] : none;
    const int cnt = (hi - iy0 + 1) < 64 ? (hi - iy0 + 1) : 64;
    for (int j0 = 0; j0 < cnt; j0 += 8) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        v[j] = (j0 + j < cnt && my < My) ? Ay[(long long)(iy0 + j0 + j) * My] : 0.0f;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (j0 + j < cnt) {
          const int code = __builtin_amdgcn_readlane(mine, j0 + j);
          if (code != cur) {
            if (cur < none) trow[(cur >> 2) * 64 + lane] += (float)acc;
            acc = 0.0;
            cur = code;
          }
          acc += (double)v[j];
        }
      }
    }
  }
  if (cur < none) trow[(cur >> 2) * 64 + lane] += (float)acc;
  __syncthreads();
  if (my < My) {
    float* Trow = a.T + (long long)ix * B * My;
    for (int b = 0; b < B; ++b) Trow[(long long)b * My + my] = trow[b * 64 + lane];
  }
}

// G[i][my] = sum_{iy < i} A_y[iy][my], i = 0..n_y, in FP64 from the FP32
// factors. One workgroup per my: thread t sums a contiguous stretch of y in
// order, an exclusive scan of the stretch totals (waves, then across waves in
// LDS) gives each stretch its start, and the thread writes its prefix sums.
__global__ __launch_bounds__(256) void k_axis_prefix(SepArgs a) {
  __shared__ double wtot[kWaves];
  const int my = blockIdx.x;
  const int ny = a.n[1], My = a.M[1];
  const int len = (ny + 255) / 256;
  const int i0 = threadIdx.x * len, i1 = min(ny, i0 + len);
  const float* Ay = a.A[1] + my;
  double s = 0.0;
  for (int i = i0; i < i1; ++i) s += (double)Ay[(long long)i * My];
  const double incl = wave_scan(s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 63) wtot[wave] = incl;
  __syncthreads();
  double run = incl - s;
  for (int w = 0; w < wave; ++w) run += wtot[w];
  double* Gm = a.G + my;
  for (int i = i0; i < i1; ++i) {
    Gm[(long long)i * My] = run;
    run += (double)Ay[(long long)i * My];
  }
  if (threadIdx.x == 255) Gm[(long long)ny * My] = run;
}

// T[ix][b][my] from the runs of equal bin along y: a run [s, e) of bin b adds
// G[e][my] - G[s][my] (the run's factor mass, zero outside the window). One
// workgroup per (row ix, 256 my), thread = my: the thread owns its T column,
// zeroes it and adds the row's runs in order (deterministic, no atomics; the
// row's T block stays in L2 between the zeroing and the adds). Runs go in
// batches of 8 whose repeated bins are merged first (the bins are the same
// for every thread), so the batch's reads of T are independent.
constexpr int kRunBatch = 8;

__global__ __launch_bounds__(256) void k_sep_runs(SepArgs a) {
  const int ix = blockIdx.x;
  const int my = blockIdx.y * 256 + threadIdx.x;
  const int My = a.M[1], B = a.B;
  if (my >= My) return;
  float* Trow = a.T + (long long)ix * B * My + my;
  for (int b = 0; b < B; ++b) Trow[(long long)b * My] = 0.0f;
  const int r0 = a.rowptr[ix], r1 = a.rowptr[ix + 1];  // last record: terminator
  const double* Gm = a.G + my;
  const uint32_t none = 4u * (uint32_t)B;
  for (int r = r0; r + 1 < r1; r += kRunBatch) {
    uint32_t rec[kRunBatch + 1];
    double g[kRunBatch + 1];
#pragma unroll
    for (int i = 0; i <= kRunBatch; ++i) {
      const int ri = min(r + i, r1 - 1);
      rec[i] = a.runs[ri];
      g[i] = Gm[(long long)(rec[i] & 0xFFFFu) * My];
    }
    int bi[kRunBatch];
    float d[kRunBatch];
#pragma unroll
    for (int i = 0; i < kRunBatch; ++i) {
      const uint32_t code = rec[i] >> 16;
      bi[i] = (r + i + 1 < r1 && code < none) ? (int)(code >> 2) : -1;
      d[i] = (float)(g[i + 1] - g[i]);
    }
    // merge repeated bins of the batch into their first occurrence
#pragma unroll
    for (int i = 1; i < kRunBatch; ++i) {
#pragma unroll
      for (int j = 0; j < i; ++j) {
        if (bi[i] >= 0 && bi[j] == bi[i]) {
          d[j] += d[i];
          bi[i] = -1;
        }
      }
    }
    float t[kRunBatch];
#pragma unroll
    for (int i = 0; i < kRunBatch; ++i) t[i] = bi[i] >= 0 ? Trow[(long long)bi[i] * My] : 0.0f;
#pragma unroll
    for (int i = 0; i < kRunBatch; ++i)
      if (bi[i] >= 0) Trow[(long long)bi[i] * My] = t[i] + d[i];
  }
}

// T[ix][b][my] from the runs, written once: one workgroup per (row ix, 256 my),
// thread = my. Wave 0 first sorts the row's runs by 32-bin tile into LDS
// (stable: run order kept inside a tile, using ballots per distinct tile of
// each 64-run chunk). Then, tile by tile, every thread accumulates its
// column of the tile's 32 bins in LDS (slots owned by the thread, runs in row
// order, batches of 8 runs whose G loads are issued together) and writes the
// 32 T entries once. Used for rows of at most kRunRowMax cells.
constexpr int kTileBins = 32;
constexpr int kRunRowMax = 4096;

__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
}

__global__ __launch_bounds__(256) void k_sep_runs_tiled(SepArgs a) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  const int B = a.B, My = a.M[1];
  const int ntiles = (B + kTileBins - 1) / kTileBins;
  float* acc = smem;                                          // [kTileBins][256]
  int* start = reinterpret_cast<int*>(acc + kTileBins * 256);  // [ntiles + 1]
  int* cur = start + (ntiles + 1);                             // [ntiles]
  uint32_t* lse = reinterpret_cast<uint32_t*>(cur + ntiles);   // [runs] s | e << 16
  uint16_t* lbin = reinterpret_cast<uint16_t*>(lse + (a.n[1] + 1));  // [runs]
  const int ix = blockIdx.x, tid = threadIdx.x;
  const int my = blockIdx.y * 256 + tid;
  const int r0 = a.rowptr[ix], r1 = a.rowptr[ix + 1];
  const int R = r1 - 1 - r0;  // runs of the row (the last record is the terminator)
  const uint32_t none = 4u * (uint32_t)B;
  for (int t = tid; t <= ntiles; t += 256) start[t] = 0;
  __syncthreads();
  if (tid < 64) {
    const int lane = tid;
    // pass 1: runs per tile; pass 2: stable placement
    for (int pass = 0; pass < 2; ++pass) {
      if (pass == 1) {
        if (lane == 0) {
          int run = 0;
          for (int t = 0; t < ntiles; ++t) {
            const int c = start[t + 1];
            start[t] = run;
            cur[t] = run;
            run += c;
          }
          start[ntiles] = run;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      for (int c0 = 0; c0 < R; c0 += 64) {
        const int r = c0 + lane;
        uint32_t rec = 0, nxt = 0;
        int tile = -1;
        if (r < R) {
          rec = a.runs[r0 + r];
          nxt = a.runs[r0 + r + 1];
          if ((rec >> 16) < none) tile = (int)((rec >> 16) >> 2) / kTileBins;
        }
        unsigned long long todo = __ballot(tile >= 0);
        while (todo) {
          const int first = __ffsll((long long)todo) - 1;
          const int t = __shfl(tile, first, 64);
          const unsigned long long m = __ballot(tile == t);
          if (pass == 0) {
            if (lane == 0) start[t + 1] += __popcll(m);
          } else {
            const int base = cur[t];
            if (tile == t) {
              const int pos = base + lanes_below(m);
              lse[pos] = (rec & 0xFFFFu) | ((nxt & 0xFFFFu) << 16);
              lbin[pos] = (uint16_t)((rec >> 16) >> 2);
            }
            if (lane == 0) cur[t] = base + __popcll(m);
          }
          todo &= ~m;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
    }
  }
  __syncthreads();
  if (my >= My) return;  // no barrier below
  const double* Gm = a.G + my;
  float* Tcol = a.T + (long long)ix * B * My + my;
  float* mine = acc + tid;
  for (int t = 0; t < ntiles; ++t) {
    const int bt = t * kTileBins;
#pragma unroll
    for (int q = 0; q < kTileBins; ++q) mine[q * 256] = 0.0f;
    const int st = start[t], en = start[t + 1];
    for (int k = st; k < en; k += 8) {
      double g0[8], g1[8];
      int bb[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int kk = min(k + i, en - 1);
        const uint32_t se = lse[kk];
        bb[i] = k + i < en ? (int)lbin[kk] - bt : -1;
        g0[i] = Gm[(long long)(se & 0xFFFFu) * My];
        g1[i] = Gm[(long long)(se >> 16) * My];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (bb[i] >= 0) mine[bb[i] * 256] += (float)(g1[i] - g0[i]);
    }
    const int nq = min(kTileBins, B - bt);
    for (int q = 0; q < nq; ++q) Tcol[(long long)(bt + q) * My] = mine[q * 256];
  }
}

static size_t runs_tiled_lds(int B, int ny) {
  const int ntiles = (B + kTileBins - 1) / kTileBins;
  return (size_t)kTileBins * 256 * 4 + (size_t)(2 * ntiles + 1) * 4 + (size_t)(ny + 1) * 4 +
         (size_t)(ny + 1) * 2;
}

// Banded contraction on the matrix cores: C_b[mx][my] = sum_ix A_x[ix][mx]
// T[ix][b][my]. A workgroup (4 waves) owns 16 my x NB bins and 256 mx (16 mx
// tiles; wave w takes tiles w, w+4, w+8, w+12, so the tiles inside the band
// of any ix chunk are spread over the four waves). The ix axis is walked in
// chunks of 16 over the union of the tiles' windows; each chunk's T block
// (16 ix x NB bins x 16 my) is staged in LDS, double buffered, with a row
// pitch of 16 NB + 16 floats so the 4 ix rows of one MFMA operand read hit
// distinct banks; A_x comes from L2 straight into registers, only for tiles
// whose window meets the chunk (the others skip their MFMAs: A_x is zero
// there). 16x16x4 FP32 MFMA lane layout: A[i][k] and B[k][j] from lane
// i + 16 k (resp. j + 16 k), D[4 q + r][j] in lane j + 16 q, slot r.
#ifndef VUP_SEP_BINS
#define VUP_SEP_BINS 4
#endif
constexpr int kSepBins = VUP_SEP_BINS;  // bins per workgroup of the contraction
// families with fewer locations along y go to the general sweep
constexpr int kSepMinMy = 16;

// A workgroup owns 16 my x NB bins (the column tile q is bin b0 + q, its 16
// columns the my).
template <int NB>
__global__ __launch_bounds__(256, 4) void k_sep_gemm(SepArgs a) {
  constexpr int kPitch = 16 * NB + 16;
  constexpr int kTile = 16 * kPitch;
  __shared__ __attribute__((aligned(16))) float Ts[2 * kTile];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int Mx = a.M[0], My = a.M[1], B = a.B, nx = a.n[0];
  const int my0 = blockIdx.x * 16;
  const int b0 = blockIdx.y * NB;
  const int mxb = blockIdx.z * 256;
  // windows of this wave's four tiles (uniform), and of the workgroup's 16
  int tlo[4], thi[4];
  int glo = 0x7fffffff, ghi = -1;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int mx = mxb + 16 * t + li;
    int lo = 0x7fffffff, hi = -1;
    if (mx < Mx) {
      const int l = a.win[0][2 * mx], h = a.win[0][2 * mx + 1];
      if (h >= l) {
        lo = l;
        hi = h;
      }
    }
    for (int o = 8; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    glo = min(glo, lo);
    ghi = max(ghi, hi);
    if ((t & 3) == w) {
      tlo[t >> 2] = lo;
      thi[t >> 2] = hi;
    }
  }
  f32x4 acc[4][NB];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[j][q] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
  if (ghi >= glo) {
    const bool vec = (My & 3) == 0;
    // staging: element e = threadIdx.x + 256 u -> (ix row, bin q, 4 my)
    auto load_t = [&](int ix0, float4 (&tv)[NB / 4]) {
#pragma unroll
      for (int u = 0; u < NB / 4; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int ix = ix0 + e / (4 * NB);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        const int b = b0 + (e >> 2) % NB, my = my0 + 4 * (e & 3);
        if (ix <= ghi && ix < nx && b < B) {
          const float* src = a.T + ((long long)ix * B + b) * My + my;
          if (vec && my + 3 < My) {
            v = *reinterpret_cast<const float4*>(src);
          } else {
            if (my < My) v.x = src[0];
            if (my + 1 < My) v.y = src[1];
            if (my + 2 < My) v.z = src[2];
            if (my + 3 < My) v.w = src[3];
          }
        }
        tv[u] = v;
      }
    };
    auto store_t = [&](int buf, const float4 (&tv)[NB / 4]) {
#pragma unroll
      for (int u = 0; u < NB / 4; ++u) {
        const int e = threadIdx.x + 256 * u;
        *reinterpret_cast<float4*>(&Ts[buf * kTile + (e / (4 * NB)) * kPitch +
                                       ((e >> 2) % NB) * 16 + 4 * (e & 3)]) = tv[u];
      }
    };
    // A_x is zero-padded: rows up to n_x + 15 and columns up to ldA0 exist
    const int ldA = a.ldA0;
    const float* Abase = a.A[0] + mxb + 16 * w + li + (long long)lk * ldA;
    auto live = [&](int j, int ix0) { return tlo[j] <= ix0 + 15 && thi[j] >= ix0; };
    auto load_a = [&](int ix0, float (&av)[4][4]) {
      const float* p = Abase + (long long)ix0 * ldA;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (live(j, ix0))
#pragma unroll
          for (int s = 0; s < 4; ++s) av[j][s] = p[64 * j + 4 * s * ldA];
    };
    const int c0 = glo >> 4, c1 = ghi >> 4;
    float4 tv[NB / 4];
    load_t(16 * c0, tv);
    store_t(0, tv);
    float av[4][4], an[4][4];
    load_a(16 * c0, av);
    __syncthreads();
    // one chunk: MFMAs from LDS buffer `buf` and A operands `cur`, while the
    // next chunk's T block and A operands are in flight
    auto step = [&](int c, int buf, float (&cur)[4][4], float (&nxt)[4][4]) {
      const int ix0 = 16 * c;
      const bool more = c < c1;
      if (more) {
        load_t(ix0 + 16, tv);
        load_a(ix0 + 16, nxt);
      }
      const float* Tb = Ts + buf * kTile;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (live(j, ix0)) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const float* row = Tb + (4 * s + lk) * kPitch + li;
#pragma unroll
            for (int q = 0; q < NB; ++q)
              acc[j][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[j][s], row[16 * q], acc[j][q],
                                                                0, 0, 0);
          }
        }
      }
      if (more) store_t(buf ^ 1, tv);
      __syncthreads();
    };
    for (int c = c0; c <= c1; c += 2) {
      step(c, 0, av, an);
      if (c + 1 <= c1) step(c + 1, 1, an, av);
    }
  }
  // D[4 lk + r][li] = C[tile mx + 4 lk + r][column li of tile q]; normalise and
  // store
  const int my = my0 + li;
  if (my >= My) return;
  const double zy = a.Zd[1][my];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mx = mxb + 16 * (4 * j + w) + 4 * lk + r;
      if (mx >= Mx) continue;
      const double z = a.Zd[0][mx] * zy;
      const double rz = 1.0 / z;
      const long long k = (long long)mx * My + my;
      float* dst = a.P + k * B + b0;
#pragma unroll
      for (int q4 = 0; q4 < NB / 4; ++q4) {
        float o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          o[q] = (z > 0.0) ? (float)((double)acc[j][4 * q4 + q][r] * rz)
                           : (z == 0.0 ? 0.0f : __builtin_nanf(""));
        if (a.pvec && b0 + 4 * q4 + 3 < B) {
          *reinterpret_cast<float4*>(dst + 4 * q4) = make_float4(o[0], o[1], o[2], o[3]);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (b0 + 4 * q4 + q < B) dst[4 * q4 + q] = o[q];
        }
      }
    }
  }
}

// The same contraction on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation): A_x and T rounded to BF16 (nearest even), or, with
// SPLIT, each written as hi + lo (hi = bf16(v), lo = bf16(v - hi)) and the
// product taken as hi hi + hi lo + lo hi (the dropped lo lo term is below
// 2^-16 of it). One MFMA covers 32 rows of ix: lane (li, g) holds rows
// ix0 + 8 g .. + 7 of A's column mx and of T's column my, the same rows in
// the same slots of both operands, so the sum over the chunk does not depend
// on how the instruction orders its k. T blocks are staged in LDS as BF16
// with ix contiguous ([bin][my][ix], row pitch 40), so a lane's eight values
// are one 16-byte read; A_x comes as the transposed BF16 copies that
// k_axis_factors writes (rows of ix, zero past n_x), also one 16-byte read.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int NB, bool SPLIT>
__global__ __launch_bounds__(256, 4) void k_sep_gemm_bf16(SepArgs a) {
  constexpr int kPB = 40;                 // BF16 per (bin, my) row: 32 ix + 8 pad
  constexpr int kTileB = NB * 16 * kPB;   // one chunk's T block (BF16 elements)
  constexpr int kParts = SPLIT ? 2 : 1;   // hi (and lo) blocks
  __shared__ __attribute__((aligned(16))) __bf16 Ts[2 * kParts * kTileB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int Mx = a.M[0], My = a.M[1], B = a.B, nx = a.n[0];
  const int my0 = blockIdx.x * 16;
  const int b0 = blockIdx.y * NB;
  const int mxb = blockIdx.z * 256;
  int tlo[4], thi[4];
  int glo = 0x7fffffff, ghi = -1;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int mx = mxb + 16 * t + li;
    int lo = 0x7fffffff, hi = -1;
    if (mx < Mx) {
      const int l = a.win[0][2 * mx], h = a.win[0][2 * mx + 1];
      if (h >= l) {
        lo = l;
        hi = h;
      }
    }
    for (int o = 8; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    glo = min(glo, lo);
    ghi = max(ghi, hi);
    if ((t & 3) == w) {
      tlo[t >> 2] = lo;
      thi[t >> 2] = hi;
    }
  }
  f32x4 acc[4][NB];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[j][q] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
  if (ghi >= glo) {
    const bool vec = (My & 3) == 0;
    // staging: element e = threadIdx.x + 256 u -> (ix row of the chunk, bin
    // q, four my); 32 rows x NB bins x 4 float4 = 128 NB float4 per chunk
    constexpr int kPer = NB / 2;
    auto load_t = [&](int ix0, float4 (&tv)[kPer]) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int ix = ix0 + e / (4 * NB);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        const int b = b0 + (e >> 2) % NB, my = my0 + 4 * (e & 3);
        if (ix <= ghi && ix < nx && b < B) {
          const float* src = a.T + ((long long)ix * B + b) * My + my;
          if (vec && my + 3 < My) {
            v = *reinterpret_cast<const float4*>(src);
          } else {
            if (my < My) v.x = src[0];
            if (my + 1 < My) v.y = src[1];
            if (my + 2 < My) v.z = src[2];
            if (my + 3 < My) v.w = src[3];
          }
        }
        tv[u] = v;
      }
    };
    auto store_t = [&](int buf, const float4 (&tv)[kPer]) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int r = e / (4 * NB), q = (e >> 2) % NB, m4 = 4 * (e & 3);
        __bf16* hi = Ts + (buf * kParts) * kTileB + (q * 16 + m4) * kPB + r;
        const float v[4] = {tv[u].x, tv[u].y, tv[u].z, tv[u].w};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const __bf16 h = (__bf16)v[m];
          hi[m * kPB] = h;
          if constexpr (SPLIT) hi[kTileB + m * kPB] = (__bf16)(v[m] - (float)h);
        }
      }
    };
    // A operands: row mx of the transposed BF16 copies, ix0 + 8 lg .. + 7 in
    // one 16-byte load (rows are zero past n_x up to ix n_x + 31)
    const long long ldt = a.ldt;
    const __bf16* Ah = a.At[0] + (long long)(mxb + 16 * w + li) * ldt + 8 * lg;
    const __bf16* Al = a.At[1] + (long long)(mxb + 16 * w + li) * ldt + 8 * lg;
    auto live = [&](int j, int ix0) { return tlo[j] <= ix0 + 31 && thi[j] >= ix0; };
    auto load_a = [&](int ix0, bf16x8 (&h)[4], bf16x8 (&l)[4]) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (live(j, ix0)) {
          h[j] = *reinterpret_cast<const bf16x8*>(Ah + 64 * j * ldt + ix0);
          if constexpr (SPLIT) l[j] = *reinterpret_cast<const bf16x8*>(Al + 64 * j * ldt + ix0);
        }
      }
    };
    const int c0 = glo >> 5, c1 = ghi >> 5;
    float4 tv[kPer];
    load_t(32 * c0, tv);
    store_t(0, tv);
    // BF16: the next chunk's A is loaded during the current MFMAs (ping-pong
    // registers); SPLIT holds twice the operands and loads each chunk's A at
    // its start instead, which keeps both variants within 128 VGPRs
    auto mfmas = [&](int ix0, int buf, const bf16x8 (&ch)[4], const bf16x8 (&cl)[4]) {
      const __bf16* Th = Ts + (buf * kParts) * kTileB + li * kPB + 8 * lg;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (live(j, ix0)) {
#pragma unroll
          for (int q = 0; q < NB; ++q) {
            const bf16x8 th = *reinterpret_cast<const bf16x8*>(Th + q * 16 * kPB);
            acc[j][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch[j], th, acc[j][q], 0, 0, 0);
            if constexpr (SPLIT) {
              const bf16x8 tl = *reinterpret_cast<const bf16x8*>(Th + kTileB + q * 16 * kPB);
              acc[j][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ch[j], tl, acc[j][q], 0, 0, 0);
              acc[j][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cl[j], th, acc[j][q], 0, 0, 0);
            }
          }
        }
      }
    };
    if constexpr (SPLIT) {
      // twice the operands: each chunk's A is loaded at its start
      bf16x8 h[4], l[4];
      __syncthreads();
      for (int c = c0, buf = 0; c <= c1; ++c, buf ^= 1) {
        const int ix0 = 32 * c;
        const bool more = c < c1;
        if (more) load_t(ix0 + 32, tv);
        load_a(ix0, h, l);
        mfmas(ix0, buf, h, l);
        if (more) store_t(buf ^ 1, tv);
        __syncthreads();
      }
    } else {
      // the next chunk's A is loaded during the current MFMAs (ping-pong)
      bf16x8 ha[4], hb[4], unused[4];
      load_a(32 * c0, ha, unused);
      __syncthreads();
      auto step = [&](int c, int buf, bf16x8 (&ch)[4], bf16x8 (&nh)[4]) {
        const int ix0 = 32 * c;
        const bool more = c < c1;
        if (more) {
          load_t(ix0 + 32, tv);
          load_a(ix0 + 32, nh, unused);
        }
        mfmas(ix0, buf, ch, unused);
        if (more) store_t(buf ^ 1, tv);
        __syncthreads();
      };
      for (int c = c0; c <= c1; c += 2) {
        step(c, 0, ha, hb);
        if (c + 1 <= c1) step(c + 1, 1, hb, ha);
      }
    }
  }
  const int my = my0 + li;
  if (my >= My) return;
  const double zy = a.Zd[1][my];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mx = mxb + 16 * (4 * j + w) + 4 * lg + r;
      if (mx >= Mx) continue;
      const double z = a.Zd[0][mx] * zy;
      const double rz = 1.0 / z;
      const long long k = (long long)mx * My + my;
      float* dst = a.P + k * B + b0;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const float o = (z > 0.0) ? (float)((double)acc[j][q][r] * rz)
                                  : (z == 0.0 ? 0.0f : __builtin_nanf(""));
        if (b0 + q < B) dst[q] = o;
      }
    }
  }
}

// Z[k] for k = mx M_y + my: the product of the two axes' factor sums, times
// 2^-(m_x + m_y) to undo the columns' scaling (k_axis_factors), so that Z is
// the mass of the truncated densities themselves
__global__ __launch_bounds__(256) void k_sep_z(SepArgs a) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long K = (long long)a.M[0] * a.M[1];
  if (k >= K) return;
  const int m[2] = {(int)(k / a.M[1]), (int)(k % a.M[1])};
  double z = 1.0;
  int ms = 0;
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    z *= a.Zd[d][m[d]];
    const int jlo = a.win[d][2 * m[d]], jhi = a.win[d][2 * m[d] + 1];
    if (jhi >= jlo)
      ms += axis_scale_exp(a.lo[d], a.hi[d], a.n[d], jlo, jhi, a.mu[d][m[d]],
                           1.0 / a.sigma[d][m[d]]);
  }
  a.Z[k] = ldexp(z, -ms);
}

// per-distribution parameters of a family propagated by the general sweep:
// mu[k][0][d], sigma[k][0][d] for k = mx M_y + my
__global__ __launch_bounds__(256) void k_sep_expand(int Mx, int My, const double* mux,
                                                    const double* muy, const double* sgx,
                                                    const double* sgy, double* mu, double* sg) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= (long long)Mx * My) return;
  const int mx = (int)(k / My), my = (int)(k % My);
  mu[2 * k] = mux[mx];
  mu[2 * k + 1] = muy[my];
  sg[2 * k] = sgx[mx];
  sg[2 * k + 1] = sgy[my];
}

size_t sep_workspace_bytes(const vup_grid& g, int B, int Mx, int My) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  if (My < kSepMinMy) return 2 * al((size_t)Mx * My * 2 * sizeof(double));
  size_t o = 0;
  const size_t ld0 = ((size_t)Mx + 255) / 256 * 256;
  o += al(((size_t)g.n[0] + 32) * ld0 * 4);
  o += al((size_t)g.n[1] * My * 4);
  o += al((size_t)Mx * 8) + al((size_t)My * 8);
  o += al((size_t)Mx * 8) + al((size_t)My * 8);
  o += al((size_t)g.n[0] * B * My * 4);
  o += al((size_t)(g.n[1] + 1) * My * 8);
  const size_t ldt = ((size_t)g.n[0] + 32 + 7) / 8 * 8;
  o += 2 * al(ld0 * ldt * 2);
  return o;
}

hipError_t launch_separable(const vup_mm& mm, int Mx, int My, const double* mu_x,
                            const double* mu_y, const double* sg_x, const double* sg_y,
                            double ns, int prec, void* ws, float* P, double* Z, hipStream_t s) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  if (My < kSepMinMy) {
    const long long K = (long long)Mx * My;
    double* mu = static_cast<double*>(ws);
    double* sg = reinterpret_cast<double*>(static_cast<char*>(ws) + al((size_t)K * 16));
    hipLaunchKernelGGL(k_sep_expand, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, Mx, My,
                       mu_x, mu_y, sg_x, sg_y, mu, sg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    vup_dists d{};
    d.K = K;
    d.ncomp = 1;
    d.ndim = 2;
    d.n_sigma = ns;
    d.mu = mu;
    d.sigma = sg;
    d.weight = nullptr;
    return launch_propagate(mm, d, VUP_FP32, P, Z, s);
  }
  SepArgs a{};
  for (int d = 0; d < 2; ++d) {
    a.n[d] = mm.grid.n[d];
    a.lo[d] = mm.grid.lo[d];
    a.hi[d] = mm.grid.hi[d];
  }
  a.M[0] = Mx;
  a.M[1] = My;
  a.ns = ns;
  a.mu[0] = mu_x;
  a.mu[1] = mu_y;
  a.sigma[0] = sg_x;
  a.sigma[1] = sg_y;
  a.B = mm.B;
  a.pitch = mm.pitch;
  a.binmap = reinterpret_cast<const uint16_t*>(static_cast<const char*>(mm.ws) + mm.off_binmap);
  char* w = static_cast<char*>(ws);
  a.ldA0 = (Mx + 255) / 256 * 256;
  a.A[0] = reinterpret_cast<float*>(w);
  w += al(((size_t)a.n[0] + 32) * a.ldA0 * 4);
  a.A[1] = reinterpret_cast<float*>(w);
  w += al((size_t)a.n[1] * My * 4);
  a.Zd[0] = reinterpret_cast<double*>(w);
  w += al((size_t)Mx * 8);
  a.Zd[1] = reinterpret_cast<double*>(w);
  w += al((size_t)My * 8);
  a.win[0] = reinterpret_cast<int*>(w);
  w += al((size_t)Mx * 8);
  a.win[1] = reinterpret_cast<int*>(w);
  w += al((size_t)My * 8);
  a.T = reinterpret_cast<float*>(w);
  w += al((size_t)a.n[0] * mm.B * My * 4);
  a.G = reinterpret_cast<double*>(w);
  w += al(((size_t)a.n[1] + 1) * My * 8);
  a.ldt = (a.n[0] + 32 + 7) / 8 * 8;
  a.At[0] = reinterpret_cast<__bf16*>(w);
  w += al((size_t)a.ldA0 * a.ldt * 2);
  a.At[1] = reinterpret_cast<__bf16*>(w);
  a.runs = reinterpret_cast<const uint32_t*>(static_cast<const char*>(mm.ws) + mm.off_runs);
  a.rowptr = reinterpret_cast<const int*>(static_cast<const char*>(mm.ws) + mm.off_rowptr);
  a.P = P;
  a.Z = Z;
  a.pvec = (mm.B % 4 == 0) && ((reinterpret_cast<uintptr_t>(P) & 15u) == 0);
  const int Mmax = a.ldA0 > My ? a.ldA0 : My;
  hipLaunchKernelGGL(k_axis_factors, dim3(Mmax, 2), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (Z) {
    const long long K = (long long)Mx * My;
    hipLaunchKernelGGL(k_sep_z, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.n[1] <= 65534) {
    // run records hold 16-bit columns: T from the runs and the y prefix sums
    hipLaunchKernelGGL(k_axis_prefix, dim3(My), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.n[1] <= kRunRowMax) {
      const size_t lds = runs_tiled_lds(mm.B, a.n[1]);
      if (lds > 65536) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_sep_runs_tiled),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
      }
      hipLaunchKernelGGL(k_sep_runs_tiled, dim3(a.n[0], (My + 255) / 256), dim3(256), lds, s, a);
    } else {
      hipLaunchKernelGGL(k_sep_runs, dim3(a.n[0], (My + 255) / 256), dim3(256), 0, s, a);
    }
  } else {
    const size_t lds = (size_t)mm.B * 64 * 4;
    if (lds > 65536) {
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_sep_scatter),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_sep_scatter, dim3(a.n[0], (My + 63) / 64), dim3(64), lds, s, a);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int NB = kSepBins;
  const dim3 grid((My + 15) / 16, (mm.B + NB - 1) / NB, (Mx + 255) / 256);
  // the BF16 contraction takes two bins per workgroup (its operand registers
  // then fit the 128-VGPR budget of four waves per SIMD)
  constexpr int NBH = 2;
  const dim3 gridh((My + 15) / 16, (mm.B + NBH - 1) / NBH, (Mx + 255) / 256);
  if (prec == VUP_BF16)
    hipLaunchKernelGGL((k_sep_gemm_bf16<NBH, false>), gridh, dim3(256), 0, s, a);
  else if (prec == VUP_BF16X2)
    hipLaunchKernelGGL((k_sep_gemm_bf16<NBH, true>), gridh, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_sep_gemm<NB>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace vup
