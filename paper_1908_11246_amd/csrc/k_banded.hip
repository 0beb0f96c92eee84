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
//   k_axis_factors   A_d, Zd = sum_i A_d[i][m] (FP64), window bounds
//   k_sep_scatter    T, one wave per (ix, 64 consecutive my), conflict-free
//                    LDS accumulation (lane = my), cells in increasing iy,
//                    same-bin runs summed in registers
//   k_sep_mfma       one wave per (16 mx, 16 my, 16 bins): 16x16x4 FP32 MFMA
//                    over the union of the 16 mx windows
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
  float* A[2];     // [n_d][M_d]
  double* Zd[2];   // [M_d]
  int* win[2];     // [M_d][2]
  float* T;        // [n_x][B][M_y]
  float* P;        // [M_x*M_y][B]
  double* Z;       // [M_x*M_y] or null
};

// one block per (axis, m): column m of A_d, its sum and its window
__global__ __launch_bounds__(256) void k_axis_factors(SepArgs a) {
  const int d = blockIdx.y;
  const int m = blockIdx.x;
  if (m >= a.M[d]) return;
  __shared__ double red[kWaves];
  const int n = a.n[d];
  const double mu = a.mu[d][m], sg = a.sigma[d][m];
  int jlo, jhi;
  const bool ok = axis_window(a.lo[d], a.hi[d], n, mu, sg, a.ns, jlo, jhi);
  double zp = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    float v = 0.0f;
    if (ok && i >= jlo && i <= jhi) v = gauss_factor(cell_centre(a.lo[d], a.hi[d], n, i), mu, sg);
    a.A[d][(long long)i * a.M[d] + m] = v;
    zp += (double)v;
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
  float acc = 0.0f;
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
            if (cur < none) trow[(cur >> 2) * 64 + lane] += acc;
            acc = 0.0f;
            cur = code;
          }
          acc += v[j];
        }
      }
    }
  }
  if (cur < none) trow[(cur >> 2) * 64 + lane] += acc;
  __syncthreads();
  if (my < My) {
    float* Trow = a.T + (long long)ix * B * My;
    for (int b = 0; b < B; ++b) Trow[(long long)b * My + my] = trow[b * 64 + lane];
  }
}

// C[mx][my] for 16 bins at once: A operand = A_x^T tile (16 mx x 4 ix),
// B operand = T tile (4 ix x 16 my), 16x16x4 FP32 MFMA, K = the union of the
// tile's mx windows. Lane layout of v_mfma_f32_16x16x4f32: A[i][k] from lane
// i + 16k, B[k][j] from lane j + 16k, D[4q + r][j] in lane j + 16q, slot r.
__global__ __launch_bounds__(64) void k_sep_mfma(SepArgs a) {
  const int mx0 = blockIdx.x * 16;
  const int my0 = blockIdx.y * 16;
  const int b0 = blockIdx.z * 16;
  const int lane = threadIdx.x;
  const int Mx = a.M[0], My = a.M[1], B = a.B, nx = a.n[0];
  const int li = lane & 15, lk = lane >> 4;
  // union of the 16 mx windows
  int lo = 0x7fffffff, hi = -1;
  {
    const int mx = mx0 + li;
    if (mx < Mx) {
      const int l = a.win[0][2 * mx], h = a.win[0][2 * mx + 1];
      if (h >= l) {
        lo = l;
        hi = h;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
  }
  f32x4 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
  const int mxa = mx0 + li;  // A row handled by this lane
  const int myb = my0 + li;  // B column handled by this lane
  for (int k0 = lo; k0 <= hi; k0 += 4) {
    const int ix = k0 + lk;
    const bool inx = ix <= hi && ix < nx;
    const float av = (inx && mxa < Mx) ? a.A[0][(long long)ix * Mx + mxa] : 0.0f;
    const float* Tr = a.T + (long long)(inx ? ix : 0) * B * My;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int b = b0 + q;
      const float bv = (inx && myb < My && b < B) ? Tr[(long long)b * My + myb] : 0.0f;
      acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[q], 0, 0, 0);
    }
  }
  // D[4 lk + r][li] = C[mx0 + 4 lk + r][my0 + li]
  const int my = my0 + li;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int mx = mx0 + 4 * lk + r;
    if (mx >= Mx || my >= My) continue;
    const double zx = a.Zd[0][mx], zy = a.Zd[1][my];
    const double z = zx * zy;
    const long long k = (long long)mx * My + my;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int b = b0 + q;
      if (b >= B) continue;
      const double v = (double)acc[q][r];
      a.P[k * B + b] = (z > 0.0) ? (float)(v / z) : (z == 0.0 ? 0.0f : __builtin_nanf(""));
    }
    if (a.Z && blockIdx.z == 0) a.Z[k] = z;
  }
}

size_t sep_workspace_bytes(const vup_grid& g, int B, int Mx, int My) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t o = 0;
  o += al((size_t)g.n[0] * Mx * 4);
  o += al((size_t)g.n[1] * My * 4);
  o += al((size_t)Mx * 8) + al((size_t)My * 8);
  o += al((size_t)Mx * 8) + al((size_t)My * 8);
  o += al((size_t)g.n[0] * B * My * 4);
  return o;
}

hipError_t launch_separable(const vup_mm& mm, int Mx, int My, const double* mu_x,
                            const double* mu_y, const double* sg_x, const double* sg_y,
                            double ns, void* ws, float* P, double* Z, hipStream_t s) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
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
  a.A[0] = reinterpret_cast<float*>(w);
  w += al((size_t)a.n[0] * Mx * 4);
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
  a.P = P;
  a.Z = Z;
  const int Mmax = Mx > My ? Mx : My;
  hipLaunchKernelGGL(k_axis_factors, dim3(Mmax, 2), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)mm.B * 64 * 4;
  if (lds > 65536) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_sep_scatter),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sep_scatter, dim3(a.n[0], (My + 63) / 64), dim3(64), lds, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sep_mfma, dim3((Mx + 15) / 16, (My + 15) / 16, (mm.B + 15) / 16), dim3(64),
                     0, s, a);
  return hipGetLastError();
}

}  // namespace vup
