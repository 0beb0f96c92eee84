// Exact-f moments (eq. UP) of single-component pdfs on 2-D grids by tiles of
// the model values on the int8 matrix cores.
//
// A separable density is gx(i) gy(j) on cell (i, j), so its moment sums over
// one 64 x 64 tile T of the grid are bilinear forms in the model values:
//   S1_T = sum_ij gx(i) (f_ij - a_T) gy(j),
//   S2_T = sum_ij gx(i) (f_ij - a_T)^2 gy(j),
// a_T an anchor of the tile (the midpoint of its model values). The inner
// sums over j are matrix products of the tile's values with the column
// factors of the pdfs whose windows meet the tile; they are formed exactly
// from fixed-point operands (see k_mt_main), so the only errors are those of
// the operands' quantisation. Exactness matters because the variance is a
// difference: an error e in S2_T or e_1 in S1_T moves Var Z by about
// e + 2 (a_T - mean) e_1, and rounded sums (FP32 accumulation) carry errors
// relative to sum g (f - a_T)^2 ~ Z (a_T - mean)^2, which exceeds Z Var by up
// to (tile range / window spread)^2: FP32 accumulation measured variance
// errors of up to 27 times the 1e-5 relative bar on a coarse grid. With s the
// pdf's shift (the model value at its window's centre cell), delta = a_T - s
// and Z_T the tile's factor sum,
//   sum_T g (f - s)   = S1_T + delta Z_T,
//   sum_T g (f - s)^2 = S2_T + 2 delta S1_T + delta^2 Z_T     (FP64),
// and each tile's contribution is added to the pdf's totals as a 64-bit
// fixed-point integer: a power-of-two scale per pdf from Z and a bound of
// |f - s| over the tiles its window meets keeps every partial total below
// 2^60, and integer additions make the result independent of their order.
//
// The factors are exp(-t^2/2) = exp2(-(c t)^2), c = sqrt(log2(e)/2), with
// c t = c (x_lo - mu)/sigma + j c h/sigma for the j-th cell of the window: two
// FP32 constants per axis and pdf (rounded from FP64 once), one FMA, one
// multiply-add and v_exp_f32 per factor, the same instructions wherever a
// factor is formed, so the normaliser Z (the FP64 sum of the factors) and the
// tiles use identical values. Each axis's factors are divided by that axis's
// largest one, exp2(-(c t*)^2) at the cell t* nearest the mean (the moments
// do not change when an axis's factors are scaled alike): the largest factor
// is 1, so a window far from its mean (a one-cell window of a narrow pdf)
// neither underflows FP32 nor falls below the factors' fixed-point quantum.

#include <math.h>

#include "vup_device.hpp"
#include "vup_internal.hpp"

namespace vup {

namespace {

constexpr int kMT = 64;               // tile edge in cells
constexpr int kMTMaxTiles = 65535;    // tiles per axis (16-bit tile indices)
constexpr int kRing = 512;            // candidate ring: < 256 pending + one scan step of 256
constexpr double kC = 0.8493218002880191;  // sqrt(log2(e) / 2)

struct MTRec {
  float t0[2];    // c (x_lo - mu) / sigma per axis, x_lo the window's first cell
  float dt[2];    // c h / sigma per axis
  float tm2[2];   // (c t*)^2 per axis, t* the window's cell nearest the mean
  int lo[2];      // window (hi < lo: empty)
  int hi[2];
  double shift;   // model value at the window's centre cell
  double Z;       // product of the per-axis factor sums
  double sc1;     // fixed-point scales of sum g (f - s) and sum g (f - s)^2
  double sc2;
  int flags;      // 1 bad parameters, 2 empty window, 4 non-finite f in the window
  int pad;
};
static_assert(sizeof(MTRec) == 80, "record layout");

struct MTTile {
  double a;       // anchor: midpoint of the tile's finite model values
  double fmin, fmax;
  int nonfinite;  // the tile holds a non-finite model value
  int nfinite;    // finite cells
};
static_assert(sizeof(MTTile) == 32, "tile layout");

struct MTArgs {
  int n0, n1;           // cells along axis 0 (rows) and axis 1 (columns)
  double lo[2], hi[2];
  long long rowstride;  // elements per row of the padded FP32 model copy
  const float* __restrict__ f32;
  long long K;
  double ns;
  const double* __restrict__ mu;
  const double* __restrict__ sigma;
  int ntx, nty, parts;
  MTRec* rec;
  unsigned long long* bbox;  // tile range of each window: tx_lo, tx_hi, ty_lo, ty_hi (16 bits each)
  unsigned long long* acc;  // [K][2] fixed-point totals
  MTTile* tiles;
  double* mean;
  double* var;
  double* delta2;
  vup_model model;
  int has_model;
};

// model value of cell (row, col) from the anchored FP32 copy (columns 8m
// hold f, the seven after each their offset from it, or their own value when
// the anchor is not finite), in FP64
__device__ __forceinline__ double mt_f(const MTArgs& a, int row, int col) {
  const float* p = a.f32 + (long long)row * a.rowstride;
  const int c0 = col & ~7;
  const double f0 = (double)p[c0];
  if (col == c0) return f0;
  return isfinite(f0) ? f0 + (double)p[col] : (double)p[col];
}

// Gaussian factor of the j-th cell of a window, relative to the axis's
// largest (see the header comment)
__device__ __forceinline__ float mt_factor(int j, float t0, float dt, float tm2) {
  const float t = __builtin_fmaf((float)j, dt, t0);
  return __builtin_amdgcn_exp2f(-__builtin_fmaf(t, t, -tm2));
}

// (c t*)^2 for the cell of a window of W cells nearest the mean, with the
// factor's own rounding of c t
__device__ __forceinline__ float mt_tmin2(float t0, float dt, int W) {
  int j = (int)__builtin_rintf(-t0 / dt);
  j = j < 0 ? 0 : (j > W - 1 ? W - 1 : j);
  const float t = __builtin_fmaf((float)j, dt, t0);
  return t * t;
}

// column factors as integers of 30 bits, G = rint(g 2^30) (g <= 1); the
// normaliser and the tiles use the same
__device__ __forceinline__ int mt_quant(float g) {
  return (int)__builtin_rintf(g * 1073741824.0f);  // 2^30
}

__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------------------
// per tile: range and anchor of the model values
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mt_tiles(MTArgs a) {
  __shared__ double smin[4], smax[4];
  __shared__ int sbad[4], scnt[4];
  const int tx = blockIdx.x % a.ntx, ty = blockIdx.x / a.ntx;
  const int r0 = ty * kMT, c0 = tx * kMT;
  double mn = INFINITY, mx = -INFINITY;
  int bad = 0, cnt = 0;
  for (int e = threadIdx.x; e < kMT * kMT; e += 256) {
    const int row = r0 + (e >> 6), col = c0 + (e & 63);
    if (row < a.n0 && col < a.n1) {
      const double f = mt_f(a, row, col);
      if (isfinite(f)) {
        mn = fmin(mn, f);
        mx = fmax(mx, f);
        ++cnt;
      } else {
        bad = 1;
      }
    }
  }
  mn = wave_min_f64(mn);
  mx = wave_max_f64(mx);
  bad = __any(bad) ? 1 : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smin[w] = mn;
    smax[w] = mx;
    sbad[w] = bad;
    scnt[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    MTTile t;
    t.fmin = fmin(fmin(smin[0], smin[1]), fmin(smin[2], smin[3]));
    t.fmax = fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
    t.nonfinite = sbad[0] | sbad[1] | sbad[2] | sbad[3];
    t.nfinite = scnt[0] + scnt[1] + scnt[2] + scnt[3];
    t.a = t.nfinite ? 0.5 * t.fmin + 0.5 * t.fmax : 0.0;
    if (!t.nfinite) t.fmin = t.fmax = 0.0;
    a.tiles[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// per pdf (16 lanes each): window, factor constants, normaliser, shift,
// fixed-point scales; clears the totals
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sum16(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
  return v;
}
__device__ __forceinline__ double max16(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 16));
  return v;
}

__global__ __launch_bounds__(256) void k_mt_prep(MTArgs a) {
  const int l16 = threadIdx.x & 15;
  const long long k = (long long)blockIdx.x * 16 + (threadIdx.x >> 4);
  if (k >= a.K) return;  // the 16 lanes of a pdf leave together
  MTRec r;
  r.pad = 0;
  r.shift = r.Z = 0.0;
  r.sc1 = r.sc2 = 1.0;
  int lo0, hi0, lo1, hi1;
  const double mu0 = a.mu[2 * k], mu1 = a.mu[2 * k + 1];
  const double s0 = a.sigma[2 * k], s1 = a.sigma[2 * k + 1];
  const bool ok0 = axis_window(a.lo[0], a.hi[0], a.n0, mu0, s0, a.ns, lo0, hi0);
  const bool ok1 = axis_window(a.lo[1], a.hi[1], a.n1, mu1, s1, a.ns, lo1, hi1);
  r.flags = (!ok0 || !ok1) ? 1 : ((hi0 < lo0 || hi1 < lo1) ? 2 : 0);
  r.lo[0] = lo0;
  r.hi[0] = hi0;
  r.lo[1] = lo1;
  r.hi[1] = hi1;
  r.t0[0] = r.t0[1] = r.dt[0] = r.dt[1] = r.tm2[0] = r.tm2[1] = 0.0f;
  unsigned long long bb = 1ull;  // tx_lo = 1 > tx_hi = 0: meets no tile
  if (r.flags == 0) {
    const double rs0 = 1.0 / s0, rs1 = 1.0 / s1;
    const double h0 = (a.hi[0] - a.lo[0]) / a.n0, h1 = (a.hi[1] - a.lo[1]) / a.n1;
    r.t0[0] = (float)((cell_centre(a.lo[0], a.hi[0], a.n0, lo0) - mu0) * rs0 * kC);
    r.t0[1] = (float)((cell_centre(a.lo[1], a.hi[1], a.n1, lo1) - mu1) * rs1 * kC);
    r.dt[0] = (float)(h0 * rs0 * kC);
    r.dt[1] = (float)(h1 * rs1 * kC);
    double zx = 0.0, zy = 0.0;
    r.tm2[0] = mt_tmin2(r.t0[0], r.dt[0], hi0 - lo0 + 1);
    r.tm2[1] = mt_tmin2(r.t0[1], r.dt[1], hi1 - lo1 + 1);
    for (int j = l16; j <= hi0 - lo0; j += 16)
      zx += (double)mt_factor(j, r.t0[0], r.dt[0], r.tm2[0]);
    for (int j = l16; j <= hi1 - lo1; j += 16)
      zy += (double)mt_quant(mt_factor(j, r.t0[1], r.dt[1], r.tm2[1]));
    r.Z = sum16(zx) * (sum16(zy) * 0x1p-30);
    double s = mt_f(a, lo0 + (hi0 - lo0 + 1) / 2, lo1 + (hi1 - lo1 + 1) / 2);
    if (!isfinite(s)) s = 0.0;  // the window holds a non-finite value: NaN result
    r.shift = s;
    // bound of |f - s| over the tiles the window meets
    const int tx0 = lo1 / kMT, tx1 = hi1 / kMT, ty0 = lo0 / kMT, ty1 = hi0 / kMT;
    const int ntw = tx1 - tx0 + 1, nt = ntw * (ty1 - ty0 + 1);
    double R = 0.0;
    for (int t = l16; t < nt; t += 16) {
      const MTTile T = a.tiles[(long long)(ty0 + t / ntw) * a.ntx + tx0 + t % ntw];
      if (T.nfinite) R = fmax(R, fmax(T.fmax - s, s - T.fmin));
    }
    R = max16(R);
    if (r.Z > 0.0 && R > 0.0 && isfinite(R)) {
      // Z < 2^(ez+1), R < 2^(er+1): |sum g (f-s)| < 2^(ez+er+2) and
      // sum g (f-s)^2 < 2^(ez+2er+3); the scales bring both below 2^60
      const int ez = ilogb(r.Z), er = ilogb(R);
      r.sc1 = ldexp(1.0, min(60 - (ez + er + 2), 1000));
      r.sc2 = ldexp(1.0, min(60 - (ez + 2 * er + 3), 1000));
    }
    bb = (unsigned long long)tx0 | ((unsigned long long)tx1 << 16) |
         ((unsigned long long)ty0 << 32) | ((unsigned long long)ty1 << 48);
  }
  if (l16 == 0) {
    a.rec[k] = r;
    a.bbox[k] = bb;
    a.acc[2 * k] = 0ull;
    a.acc[2 * k + 1] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// per (tile, part of the pdf list): the tile's sums of every pdf of the part
// whose window meets it, by exact integer products on the int8 matrix cores.
// The tile's F' = f - a_T and F'^2 are fixed-point integers of 30 bits
// (scales 2^eF, 2^eS from the tile's range R = max |F'|), the column factors
// integers G = rint(g 2^30); each is written as four balanced base-256
// digits in [-128, 127] (the bytes of (x + 0x80808080) xor 0x80808080). A
// digit pair (a, b) contributes 2^(8(a+b)) sum_j dF_a(j) dG_b(j);
// v_mfma_i32_16x16x64_i8 forms each such sum over the tile's 64 columns
// exactly (|terms| <= 2^14, 64 of them, at most four pairs per weight in one
// int32 accumulator: at most 2^22). The pairs of weight below 2^16 (a + b < 2)
// are left out: together below 2^(eF - 1) per row sum, under the
// quantisation of F' itself. The five accumulators per row are combined in
// FP64 and weighted by the row factors. So the sums are those of the
// quantised model values (within R 2^-31 of f - a_T), of their squares
// (within R^2 2^-31) and of the factors (within 2^-31), up to FP64 rounding,
// with no error from the order or length of the accumulation (an FP32
// accumulation would carry errors relative to sum g F'^2, amplified in the
// variance by (a_T - mean)^2 / Var). F' and F'^2 are quantised separately,
// so sum g F'^2 is not exactly the sum of the quantised F' squared: the
// difference, at most about 2 |F'| R 2^-31 <= R^2 2^-30 per unit weight,
// sets the 30 bits (26 left variance errors of R^2 2^-26, above the
// 1e-9 range^2 floor of the parity bar, on windows of one or two cells).
// The tile's digits are staged in LDS once; the workgroup scans the part for
// pdfs whose windows meet the tile, 256 at a time into a ring, and each wave
// takes 16 of them at once over all 64 rows: lane (li, g) forms the column
// factors of pdf li for columns 16g .. 16g + 15 in registers (the B operand)
// and the row factors of the rows its results belong to; the sums over the
// tile stay inside the wave.
// ---------------------------------------------------------------------------
// LDS bytes per tile row of one digit plane; the row's four 16-byte chunks
// are stored in the order chunk xor (row / 4) mod 4, so that the eight rows
// one 16-byte read serves at a time fall on distinct banks
constexpr int kDPitch = 64;
constexpr int kFBits = 30;    // fixed-point bits of F', F'^2 and the factors
constexpr int kDig = 4;       // their base-256 digits

typedef int mt_i32x4 __attribute__((ext_vector_type(4)));

// the four balanced base-256 digits of x (|x| < 0x7F7F7F7F), as the bytes of
// one word: x + sum 128 256^b has the digits plus 128 as its bytes
__device__ __forceinline__ uint32_t digits4(int x) {
  return ((uint32_t)x + 0x80808080u) ^ 0x80808080u;
}

// byte b of words w0..w3 -> word b (a 4 x 4 byte transpose, v_perm_b32)
__device__ __forceinline__ void transpose4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                           uint32_t (&o)[4]) {
  const uint32_t a_lo = __builtin_amdgcn_perm(w1, w0, 0x05010400u);  // w0.0 w1.0 w0.1 w1.1
  const uint32_t a_hi = __builtin_amdgcn_perm(w1, w0, 0x07030602u);  // w0.2 w1.2 w0.3 w1.3
  const uint32_t b_lo = __builtin_amdgcn_perm(w3, w2, 0x05010400u);
  const uint32_t b_hi = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
  o[0] = __builtin_amdgcn_perm(b_lo, a_lo, 0x05040100u);
  o[1] = __builtin_amdgcn_perm(b_lo, a_lo, 0x07060302u);
  o[2] = __builtin_amdgcn_perm(b_hi, a_hi, 0x05040100u);
  o[3] = __builtin_amdgcn_perm(b_hi, a_hi, 0x07060302u);
}

// four workgroups per CU: 128 VGPRs, 34 KB of LDS
__global__ __launch_bounds__(256, 4) void k_mt_main(MTArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t Dg[2 * kDig][kMT * kDPitch];  // digit planes: F', then F'^2
  __shared__ uint16_t ring[kRing];
  __shared__ int wcnt[4];
  __shared__ unsigned long long nfmask[kMT];

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int part = blockIdx.x % a.parts, tile = blockIdx.x / a.parts;
  const int tx = tile % a.ntx, ty = tile / a.ntx;
  const int r0 = ty * kMT, c0 = tx * kMT;
  const MTTile T = a.tiles[tile];
  const bool tbad = T.nonfinite != 0;  // uniform
  // fixed-point scales: rounding is monotonic, so every F' = f - a_T of the
  // tile (the same FP64 subtraction) is within R = max(fmax - a_T, a_T - fmin)
  // and F'^2 within R^2, both below 2^(ilogb + 1): |integers| <= 2^30
  const double R = fmax(T.fmax - T.a, T.a - T.fmin);
  const int eF = R > 0.0 ? ilogb(R) + 1 - kFBits : 0;
  const int eS = R > 0.0 ? ilogb(R * R) + 1 - kFBits : 0;
  if (threadIdx.x < kMT) nfmask[threadIdx.x] = 0ull;
  __syncthreads();
  // stage the digits: thread t writes 4 columns x 4 rows
  {
    const int cq = (threadIdx.x & 15) * 4;
    for (int rr = threadIdx.x >> 4; rr < kMT; rr += 16) {
      uint32_t hf[4], hs[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = r0 + rr, col = c0 + cq + u;
        int fi = 0, si = 0;
        if (row < a.n0 && col < a.n1) {
          const double f = mt_f(a, row, col);
          if (isfinite(f)) {
            const double v = f - T.a;
            fi = (int)rint(ldexp(v, -eF));
            si = (int)rint(ldexp(v * v, -eS));
          } else {
            atomicOr(&nfmask[rr], 1ull << (cq + u));
          }
        }
        hf[u] = digits4(fi);
        hs[u] = digits4(si);
      }
      uint32_t pf[4], ps[4];
      transpose4(hf[0], hf[1], hf[2], hf[3], pf);
      transpose4(hs[0], hs[1], hs[2], hs[3], ps);
#pragma unroll
      for (int d = 0; d < kDig; ++d) {
        const int sw = rr * kDPitch + ((((cq >> 4) ^ (rr >> 2)) & 3) << 4) + (cq & 15);
        *reinterpret_cast<uint32_t*>(&Dg[d][sw]) = pf[d];
        *reinterpret_cast<uint32_t*>(&Dg[kDig + d][sw]) = ps[d];
      }
    }
  }
  const long long kbeg = a.K * part / a.parts, kend = a.K * (part + 1) / a.parts;
  const double scF = ldexp(1.0, eF + 16 - kFBits), scS = ldexp(1.0, eS + 16 - kFBits);

  // the record of pdf li of a batch of 16 (ring positions pos .. pos + cnt -
  // 1); an empty window for li >= cnt
  struct Params {
    long long k;
    int l0, h0, l1, h1;
    float t00, d0, t01, d1, m0, m1;
  };
  auto load_params = [&](int pos, int cnt) {
    Params p = {0, 1, 0, 1, 0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (li < cnt) {
      p.k = kbeg + ring[(pos + li) & (kRing - 1)];
      const MTRec& r = a.rec[p.k];
      p.l0 = r.lo[0];
      p.h0 = r.hi[0];
      p.l1 = r.lo[1];
      p.h1 = r.hi[1];
      p.t00 = r.t0[0];
      p.d0 = r.dt[0];
      p.t01 = r.t0[1];
      p.d1 = r.dt[1];
      p.m0 = r.tm2[0];
      p.m1 = r.tm2[1];
    }
    return p;
  };

  // 16 pdfs on this wave, their records in P
  auto wave_batch = [&](const Params& P, int cnt) {
    const bool valid = li < cnt;
    const long long k = P.k;
    const int l0 = P.l0, h0 = P.h0, l1 = P.l1, h1 = P.h1;
    const float t00 = P.t00, d0 = P.d0, t01 = P.t01, d1 = P.d1;
    // B operands: digits of the quantised column factors of pdf li, columns
    // 16 lg + q (q < 16), one plane per digit; their sum (exact in FP64)
    mt_i32x4 gb[kDig];
    double zy = 0.0;
#pragma unroll
    for (int qw = 0; qw < 4; ++qw) {
      uint32_t h[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int col = c0 + 16 * lg + 4 * qw + u;
        int G = 0;
        if (col >= l1 && col <= h1) G = mt_quant(mt_factor(col - l1, t01, d1, P.m1));
        zy += (double)G;
        h[u] = digits4(G);
      }
      uint32_t pk[4];
      transpose4(h[0], h[1], h[2], h[3], pk);
#pragma unroll
      for (int d = 0; d < kDig; ++d) gb[d][qw] = (int)pk[d];
    }
    double s1 = 0.0, s2 = 0.0, sx = 0.0;
#pragma unroll 1
    for (int ib = 0; ib < 4; ++ib) {
      const int rowoff = (16 * ib + li) * kDPitch + (((lg ^ ((16 * ib + li) >> 2)) & 3) << 4);
      // lane (li, lg) holds rows 16 ib + 4 lg + r of pdf li (D[4q + r][j] in
      // lane j + 16q, slot r)
      double gr[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 16 * ib + 4 * lg + r;
        float gx = 0.0f;
        if (row >= l0 && row <= h0) gx = mt_factor(row - l0, t00, d0, P.m0);
        gr[r] = (double)gx;
        sx += gr[r];
      }
#pragma unroll
      for (int kind = 0; kind < 2; ++kind) {
        mt_i32x4 fa[kDig];
#pragma unroll
        for (int d = 0; d < kDig; ++d)
          fa[d] = *reinterpret_cast<const mt_i32x4*>(&Dg[kind * kDig + d][rowoff]);
        // accumulators by weight 2^(8L), L = a + b = 2 .. 6
        mt_i32x4 y[5];
#pragma unroll
        for (int L = 0; L < 5; ++L) y[L] = (mt_i32x4){0, 0, 0, 0};
#pragma unroll
        for (int da = 0; da < kDig; ++da) {
#pragma unroll
          for (int db = 0; db < kDig; ++db) {
            if (da + db < 2) continue;
            y[da + db - 2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[da], gb[db], y[da + db - 2], 0, 0, 0);
          }
        }
        // sum_L 2^(8L) acc_L = 2^16 (acc2 + 2^8 u + 2^24 v) with
        // u = acc3 + 2^8 acc4, v = acc5 + 2^8 acc6 (below 2^31 in magnitude)
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int u = y[1][r] + y[2][r] * 256, v = y[3][r] + y[4][r] * 256;
          const double Y = __builtin_fma((double)v, 16777216.0,
                                         __builtin_fma((double)u, 256.0, (double)y[0][r]));
          s = __builtin_fma(gr[r], Y, s);
        }
        if (kind == 0)
          s1 += s;
        else
          s2 += s;
      }
    }
    // sums over the four lane groups (rows by group, columns by group)
    s1 += __shfl_xor(s1, 16, 64);
    s2 += __shfl_xor(s2, 16, 64);
    sx += __shfl_xor(sx, 16, 64);
    zy += __shfl_xor(zy, 16, 64);
    s1 += __shfl_xor(s1, 32, 64);
    s2 += __shfl_xor(s2, 32, 64);
    sx += __shfl_xor(sx, 32, 64);
    zy += __shfl_xor(zy, 32, 64);
    if (valid && lg == 0) {
      const MTRec& r = a.rec[k];
      const double S1 = s1 * scF, S2 = s2 * scS;
      const double Zt = sx * (zy * 0x1p-30);
      const double dl = T.a - r.shift;
      const double A1 = S1 + dl * Zt;
      const double A2 = S2 + 2.0 * dl * S1 + dl * dl * Zt;
      atomicAdd(&a.acc[2 * k], (unsigned long long)llrint(A1 * r.sc1));
      atomicAdd(&a.acc[2 * k + 1], (unsigned long long)llrint(A2 * r.sc2));
      if (tbad) {
        // does the window's part of the tile hold a non-finite value?
        const int ra = max(l0, r0) - r0, rb = min(h0, r0 + kMT - 1) - r0;
        const int ca = max(l1, c0) - c0, cb = min(h1, c0 + kMT - 1) - c0;
        const unsigned long long cm =
            (cb - ca == 63) ? ~0ull : (((1ull << (cb - ca + 1)) - 1ull) << ca);
        unsigned long long hit = 0ull;
        for (int i = ra; i <= rb; ++i) hit |= nfmask[i] & cm;
        if (hit) atomicOr(&a.rec[k].flags, 4);
      }
    }
  };

  int head = 0, tail = 0;  // uniform
  long long k0 = kbeg;
  // tile ranges of the next scan step, loaded one step ahead
  unsigned long long bb_next = (k0 + threadIdx.x < kend) ? a.bbox[k0 + threadIdx.x] : 1ull;
  for (;;) {
    // fill the ring up to 256 pending pdfs (or the end of the part)
    while (tail - head < 256 && k0 < kend) {
      const long long k = k0 + threadIdx.x;
      const unsigned long long bb = bb_next;
      bb_next = (k + 256 < kend) ? a.bbox[k + 256] : 1ull;
      const bool hit = k < kend && tx >= (int)(bb & 0xFFFFu) && tx <= (int)((bb >> 16) & 0xFFFFu) &&
                       ty >= (int)((bb >> 32) & 0xFFFFu) && ty <= (int)(bb >> 48);
      const unsigned long long m = __ballot(hit);
      __syncthreads();  // earlier readers of wcnt are done
      if (lane == 0) wcnt[w] = __popcll(m);
      __syncthreads();
      int off = tail;
      for (int v = 0; v < w; ++v) off += wcnt[v];
      if (hit)
        ring[(off + __popcll(m & ((1ull << lane) - 1ull))) & (kRing - 1)] = (uint16_t)(k - kbeg);
      tail += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
      k0 += 256;
    }
    const int avail = min(tail - head, 256);
    if (avail == 0) break;
    __syncthreads();  // ring entries and the staged tile are visible
    // wave w: pending pdfs 64w .. 64w + 63, 16 at a time
    const int bend = min(64 * w + 64, avail);
    for (int b = 64 * w; b < bend; b += 16) wave_batch(load_params(head + b, min(16, avail - b)), min(16, avail - b));
    head += avail;
    __syncthreads();  // the ring slots just used may be refilled
  }
}

// ---------------------------------------------------------------------------
// per pdf: moments from the fixed-point totals
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mt_final(MTArgs a) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.K) return;
  const MTRec r = a.rec[k];
  double E = __builtin_nan(""), V = __builtin_nan("");
  if (r.flags == 0) {
    const double A1 = (double)(long long)a.acc[2 * k] / r.sc1;
    const double A2 = (double)(long long)a.acc[2 * k + 1] / r.sc2;
    const double s1 = A1 / r.Z, s2 = A2 / r.Z;
    E = r.shift + s1;
    // a one-cell window is a point mass: variance 0 exactly
    V = (r.lo[0] == r.hi[0] && r.lo[1] == r.hi[1]) ? 0.0 : s2 - s1 * s1;
    if (!(r.Z > 0.0)) E = V = __builtin_nan("");
  }
  a.mean[k] = E;
  a.var[k] = V;
  if (a.delta2) {
    double d2 = __builtin_nan("");
    if ((r.flags & 3) == 0 && a.has_model) {
      const double x[2] = {a.mu[2 * k], a.mu[2 * k + 1]};
      const double fm = model_at(a.model.kind, 2, a.model.theta, x);
      d2 = 0.5 * (V + (E - fm) * (E - fm));
    }
    a.delta2[k] = d2;
  }
}

constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct MTLayout {
  size_t rec, bbox, acc, tiles, bytes;
};

MTLayout mt_layout(int ntiles, long long K) {
  MTLayout L;
  L.rec = 0;
  L.bbox = L.rec + al256((size_t)K * sizeof(MTRec));
  L.acc = L.bbox + al256((size_t)K * 8);
  L.tiles = L.acc + al256((size_t)K * 16);
  L.bytes = L.tiles + al256((size_t)ntiles * sizeof(MTTile));
  return L;
}

}  // namespace

// tile indices are 16 bits, the per-tile table and the workgroup count are
// kept bounded (at most 2^20 tiles, parts of at most 65 536 pdfs each)
bool moments_tiled_applies(const vup_mm& mm, const vup_dists& d) {
  if (mm.grid.ndim != 2 || d.ncomp != 1) return false;
  const long long ntx = (mm.grid.n[1] + kMT - 1) / kMT, nty = (mm.grid.n[0] + kMT - 1) / kMT;
  return ntx <= kMTMaxTiles && nty <= kMTMaxTiles && ntx * nty <= (1ll << 20) &&
         d.K < (1ll << 26);
}

size_t moments_tiled_ws_bytes(const vup_mm& mm, long long K) {
  const long long ntx = (mm.grid.n[1] + kMT - 1) / kMT, nty = (mm.grid.n[0] + kMT - 1) / kMT;
  return mt_layout((int)(ntx * nty), K).bytes;
}

hipError_t launch_moments_tiled(const vup_mm& mm, const vup_dists& d, const vup_model* model,
                                void* ws, double* mean, double* var, double* delta2,
                                hipStream_t s) {
  if (d.K == 0) return hipSuccess;
  MTArgs a{};
  a.n0 = mm.grid.n[0];
  a.n1 = mm.grid.n[1];
  for (int i = 0; i < 2; ++i) {
    a.lo[i] = mm.grid.lo[i];
    a.hi[i] = mm.grid.hi[i];
  }
  a.rowstride = mm.pitch;
  a.f32 = reinterpret_cast<const float*>(static_cast<const char*>(mm.ws) + mm.off_f32);
  a.K = d.K;
  a.ns = d.n_sigma;
  a.mu = d.mu;
  a.sigma = d.sigma;
  a.ntx = (a.n1 + kMT - 1) / kMT;
  a.nty = (a.n0 + kMT - 1) / kMT;
  const int ntiles = a.ntx * a.nty;
  // parts of the pdf list per tile: about 2048 workgroups, at least 256
  // pdfs per part, at most 65 536 (16-bit ring entries)
  long long parts = (2048 + ntiles - 1) / ntiles;
  parts = parts < d.K / 256 ? parts : d.K / 256;
  parts = parts < 1 ? 1 : (parts > 64 ? 64 : parts);
  const long long need = (d.K + 65535) / 65536;
  a.parts = (int)(parts > need ? parts : need);
  const MTLayout L = mt_layout(ntiles, d.K);
  char* base = static_cast<char*>(ws);
  a.rec = reinterpret_cast<MTRec*>(base + L.rec);
  a.bbox = reinterpret_cast<unsigned long long*>(base + L.bbox);
  a.acc = reinterpret_cast<unsigned long long*>(base + L.acc);
  a.tiles = reinterpret_cast<MTTile*>(base + L.tiles);
  a.mean = mean;
  a.var = var;
  a.delta2 = delta2;
  a.has_model = model != nullptr;
  if (model) a.model = *model;
  hipLaunchKernelGGL(k_mt_tiles, dim3(ntiles), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_mt_prep, dim3((unsigned)((d.K + 15) / 16)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_mt_main, dim3((unsigned)(ntiles * a.parts)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_mt_final, dim3((unsigned)((d.K + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace vup
