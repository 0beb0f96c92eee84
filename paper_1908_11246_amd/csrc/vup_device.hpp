// Device-side helpers shared by the VUP kernels (gfx950, wave64).
// Grid convention: uniform cell-centred grid (composite midpoint rule, Sec. 3),
// flat index row major with axis 0 slowest.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vup.h"

namespace vup {

constexpr int kThreads = 256;     // threads per workgroup of the sweep kernels
constexpr int kWaves = kThreads / 64;
constexpr int kRowChunk = 512;    // rows of the row table held in LDS at once
// rows per row-table pass of the run-form propagation when many distributions
// are propagated: 256 keeps a workgroup's LDS near 20 KB at 1024-cell rows, so
// seven workgroups (seven waves per SIMD, the kernel held to 72 VGPRs without
// spills) fit on a CU; with fewer distributions than resident workgroups, 512
// (fewer passes)
constexpr int kRunRowChunk = 256;
// rows per row-table pass of the cell-form propagation (8-byte entries, 4 KB;
// a multiple of the workgroup size, as its row builder steps by whole
// workgroups)
constexpr int kPropRowChunk = 512;
constexpr int kMaxSW = 16;        // widest strip of the fastest axis
constexpr int kMaxBinsPerThread = (VUP_MAX_BINS + 1 + kThreads - 1) / kThreads;

// counters stored in the workspace (int64 each)
// [4]: number of runs of equal bin along the fastest axis (set by vup_bin,
// not cleared by vup_counters); the propagation uses the run form when the
// mean run length is at least kRunMinLength cells.
// [5]: scratch of the run construction; [6]: sweep mode (VUP_SWEEP_*).
enum Counter {
  kCntOutside = 0,
  kCntBadEdges = 1,
  kCntBadParam = 2,
  kCntEmpty = 3,
  kCntRuns = 4,
  kCntScratch = 5,
  kCntMode = 6
};
constexpr int kRunMinLength = 3;

// grid + bin-map description passed by value to every sweep kernel
struct GridDev {
  int ndim;
  int n[4];
  double lo[4];
  double hi[4];
  int pitch;                 // padded length of the last axis in the bin map
  long long rowstride[4];    // bin-map element stride of axes 0..ndim-2
};

struct DistsDev {
  long long K;
  int C;
  double ns;
  const double* __restrict__ mu;
  const double* __restrict__ sigma;
  const double* __restrict__ weight;
};

// ---------------------------------------------------------------------------
// truncation window of one axis: kept cells j with |x_j - mu| <= ns*sigma,
// evaluated in FP64 in a fixed operation order with contraction disabled so
// that the integer bounds are reproducible bit for bit. Returns false for
// invalid parameters; an empty window is lo = 0, hi = -1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool axis_window(double lo, double hi, int n, double mu, double sigma,
                                            double ns, int& jlo, int& jhi) {
#pragma clang fp contract(off)
  if (!(sigma > 0.0) || !isfinite(sigma) || !isfinite(mu)) {
    jlo = 0;
    jhi = -1;
    return false;
  }
  const double h = (hi - lo) / n;
  const double tlo = ((mu - ns * sigma) - lo) / h - 0.5;
  const double thi = ((mu + ns * sigma) - lo) / h - 0.5;
  double a = ceil(tlo), b = floor(thi);
  a = a < 0.0 ? 0.0 : a;
  b = b > (double)(n - 1) ? (double)(n - 1) : b;
  if (a > b) {
    if (mu >= lo && mu <= hi) {
      double c = floor((mu - lo) / h);
      c = c < 0.0 ? 0.0 : c;
      c = c > (double)(n - 1) ? (double)(n - 1) : c;
      a = b = c;
    } else {
      jlo = 0;
      jhi = -1;
      return true;
    }
  }
  jlo = (int)a;
  jhi = (int)b;
  return true;
}

// cell centre of axis d
__device__ __forceinline__ double cell_centre(double lo, double hi, int n, int j) {
#pragma clang fp contract(off)
  return lo + (j + 0.5) * ((hi - lo) / n);
}

// The per-axis Gaussian factors exp(-t^2/2), t = (x_j - mu)/sigma, of a pdf
// much narrower than a cell would fall below FP32's range: its window is the
// one cell holding the mean, whose centre can lie up to half a cell, i.e. many
// sigma, away. Such an axis's factors are scaled by 2^m, m = floor(t*^2/2
// log2 e) with t* the t of the window's cell nearest the mean, so its largest
// factor lies in (1/2, 1]; the scale cancels from every normalised result, and
// the reported normalisers are scaled back exactly (ldexp). Only axes whose
// largest factor would be below 2^-kScaleMinExp (t* above about 5.3) are
// scaled, m = 0 otherwise: every pdf the grid resolves (sigma above a tenth of
// a cell) keeps its unscaled factors and its densities' roundings (BF16 and
// E4M3 included), while the products over four axes of unscaled factors stay
// above 2^-80, where the fixed-point scales (2^32 over the mass) fit FP32. m
// is capped at kMaxScaleExp, beyond which the density is below FP64's range.
constexpr int kScaleMinExp = 20;
constexpr int kMaxScaleExp = 1100;

// m for window cells jlo .. jhi of n over [lo, hi], t formed as the factors
// form it. Out of line: it runs for few windows, and inlined its FP64 code
// raised the scalar-register pressure of the sweep kernels' set-up
__device__ __noinline__ int axis_scale_exp(double lo, double hi, int n, int jlo, int jhi,
                                           double mu, double rsig) {
  const double h = (hi - lo) / n;
  double c = floor((mu - lo) / h);
  c = c >= (double)jlo ? c : (double)jlo;  // (a NaN goes to jlo)
  c = c <= (double)jhi ? c : (double)jhi;
  const double t = (cell_centre(lo, hi, n, (int)c) - mu) * rsig;
  const double e = floor(0.5 * (t * t) * 1.4426950408889634);  // t*^2 / 2 / ln 2
  if (!(e >= (double)kScaleMinExp)) return 0;
  return e < (double)kMaxScaleExp ? (int)e : kMaxScaleExp;  // (t = inf: the cap)
}

// the natural log of an axis's scale 2^m, added to the factors' arguments
__device__ __forceinline__ double scale_log(int m) { return (double)m * 0.6931471805599453; }

// per-axis Gaussian factor 2^m exp(-t^2/2), t = (x_j - mu)/sigma, rounded to
// FP32, with off = scale_log(m). The argument fma(-1/2, t^2, off) costs the
// one FP64 operation that -t^2/2 alone does, and equals it for off = 0 (halving
// is exact). It is formed in FP64 and split into an FP32 head and tail,
// exp(a) = exp(a_hi) (1 + a_lo), which keeps the result within about one FP32
// ulp without the register cost of an FP64 exponential.
__device__ __forceinline__ float gauss_factor(double x, double mu, double sigma, double off) {
  const double t = (x - mu) / sigma;
  const double arg = fma(-0.5, t * t, off);
  const float hi = (float)arg;
  const float lo = (float)(arg - (double)hi);
  return expf(hi) * (1.0f + lo);
}

// the same with t = (x - mu) * rsig, rsig = 1/sigma computed once per axis
// (t then differs from the quotient by at most an FP64 ulp or so)
__device__ __forceinline__ float gauss_factor_r(double x, double mu, double rsig, double off) {
  const double t = (x - mu) * rsig;
  const double arg = fma(-0.5, t * t, off);
  const float hi = (float)arg;
  const float lo = (float)(arg - (double)hi);
  return expf(hi) * (1.0f + lo);
}

// ---------------------------------------------------------------------------
// built-in models (Sec. 2, eq. modelfunction)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double model_at(int kind, int ndim, const double* theta, const double* x) {
  switch (kind) {
    case VUP_MODEL_LINEAR: {
      double y = theta[0];
      for (int d = 0; d < ndim; ++d) y += theta[d + 1] * x[d];
      return y;
    }
    case VUP_MODEL_SINCOS2:
      return sin(x[0]) + 0.5 * cos(2.0 * x[1]) + x[0] * x[1] / 4.0;
    case VUP_MODEL_DAMPED3:
      return exp(-0.1 * x[2]) * sin(x[0]) * cos(x[1]) + 0.1 * x[0] * x[1] * x[2];
    case VUP_MODEL_RING4: {
      double s = 0.0, t = 0.0;
      for (int j = 0; j < 4; ++j) s += sin(x[j]) * x[(j + 1) & 3];
      for (int j = 0; j < 4; ++j) t += x[j];
      return s + 0.05 * (t * t);
    }
    case VUP_MODEL_TIMING2: {
      const double sa = sin(x[1]);
      return 1.1 * sin(x[0]) + 7.0 * (sa * sa);
    }
    case VUP_MODEL_IPSA2:
      return x[0] * x[0] + 5.0 * sin(3.0 * x[0]) + x[1];
    default:
      return __builtin_nan("");
  }
}

// ---------------------------------------------------------------------------
// density quantisers (round to nearest even), inputs are finite and in [0, 1]
// ---------------------------------------------------------------------------
__device__ __forceinline__ float round_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// OCP E4M3 value of 448*w, returned divided by 448 is NOT done here: the
// kernels accumulate the E4M3 value itself (the common scale cancels in P).
__device__ __forceinline__ float round_e4m3(float x) {
  // normals: 4 significant bits (drop 20 of FP32's 23 fraction bits);
  // below 2^-6: multiples of the subnormal quantum 2^-9
  uint32_t u = __float_as_uint(x);
  uint32_t rn = (u + 0x7FFFFu + ((u >> 20) & 1u)) & 0xFFF00000u;
  float sub = __builtin_rintf(x * 512.0f) * (1.0f / 512.0f);
  return x < 0.015625f ? sub : __uint_as_float(rn);
}

// LDS byte address of a pointer into LDS (an address-space cast, so it holds
// wherever the compiler places the kernel's LDS).
typedef __attribute__((address_space(3))) char vup_lds_char;
typedef __attribute__((address_space(3))) uint32_t vup_lds_u32;
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const vup_lds_char*)p;
}

// m * (low or high 16 bits of x) + c in one VALU op (v_mad_u32_u16, op_sel
// picking the half): an address from a packed 16-bit code; m < 2^16
__device__ __forceinline__ uint32_t mad_lo16(uint32_t x, uint32_t m, uint32_t c) {
  uint32_t r;
  asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(m), "v"(c));
  return r;
}
__device__ __forceinline__ uint32_t mad_hi16(uint32_t x, uint32_t m, uint32_t c) {
  uint32_t r;
  asm("v_mad_u32_u16 %0, %1, %2, %3 op_sel:[1,0,0,0]" : "=v"(r) : "v"(x), "v"(m), "v"(c));
  return r;
}
// M * (low 16 bits of x) + c for a uniform c and an inline-constant M
// (0 < M <= 64): no register for either
template <int M>
__device__ __forceinline__ uint32_t mad_lo16_k(uint32_t x, uint32_t c) {
  static_assert(M > 0 && M <= 64, "an inline constant");
  uint32_t r;
  asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(r) : "v"(x), "i"(M), "s"(c));
  return r;
}

// The same roundings for two values at once with gfx950's packed conversions
// (v_cvt_pk_bf16_f32, v_cvt_pk_fp8_f32 to OCP E4M3; both round to nearest
// even, checked bit for bit against the software roundings above, ties and
// E4M3 subnormals included). For VUP_FP8E4M3 the inputs are 448 w and the
// outputs the E4M3 values (the common scale cancels in P).
typedef __bf16 vup_bf16x2 __attribute__((ext_vector_type(2)));
typedef float vup_f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void bf16_pair(float a, float b, float& ra, float& rb) {
  const vup_bf16x2 v = __builtin_convertvector((vup_f32x2){a, b}, vup_bf16x2);
  const uint32_t pk = __builtin_bit_cast(uint32_t, v);
  ra = __uint_as_float(pk << 16);
  rb = __uint_as_float(pk & 0xFFFF0000u);
}

template <int PREC>
__device__ __forceinline__ void quantize2(float a, float b, float& qa, float& qb) {
  if constexpr (PREC == VUP_BF16) {
    bf16_pair(a, b, qa, qb);
  } else if constexpr (PREC == VUP_BF16X2) {
    float ha, hb, la, lb;
    bf16_pair(a, b, ha, hb);
    bf16_pair(a - ha, b - hb, la, lb);
    qa = ha + la;
    qb = hb + lb;
  } else if constexpr (PREC == VUP_FP8E4M3) {
    const int f8 = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    qa = __builtin_amdgcn_cvt_f32_fp8(f8, 0);
    qb = __builtin_amdgcn_cvt_f32_fp8(f8, 1);
  } else {
    qa = a;
    qb = b;
  }
}

template <int PREC>
__device__ __forceinline__ float quantize(float w) {
  if constexpr (PREC == VUP_BF16) {
    return round_bf16(w);
  } else if constexpr (PREC == VUP_BF16X2) {
    const float h = round_bf16(w);
    return h + round_bf16(w - h);
  } else if constexpr (PREC == VUP_FP8E4M3) {
    return round_e4m3(448.0f * w);
  } else {
    return w;
  }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
// DPP moves of an FP64 value (both halves with the same pattern); lanes whose
// source falls outside their 16-lane row read 0
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFF), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// value of one lane (uniform result)
__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFF), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// inclusive prefix sum within each 16-lane row (row_shr 1, 2, 4, 8)
__device__ __forceinline__ double row_scan(double v) {
  v += dpp_f64<0x111>(v);
  v += dpp_f64<0x112>(v);
  v += dpp_f64<0x114>(v);
  v += dpp_f64<0x118>(v);
  return v;
}

// sum over the 64 lanes (all lanes active), in a fixed order; uniform result
__device__ __forceinline__ double wave_sum(double v) {
  v = row_scan(v);
  return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}

// inclusive prefix sum over the 64 lanes (all lanes active)
__device__ __forceinline__ double wave_scan(double v) {
  v = row_scan(v);
  const int row = (threadIdx.x & 63) >> 4;
  const double r0 = lane_value(v, 15), r1 = lane_value(v, 31), r2 = lane_value(v, 47);
  const double before = row == 0 ? 0.0 : (row == 1 ? r0 : (row == 2 ? r0 + r1 : (r0 + r1) + r2));
  return v + before;
}

// deterministic block sum of one double per thread; `red` is LDS scratch of
// kWaves doubles. All threads receive the result.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kWaves; ++w) s += red[w];
  return s;
}

}  // namespace vup
