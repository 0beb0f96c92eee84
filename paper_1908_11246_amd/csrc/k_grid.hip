// Model-matrix construction (done once per grid and model, Appendix A: the
// N model evaluations and the sort are amortised over all propagated pdfs):
//   k_eval_grid     f_i = M(x_i) at cell centres, FP64
//   k_minmax / k_edges   B uniform bins over [min f, max f]
//   k_bin           indicator of eq. (4) as a bin index; padded bin map
//                   (4*bin, LDS byte offsets for the sweep kernels), padded
//                   FP32 copy of f in anchored form (every eighth column
//                   holds f, the columns after it their offset from it),
//                   per-chunk bin counts
//   k_tile_sums, k_scan_tile_sums, k_tile_scan  exclusive scan of the counts in
//                   (bin, chunk) order; k_csr_offsets  CSR row starts and counts
//   k_scatter       stable scatter of cell indices into compressed-by-bin
//                   order (the sparse one-hot model matrix of eq. (5))
// plus the per-distribution window listing.
#include <hip/hip_runtime.h>

#include "vup_device.hpp"
#include "vup_internal.hpp"

namespace vup {

// ---------------------------------------------------------------------------
// model evaluation
// ---------------------------------------------------------------------------
struct EvalArgs {
  int ndim;
  int n[4];
  double lo[4], hi[4];
  vup_model m;
  long long N;
};

__global__ __launch_bounds__(256) void k_eval_grid(EvalArgs a, double* __restrict__ f) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  double x[4];
  long long t = i;
  for (int d = a.ndim - 1; d >= 0; --d) {
    const int j = (int)(t % a.n[d]);
    t /= a.n[d];
    x[d] = cell_centre(a.lo[d], a.hi[d], a.n[d], j);
  }
  f[i] = model_at(a.m.kind, a.ndim, a.m.theta, x);
}

hipError_t launch_eval_grid(const vup_grid& g, const vup_model& m, double* f, hipStream_t s) {
  EvalArgs a{};
  a.ndim = g.ndim;
  a.N = 1;
  for (int d = 0; d < g.ndim; ++d) {
    a.n[d] = g.n[d];
    a.lo[d] = g.lo[d];
    a.hi[d] = g.hi[d];
    a.N *= g.n[d];
  }
  a.m = m;
  const long long blocks = (a.N + 255) / 256;
  hipLaunchKernelGGL(k_eval_grid, dim3((unsigned)blocks), dim3(256), 0, s, a, f);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// uniform edges: min/max via order-preserving integer images of the doubles
// (exact, order independent), then e_b = lo + b*((hi - lo)/B), e_B = hi.
// The two extreme slots of `edges` hold the running min/max images.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long ord_of(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double of_ord(unsigned long long o) {
  const unsigned long long u = (o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o;
  return __longlong_as_double((long long)u);
}

__global__ void k_minmax_init(unsigned long long* e, int B) {
  if (threadIdx.x == 0) {
    e[0] = ~0ull;  // running min image
    e[B] = 0ull;   // running max image
  }
}

// Min and max of the non-NaN model values as order-preserving integer images.
// A thread reads eight values at once (independent loads in flight), the
// workgroup reduces in LDS, and one pair of atomics per workgroup merges.
__global__ __launch_bounds__(256) void k_minmax(const double* __restrict__ f, long long N,
                                                unsigned long long* e, int B) {
  __shared__ unsigned long long smn[4], smx[4];
  unsigned long long mn = ~0ull, mx = 0ull;
  const long long stride = (long long)gridDim.x * 256;
  for (long long i0 = (long long)blockIdx.x * 256 + threadIdx.x; i0 < N; i0 += 8 * stride) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const long long i = i0 + u * stride;
      v[u] = i < N ? f[i] : __builtin_nan("");
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (v[u] != v[u]) continue;
      const unsigned long long o = ord_of(v[u]);
      mn = o < mn ? o : mn;
      mx = o > mx ? o : mx;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long a = __shfl_xor(mn, off, 64), b = __shfl_xor(mx, off, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if ((threadIdx.x & 63) == 0) {
    smn[threadIdx.x >> 6] = mn;
    smx[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      mn = smn[w] < mn ? smn[w] : mn;
      mx = smx[w] > mx ? smx[w] : mx;
    }
    atomicMin(e, mn);
    atomicMax(e + B, mx);
  }
}

__global__ __launch_bounds__(256) void k_edges(double* e, int B) {
#pragma clang fp contract(off)
  __shared__ double lohi[2];
  if (threadIdx.x == 0) {
    const unsigned long long* u = reinterpret_cast<const unsigned long long*>(e);
    lohi[0] = of_ord(u[0]);
    lohi[1] = of_ord(u[B]);
  }
  __syncthreads();
  const double lo = lohi[0], hi = lohi[1];
  const double w = (hi - lo) / B;
  for (int b = threadIdx.x; b <= B; b += blockDim.x) e[b] = (b == B) ? hi : lo + b * w;
}

hipError_t launch_uniform_edges(const double* f, int64_t N, int B, double* edges, hipStream_t s) {
  unsigned long long* e = reinterpret_cast<unsigned long long*>(edges);
  hipLaunchKernelGGL(k_minmax_init, dim3(1), dim3(64), 0, s, e, B);
  long long blocks = (N + 2047) / 2048;  // eight values per thread
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_minmax, dim3((unsigned)blocks), dim3(256), 0, s, f, (long long)N, e, B);
  hipLaunchKernelGGL(k_edges, dim3(1), dim3(256), 0, s, edges, B);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
struct BinArgs {
  const double* __restrict__ f;
  const double* __restrict__ edges_in;
  double* edges_ws;
  int32_t* bin;       // may be null
  uint16_t* binmap;   // [rows*pitch]
  float* f32;         // [rows*pitch]
  int* chunk_counts;  // [(B+1) * nblk], bin-major
  unsigned long long* counters;
  int B;
  int nL;             // cells on the fastest axis
  int pitch;
  long long rows;
  long long nblk;
  int chunk;          // padded positions per chunk
};

// bin index of y: largest b < B with e[b] <= y, when e[0] <= y <= e[B]
__device__ __forceinline__ int bin_search(const double* e, int B, double y) {
  if (!(y >= e[0] && y <= e[B])) return -1;
  int lo = 0, hi = B - 1;  // answer in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (e[mid] <= y) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_bin(BinArgs a) {
  extern __shared__ double sh[];  // edges[B+1], then int counts[B+1]
  double* e = sh;
  int* cnt = reinterpret_cast<int*>(sh + a.B + 1);
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int b = threadIdx.x; b <= a.B; b += 256) {
    const double v = a.edges_in[b];
    e[b] = v;
    if (!isfinite(v)) atomicOr(&bad, 1);
    if (b > 0 && !(a.edges_in[b - 1] < v)) atomicOr(&bad, 1);
    cnt[b] = 0;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int b = threadIdx.x; b <= a.B; b += 256) a.edges_ws[b] = e[b];
    if (threadIdx.x == 0 && bad) atomicAdd(a.counters + kCntBadEdges, 1ull);
  }
  const long long base = (long long)blockIdx.x * a.chunk;
  const long long total = a.rows * a.pitch;
  int outside = 0;
  for (int q = threadIdx.x; q < a.chunk; q += 256) {
    const long long p = base + q;
    if (p >= total) break;
    const long long row = p / a.pitch;
    const int col = (int)(p - row * a.pitch);
    uint16_t code = (uint16_t)(4 * a.B);
    float fv = 0.0f;
    if (col < a.nL) {
      const long long cell = row * a.nL + col;
      const double y = a.f[cell];
      const int b = bad ? -1 : bin_search(e, a.B, y);
      if (a.bin) a.bin[cell] = b;
      if (b >= 0) {
        code = (uint16_t)(4 * b);
        atomicAdd(&cnt[b], 1);
      } else {
        ++outside;
        atomicAdd(&cnt[a.B], 1);
      }
      // anchored FP32 form: columns 8m hold f, the seven after each their
      // difference from it (taken in FP64, rounded once); after a non-finite
      // anchor they hold their own values, which the difference would lose
      const int c0 = col & ~7;
      const double f0 = a.f[row * a.nL + c0];
      fv = col == c0 ? (float)y : (float)(isfinite(f0) ? y - f0 : y);
    }
    a.binmap[p] = code;
    a.f32[p] = fv;
  }
  for (int off = 32; off > 0; off >>= 1) outside += __shfl_xor(outside, off, 64);
  if ((threadIdx.x & 63) == 0 && outside) atomicAdd(a.counters + kCntOutside, (unsigned long long)outside);
  __syncthreads();
  for (int b = threadIdx.x; b <= a.B; b += 256) a.chunk_counts[(long long)b * a.nblk + blockIdx.x] = cnt[b];
}

// ---------------------------------------------------------------------------
// exclusive prefix sum of n ints in place (values and sums below 2^31), by
// tiles of kScanTile: tile totals, one workgroup scanning the totals, then
// each tile scanned from its offset. `tsum` holds ceil(n / kScanTile) int64.
// ---------------------------------------------------------------------------
constexpr int kScanPer = 4;                  // elements per thread (one 16-byte load)
constexpr int kScanTile = 256 * kScanPer;    // elements per workgroup

// this thread's four consecutive elements of the tile (zeros past n); the
// array is 16-byte aligned and tiles are whole multiples of four elements
__device__ __forceinline__ int4 scan_load4(const int* __restrict__ v, long long n, long long p) {
  if (p + 3 < n) return *reinterpret_cast<const int4*>(v + p);
  return make_int4(p < n ? v[p] : 0, p + 1 < n ? v[p + 1] : 0, p + 2 < n ? v[p + 2] : 0,
                   p + 3 < n ? v[p + 3] : 0);
}

__global__ __launch_bounds__(256) void k_tile_sums(const int* __restrict__ v, long long n,
                                                   long long* __restrict__ tsum) {
  __shared__ long long red[4];
  const long long p = (long long)blockIdx.x * kScanTile + kScanPer * threadIdx.x;
  const int4 x = scan_load4(v, n, p);
  long long sum = (long long)x.x + x.y + x.z + x.w;
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) tsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// inclusive scan of one value per thread across a 1024-thread (or smaller)
// workgroup; `wsum` is LDS for one value per wave
__device__ __forceinline__ long long block_incl_scan(long long x, long long* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const long long t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  long long off = 0;
  for (int w = 0; w < wave; ++w) off += wsum[w];
  __syncthreads();
  return x + off;
}

__global__ __launch_bounds__(1024) void k_scan_tile_sums(long long* tsum, long long ntiles,
                                                         int* total) {
  __shared__ long long wsum[16];
  __shared__ long long last;
  long long carry = 0;
  for (long long b0 = 0; b0 < ntiles; b0 += 1024) {
    const long long i = b0 + threadIdx.x;
    const long long x = i < ntiles ? tsum[i] : 0;
    const long long incl = block_incl_scan(x, wsum);
    if (i < ntiles) tsum[i] = carry + incl - x;
    if (threadIdx.x == 1023) last = incl;
    __syncthreads();
    carry += last;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = (int)carry;
}

__global__ __launch_bounds__(256) void k_tile_scan(int* __restrict__ v, long long n,
                                                   const long long* __restrict__ tsum) {
  __shared__ long long wsum[4];
  const long long p = (long long)blockIdx.x * kScanTile + kScanPer * threadIdx.x;
  const int4 x = scan_load4(v, n, p);
  const long long s = (long long)x.x + x.y + x.z + x.w;
  const long long e0 = block_incl_scan(s, wsum) - s + tsum[blockIdx.x];
  const int4 y = make_int4((int)e0, (int)(e0 + x.x), (int)(e0 + x.x + x.y),
                           (int)(e0 + x.x + x.y + x.z));
  if (p + 3 < n) {
    *reinterpret_cast<int4*>(v + p) = y;
  } else {
    if (p < n) v[p] = y.x;
    if (p + 1 < n) v[p + 1] = y.y;
    if (p + 2 < n) v[p + 2] = y.z;
  }
}

long long scan_tiles(long long n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_scan_excl(int* v, long long n, long long* tsum, int* total, hipStream_t s) {
  const long long nt = scan_tiles(n);
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nt), dim3(256), 0, s, v, n, tsum);
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(1024), 0, s, tsum, nt, total);
  hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)nt), dim3(256), 0, s, v, n, tsum);
  return hipGetLastError();
}

// CSR of the model matrix from the scanned chunk counts: bin b occupies
// [b*nblk, (b+1)*nblk) in (bin, chunk) order, so its first position is the
// row start; slot B collects the cells without a bin, after all binned cells.
__global__ __launch_bounds__(256) void k_csr_offsets(const int* __restrict__ cc, long long nblk,
                                                     int B, long long N, long long* counts,
                                                     long long* offsets) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b > B) return;
  const long long start = cc[(long long)b * nblk];
  const long long next = b < B ? (long long)cc[(long long)(b + 1) * nblk] : N;
  offsets[b] = start;
  counts[b] = next - start;
}

// one wave per chunk: cells in increasing order, stable within each bin
__global__ __launch_bounds__(64) void k_scatter(BinArgs a, const int* __restrict__ cc,
                                                int32_t* __restrict__ perm) {
  extern __shared__ int pos[];  // [B+1] running positions of this chunk
  for (int b = threadIdx.x; b <= a.B; b += 64) pos[b] = cc[(long long)b * a.nblk + blockIdx.x];
  __syncthreads();
  const long long base = (long long)blockIdx.x * a.chunk;
  const long long total = a.rows * a.pitch;
  const int lane = threadIdx.x;
  for (int q0 = 0; q0 < a.chunk; q0 += 64) {
    const long long p = base + q0 + lane;
    int b = -2;
    long long cell = -1;
    if (p < total) {
      const long long row = p / a.pitch;
      const int col = (int)(p - row * a.pitch);
      if (col < a.nL) {
        cell = row * a.nL + col;
        const int code = a.binmap[p];
        b = (code == 4 * a.B) ? -2 : code >> 2;
      }
    }
    // lanes holding the same bin as this lane (found one distinct bin at a
    // time with ballots), then one LDS read of the bin's position per lane;
    // the highest lane of each bin advances it. One wave per workgroup: its
    // LDS reads and writes take effect in program order, so no barrier.
    unsigned long long todo = __ballot(b >= 0), same = 0ull;
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int bl = __builtin_amdgcn_readlane(b, leader);
      const unsigned long long m = __ballot(b == bl);
      if (b == bl) same = m;
      todo &= ~m;
    }
    if (b >= 0) {
      const int start = pos[b];
      perm[start + __popcll(same & ((1ull << lane) - 1ull))] = (int32_t)cell;
      if ((same >> lane) == 1ull) pos[b] = start + __popcll(same);
    }
  }
}

hipError_t launch_runs(const vup_mm& mm, hipStream_t s);

hipError_t launch_bin(const vup_mm& mm, const double* f, const double* edges, int32_t* bin,
                      hipStream_t s) {
  char* ws = static_cast<char*>(mm.ws);
  WsLayout L;
  ws_layout(mm.grid, mm.B, &L);
  BinArgs a{};
  a.f = f;
  a.edges_in = edges;
  a.edges_ws = reinterpret_cast<double*>(ws + mm.off_edges);
  a.bin = bin;
  a.binmap = reinterpret_cast<uint16_t*>(ws + mm.off_binmap);
  a.f32 = reinterpret_cast<float*>(ws + mm.off_f32);
  a.chunk_counts = reinterpret_cast<int*>(ws + mm.off_scratch);
  a.counters = reinterpret_cast<unsigned long long*>(ws + mm.off_counters);
  a.B = mm.B;
  a.nL = mm.grid.n[mm.grid.ndim - 1];
  a.pitch = mm.pitch;
  a.rows = mm.rows;
  a.nblk = L.nblk;
  a.chunk = L.chunk;
  const size_t lds = (size_t)(mm.B + 1) * 8 + (size_t)(mm.B + 1) * 4;
  hipLaunchKernelGGL(k_bin, dim3((unsigned)L.nblk), dim3(256), lds, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const long long nc = (long long)(mm.B + 1) * L.nblk;
  err = launch_scan_excl(a.chunk_counts, nc, reinterpret_cast<long long*>(ws + L.off_tsum), nullptr,
                         s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_csr_offsets, dim3((unsigned)((mm.B + 1 + 255) / 256)), dim3(256), 0, s,
                     a.chunk_counts, L.nblk, mm.B, (long long)mm.N,
                     reinterpret_cast<long long*>(ws + mm.off_counts),
                     reinterpret_cast<long long*>(ws + mm.off_offsets));
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)L.nblk), dim3(64), (size_t)(mm.B + 1) * 4, s, a,
                     a.chunk_counts, reinterpret_cast<int32_t*>(ws + mm.off_perm));
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_runs(mm, s);
}

// ---------------------------------------------------------------------------
// windows of every (k, c)
// ---------------------------------------------------------------------------
struct WinArgs {
  int ndim;
  int n[4];
  double lo[4], hi[4];
  DistsDev d;
};

__global__ __launch_bounds__(256) void k_windows(WinArgs a, int32_t* __restrict__ win) {
  const long long kc = (long long)blockIdx.x * 256 + threadIdx.x;
  if (kc >= a.d.K * a.d.C) return;
  const int D = a.ndim;
  int lo[4], hi[4];
  bool bad = false;
  for (int d = 0; d < D; ++d) {
    if (!axis_window(a.lo[d], a.hi[d], a.n[d], a.d.mu[kc * D + d], a.d.sigma[kc * D + d], a.d.ns,
                     lo[d], hi[d]))
      bad = true;
  }
  for (int d = 0; d < D; ++d) {
    win[(kc * D + d) * 2 + 0] = bad ? 0 : lo[d];
    win[(kc * D + d) * 2 + 1] = bad ? -1 : hi[d];
  }
}

hipError_t launch_windows(const vup_grid& g, const vup_dists& d, int32_t* win, hipStream_t s) {
  const long long n = d.K * d.ncomp;
  if (n == 0) return hipSuccess;
  WinArgs a{};
  a.ndim = g.ndim;
  for (int i = 0; i < g.ndim; ++i) {
    a.n[i] = g.n[i];
    a.lo[i] = g.lo[i];
    a.hi[i] = g.hi[i];
  }
  a.d = make_dists_dev(d);
  hipLaunchKernelGGL(k_windows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, win);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool ws_layout(const vup_grid& g, int B, WsLayout* out) {
  WsLayout L{};
  const int nL = g.n[g.ndim - 1];
  L.pitch = (nL + 31) / 32 * 32;
  L.rows = 1;
  for (int d = 0; d + 1 < g.ndim; ++d) L.rows *= g.n[d];
  const long long N = L.rows * nL;
  const long long padded = L.rows * L.pitch;
  // chunks of the bin sort: small for parallelism, larger when the (bin,
  // chunk) count table would grow past 2^24 entries
  L.chunk = 1024;
  while ((long long)(B + 1) * ((padded + L.chunk - 1) / L.chunk) > (1ll << 24) && L.chunk < 65536)
    L.chunk *= 2;
  L.nblk = (padded + L.chunk - 1) / L.chunk;
  const long long rowblocks = L.rows * (L.pitch / 32);
  size_t o = 0;
  L.off_edges = o;
  o = align256(o + (size_t)(B + 1) * 8);
  L.off_binmap = o;
  o = align256(o + (size_t)padded * 2);
  L.off_f32 = o;
  o = align256(o + (size_t)padded * 4);
  L.off_counts = o;
  o = align256(o + (size_t)(B + 1) * 8);
  L.off_offsets = o;
  o = align256(o + (size_t)(B + 1) * 8);
  L.off_perm = o;
  o = align256(o + (size_t)N * 4);
  L.off_scratch = o;
  const size_t sort_scratch = (size_t)(B + 1) * (size_t)L.nblk * 4;
  const size_t run_scratch = (size_t)rowblocks * 4;
  const size_t scratch = sort_scratch > run_scratch ? sort_scratch : run_scratch;
  o = align256(o + scratch);
  L.off_tsum = o;  // tile sums of the prefix scans
  o = align256(o + (size_t)(scan_tiles((long long)(scratch / 4)) + 1) * 8);
  L.off_counters = o;
  o = align256(o + 8 * 8);
  L.off_runs = o;
  // up to one record per cell plus a terminator per row, and 128 records of
  // padding: the run sweep reads up to 79 records past a row segment's end
  o = align256(o + (size_t)(N + L.rows + 128) * 4);
  L.off_rowptr = o;
  o = align256(o + (size_t)(L.rows + 1) * 4);
  L.off_runidx = o;
  o = align256(o + (size_t)padded * 2);
  L.bytes = o;
  *out = L;
  return true;
}

// ---------------------------------------------------------------------------
// runs of equal bin along the fastest axis (a run-length form of the model
// matrix's rows). One thread per (row, 32-cell block).
// ---------------------------------------------------------------------------
struct RunArgs {
  const uint16_t* binmap;
  uint32_t* runs;
  int* rowptr;
  uint16_t* runidx;
  int* blockcnt;       // [rows * nb] counts, then exclusive positions
  unsigned long long* counters;
  long long rows;
  int nL, pitch, nb, none;
};

// the 32 bin codes of block q of a row (the row pitch is a multiple of 32
// cells, so a block is 64 aligned bytes: four 16-byte loads) and the code of
// the cell before it (0xFFFFFFFF for the row's first block, so cell 0 starts
// a run)
struct Block32 {
  uint32_t w[16];  // two codes per word, the lower column in the low half
  uint32_t prev;
};

__device__ __forceinline__ Block32 load_block32(const uint16_t* row, int q) {
  Block32 b;
  const uint4* p = reinterpret_cast<const uint4*>(row + q * 32);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint4 v = p[i];
    b.w[4 * i] = v.x;
    b.w[4 * i + 1] = v.y;
    b.w[4 * i + 2] = v.z;
    b.w[4 * i + 3] = v.w;
  }
  b.prev = q == 0 ? 0xFFFFFFFFu : (uint32_t)row[q * 32 - 1];
  return b;
}

__device__ __forceinline__ uint32_t code_at(const Block32& b, int j) {
  return (j & 1) ? (b.w[j >> 1] >> 16) : (b.w[j >> 1] & 0xFFFFu);
}

// bit j set when cell q*32 + j (a cell of the row) starts a run
__device__ __forceinline__ uint32_t run_starts(const Block32& b, int q, int nL) {
  uint32_t m = 0;
  uint32_t before = b.prev;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const uint32_t c = code_at(b, j);
    if (c != before && q * 32 + j < nL) m |= 1u << j;
    before = c;
  }
  return m;
}

__global__ __launch_bounds__(256) void k_runs_count(RunArgs a) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  unsigned long long real = 0;
  if (t < a.rows * a.nb) {
    const long long r = t / a.nb;
    const int q = (int)(t - r * a.nb);
    const Block32 blk = load_block32(a.binmap + r * a.pitch, q);
    int cnt = __popc(run_starts(blk, q, a.nL));
    real = cnt;
    if (q == a.nb - 1) ++cnt;  // terminator of the row
    a.blockcnt[t] = cnt;
  }
  for (int o = 32; o > 0; o >>= 1) real += __shfl_xor(real, o, 64);
  if ((threadIdx.x & 63) == 0 && real) atomicAdd(a.counters + kCntRuns, real);
}

__global__ __launch_bounds__(256) void k_runs_fill(RunArgs a) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.rows * a.nb) return;
  const long long r = t / a.nb;
  const int q = (int)(t - r * a.nb);
  const uint16_t* row = a.binmap + r * a.pitch;
  const Block32 blk = load_block32(row, q);
  const uint32_t starts = run_starts(blk, q, a.nL);
  const int rowstart = a.blockcnt[r * a.nb];
  int pos = a.blockcnt[t];
  if (q == 0) a.rowptr[r] = rowstart;
  int cur = pos - 1 - rowstart;  // run holding the cell before this block
  uint32_t idx[16];              // run indices of the 32 cells, two per word
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const int c = q * 32 + j;
    if ((starts >> j) & 1u) {
      a.runs[pos] = (uint32_t)c | (code_at(blk, j) << 16);
      cur = pos - rowstart;
      ++pos;
    } else if (c == a.nL) {
      // terminator: first column past the row, no bin
      a.runs[pos] = (uint32_t)a.nL | ((uint32_t)a.none << 16);
      cur = pos - rowstart;
      ++pos;
    }
    if (j & 1) idx[j >> 1] |= (uint32_t)(uint16_t)cur << 16;
    else idx[j >> 1] = (uint32_t)(uint16_t)cur;
  }
  uint4* out = reinterpret_cast<uint4*>(a.runidx + r * a.pitch + q * 32);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    out[i] = make_uint4(idx[4 * i], idx[4 * i + 1], idx[4 * i + 2], idx[4 * i + 3]);
  if (q == a.nb - 1 && a.nL == a.nb * 32) {
    // row length is a multiple of 32: terminator after the last block
    a.runs[pos] = (uint32_t)a.nL | ((uint32_t)a.none << 16);
  }
}

__global__ void k_rowptr_end(int* rowptr, long long rows, const int* total) {
  if (threadIdx.x == 0) rowptr[rows] = *total;
}

__global__ void k_set_mode(unsigned long long* counters, int mode) {
  if (threadIdx.x == 0) counters[kCntMode] = (unsigned long long)mode;
}

// zero the model matrix's counters (8 words) with a kernel rather than a
// memset, so that a caller may capture vup_bin in a graph
__global__ void k_clear_counters(unsigned long long* counters) {
  if (threadIdx.x < 8) counters[threadIdx.x] = 0ull;
}

hipError_t launch_clear_counters(void* counters, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, s,
                     static_cast<unsigned long long*>(counters));
  return hipGetLastError();
}

hipError_t launch_set_mode(const vup_mm& mm, int mode, hipStream_t s) {
  unsigned long long* c =
      reinterpret_cast<unsigned long long*>(static_cast<char*>(mm.ws) + mm.off_counters);
  hipLaunchKernelGGL(k_set_mode, dim3(1), dim3(64), 0, s, c, mode);
  return hipGetLastError();
}

hipError_t launch_runs(const vup_mm& mm, hipStream_t s) {
  char* ws = static_cast<char*>(mm.ws);
  RunArgs a{};
  a.binmap = reinterpret_cast<const uint16_t*>(ws + mm.off_binmap);
  a.runs = reinterpret_cast<uint32_t*>(ws + mm.off_runs);
  a.rowptr = reinterpret_cast<int*>(ws + mm.off_rowptr);
  a.runidx = reinterpret_cast<uint16_t*>(ws + mm.off_runidx);
  a.blockcnt = reinterpret_cast<int*>(ws + mm.off_scratch);
  a.counters = reinterpret_cast<unsigned long long*>(ws + mm.off_counters);
  a.rows = mm.rows;
  a.nL = mm.grid.n[mm.grid.ndim - 1];
  a.pitch = mm.pitch;
  a.nb = mm.pitch / 32;
  a.none = 4 * mm.B;
  const long long n = a.rows * a.nb;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_runs_count, dim3(blocks), dim3(256), 0, s, a);
  WsLayout L;
  ws_layout(mm.grid, mm.B, &L);
  const hipError_t err =
      launch_scan_excl(a.blockcnt, n, reinterpret_cast<long long*>(ws + L.off_tsum),
                       reinterpret_cast<int*>(a.counters + kCntScratch), s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_runs_fill, dim3(blocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_rowptr_end, dim3(1), dim3(64), 0, s, a.rowptr, a.rows,
                     reinterpret_cast<const int*>(a.counters + kCntScratch));
  return hipGetLastError();
}

}  // namespace vup
