// Host-side interfaces between the C ABI layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/vup.h"
#include "vup_device.hpp"

namespace vup {

constexpr uint64_t kMagic = 0x5655504d4d763031ull;  // "VUPMMv01"

// LDS layout of a sweep kernel (offsets in floats from the start of dynamic LDS)
struct SweepLayout {
  int tab_off[4];
  int cap[4];
  int row_off;      // row table: [rrows] / [kBwdRowChunk] entries in the run forms, [kRowChunk] in the cell forms
  int rrows;        // rows per row-table pass of the propagation (run and cell forms)
  int trow_off;     // float4[kRowChunk] (backward only, else -1)
  int hist_off;     // histogram copies (propagate) or v table (backward)
  int hist_stride;  // floats per histogram copy (run form); words of all copies (cell form)
  int cpw;          // histogram copies (cell form: interleaved by bin, a power of two)
  int cshift;       // log2(cpw) (cell form)
  int ncls;         // magnitude classes (1 in the cell form, 3 in the run form)
  int red_off;      // double scratch
  int g_off;        // FP64 prefix sums of the fastest-axis factors (run form)
  size_t bytes;
};

enum SweepKind {
  kSweepPropagate = 0,
  kSweepMoments = 1,
  kSweepBackward = 2,
  kSweepRuns = 3,
  kSweepBwdRuns = 4
};

// run_rows: rows per row-table pass of the run-form propagation (0: the
// default, kRunRowChunk)
bool sweep_layout(const vup_grid& g, int B, SweepKind kind, SweepLayout* out, int run_rows = 0);
GridDev make_grid_dev(const vup_mm& mm);
DistsDev make_dists_dev(const vup_dists& d);

// launches (return hipError_t of the launch)
hipError_t launch_eval_grid(const vup_grid& g, const vup_model& m, double* f, hipStream_t s);
hipError_t launch_uniform_edges(const double* f, int64_t N, int B, double* edges, hipStream_t s);
hipError_t launch_bin(const vup_mm& mm, const double* f, const double* edges, int32_t* bin,
                      hipStream_t s);
hipError_t launch_windows(const vup_grid& g, const vup_dists& d, int32_t* win, hipStream_t s);
hipError_t launch_propagate(const vup_mm& mm, const vup_dists& d, int prec, float* P, double* Z,
                            hipStream_t s);
hipError_t launch_moments(const vup_mm& mm, const vup_dists& d, const vup_model* model,
                          double* mean, double* var, double* delta2, hipStream_t s);
// moments by tiles of the model values on the matrix cores (2-D grids,
// single-component pdfs, at most 256 tiles of 64 cells per axis)
bool moments_tiled_applies(const vup_mm& mm, const vup_dists& d);
size_t moments_tiled_ws_bytes(const vup_mm& mm, long long K);
hipError_t launch_moments_tiled(const vup_mm& mm, const vup_dists& d, const vup_model* model,
                                void* ws, double* mean, double* var, double* delta2,
                                hipStream_t s);
hipError_t launch_backward(const vup_mm& mm, const vup_dists& d, const float* P,
                           const double* mean_hist, const double* g_var, const double* g_ent,
                           double* g_mu, double* g_sigma, double* g_weight, hipStream_t s);

hipError_t launch_set_mode(const vup_mm& mm, int mode, hipStream_t s);
// zero the 64 bytes of counters at `counters` (device, 8-byte aligned)
hipError_t launch_clear_counters(void* counters, hipStream_t s);
// the run form of the FP32 propagation applies to this model matrix
bool runs_allowed(const vup_mm& mm);
size_t sep_workspace_bytes(const vup_grid& g, int B, int Mx, int My);
hipError_t launch_separable(const vup_mm& mm, int Mx, int My, const double* mu_x,
                            const double* mu_y, const double* sg_x, const double* sg_y,
                            double ns, int prec, void* ws, float* P, double* Z, hipStream_t s);

// workspace sizing shared by vup_bin_workspace_bytes and vup_bin
struct WsLayout {
  int pitch;
  int64_t rows;
  int64_t nblk;  // chunks of the bin sort
  int chunk;     // padded positions per chunk
  size_t off_edges, off_binmap, off_f32, off_counts, off_offsets, off_perm, off_scratch,
      off_counters, off_runs, off_rowptr, off_runidx, off_tsum, bytes;
};
bool ws_layout(const vup_grid& g, int B, WsLayout* out);
// exclusive prefix sum of n ints in place; tsum: scan_tiles(n) int64 scratch;
// total (device int) may be null
long long scan_tiles(long long n);
hipError_t launch_scan_excl(int* v, long long n, long long* tsum, int* total, hipStream_t s);

}  // namespace vup
