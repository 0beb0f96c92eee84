// C ABI of the VUP/IPSA library: argument validation, workspace layout and
// kernel dispatch. Every check that can be done on the host happens here,
// before anything is enqueued.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "../../include/vup.h"
#include "vup_fields.hpp"
#include "vup_inverse.hpp"
#include "vup_internal.hpp"

static_assert(vup::kStaticMarginalBytes == (size_t)VUP_NOALLOC_SCRATCH_BYTES,
              "the header states the scratch array's size");

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int ok() {
  g_err[0] = '\0';
  return VUP_OK;
}

int check_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return fail(VUP_ENODEV, "no HIP device available");
  }
  return VUP_OK;
}

int launched(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(VUP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return ok();
}

int check_grid(const vup_grid* g) {
  if (!g) return fail(VUP_EINVAL, "grid is NULL");
  if (g->ndim < 1 || g->ndim > VUP_MAX_DIM) return fail(VUP_EINVAL, "ndim %d not in [1,4]", g->ndim);
  long long rows = 1, N = 1;
  for (int d = 0; d < g->ndim; ++d) {
    if (g->n[d] < 1 || g->n[d] > VUP_MAX_AXIS)
      return fail(VUP_EINVAL, "n[%d] = %d not in [1,%d]", d, g->n[d], VUP_MAX_AXIS);
    if (!std::isfinite(g->lo[d]) || !std::isfinite(g->hi[d]) || !(g->lo[d] < g->hi[d]))
      return fail(VUP_EINVAL, "axis %d: need finite lo < hi", d);
    N *= g->n[d];
    if (d + 1 < g->ndim) rows *= g->n[d];
  }
  const long long pitch = (g->n[g->ndim - 1] + 31) / 32 * 32;
  if (N > 0x7fffffffll || rows * pitch > 0x7fffffffll)
    return fail(VUP_EUNSUPPORTED, "grid of %lld cells exceeds the 2^31 cell limit", N);
  return VUP_OK;
}

int check_dists(const vup_dists* d, int ndim) {
  if (!d) return fail(VUP_EINVAL, "dists is NULL");
  if (d->K < 0) return fail(VUP_EINVAL, "K < 0");
  if (d->ncomp < 1 || d->ncomp > VUP_MAX_COMP)
    return fail(VUP_EINVAL, "ncomp %d not in [1,%d]", d->ncomp, VUP_MAX_COMP);
  if (d->ndim != ndim) return fail(VUP_EINVAL, "dists ndim %d != grid ndim %d", d->ndim, ndim);
  if (!(d->n_sigma > 0.0) || !std::isfinite(d->n_sigma))
    return fail(VUP_EINVAL, "n_sigma must be finite and > 0");
  if (d->K > 0 && (!d->mu || !d->sigma)) return fail(VUP_EINVAL, "mu/sigma is NULL");
  if (d->ncomp > 1 && d->K > 0 && !d->weight) return fail(VUP_EINVAL, "mixtures need weights");
  if (d->ncomp == 1 && d->weight) return fail(VUP_EINVAL, "weight must be NULL when ncomp == 1");
  if (d->K * d->ncomp > 0x7fffffffll * 8ll) return fail(VUP_EUNSUPPORTED, "K too large");
  return VUP_OK;
}

int check_mm(const vup_mm* mm) {
  if (!mm) return fail(VUP_EINVAL, "model matrix descriptor is NULL");
  if (mm->magic != vup::kMagic || !mm->ws)
    return fail(VUP_EWORKSPACE, "descriptor was not produced by vup_bin");
  int r = check_grid(&mm->grid);
  if (r) return r;
  return VUP_OK;
}

int check_sweep(const vup_mm* mm, vup::SweepKind kind) {
  vup::SweepLayout L;
  if (!vup::sweep_layout(mm->grid, mm->B, kind, &L))
    return fail(VUP_EUNSUPPORTED, "grid axes too long for on-chip factor tables (%zu bytes LDS)",
                L.bytes);
  return VUP_OK;
}

int check_model(const vup_model* m, int ndim) {
  if (!m) return fail(VUP_EINVAL, "model is NULL");
  const int need[] = {0, 2, 3, 4, 2, 2};
  if (m->kind < 0 || m->kind > VUP_MODEL_IPSA2) return fail(VUP_EINVAL, "unknown model %d", m->kind);
  if (m->kind == VUP_MODEL_LINEAR) {
    for (int d = 0; d <= ndim; ++d)
      if (!std::isfinite(m->theta[d])) return fail(VUP_EINVAL, "theta must be finite");
  } else if (need[m->kind] != ndim) {
    return fail(VUP_EINVAL, "model %d needs ndim %d", m->kind, need[m->kind]);
  }
  return VUP_OK;
}

}  // namespace

extern "C" {

const char* vup_last_error(void) { return g_err; }

const char* vup_version(void) { return "vup-mi355x 0.1 (gfx950)"; }

int vup_eval_grid(const vup_grid* g, const vup_model* m, double* f, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (!m || !f) return fail(VUP_EINVAL, "model or f is NULL");
  if ((r = check_model(m, g->ndim))) return r;
  if ((r = check_device())) return r;
  return launched(vup::launch_eval_grid(*g, *m, f, (hipStream_t)stream), "vup_eval_grid");
}

int vup_uniform_edges(const double* f, int64_t N, int32_t B, double* edges, void* stream) {
  if (!f || !edges) return fail(VUP_EINVAL, "f or edges is NULL");
  if (N < 1) return fail(VUP_EINVAL, "N < 1");
  if (B < 1 || B > VUP_MAX_BINS) return fail(VUP_EINVAL, "B %d not in [1,%d]", B, VUP_MAX_BINS);
  int r = check_device();
  if (r) return r;
  return launched(vup::launch_uniform_edges(f, N, B, edges, (hipStream_t)stream),
                  "vup_uniform_edges");
}

size_t vup_bin_workspace_bytes(const vup_grid* g, int32_t B) {
  if (check_grid(g) || B < 1 || B > VUP_MAX_BINS) return 0;
  vup::WsLayout L;
  vup::ws_layout(*g, B, &L);
  return L.bytes;
}

int vup_bin(const vup_grid* g, const double* f, const double* edges, int32_t B, int32_t* bin,
            void* ws, size_t ws_bytes, vup_mm* mm_out, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if (B < 1 || B > VUP_MAX_BINS) return fail(VUP_EINVAL, "B %d not in [1,%d]", B, VUP_MAX_BINS);
  if (!f || !edges || !mm_out) return fail(VUP_EINVAL, "f, edges or mm_out is NULL");
  if (!ws) return fail(VUP_EWORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(VUP_EWORKSPACE, "workspace not 256-byte aligned");
  vup::WsLayout L;
  vup::ws_layout(*g, B, &L);
  if (ws_bytes < L.bytes)
    return fail(VUP_EWORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, L.bytes);
  if ((r = check_device())) return r;
  vup_mm mm;
  memset(&mm, 0, sizeof mm);
  mm.grid = *g;
  for (int d = g->ndim; d < 4; ++d) {
    mm.grid.n[d] = 1;
    mm.grid.lo[d] = 0.0;
    mm.grid.hi[d] = 1.0;
  }
  mm.B = B;
  mm.pitch = L.pitch;
  mm.rows = L.rows;
  mm.N = L.rows * g->n[g->ndim - 1];
  mm.ws = ws;
  mm.ws_bytes = ws_bytes;
  mm.off_edges = L.off_edges;
  mm.off_binmap = L.off_binmap;
  mm.off_f32 = L.off_f32;
  mm.off_counts = L.off_counts;
  mm.off_offsets = L.off_offsets;
  mm.off_perm = L.off_perm;
  mm.off_scratch = L.off_scratch;
  mm.off_counters = L.off_counters;
  mm.off_runs = L.off_runs;
  mm.off_rowptr = L.off_rowptr;
  mm.off_runidx = L.off_runidx;
  mm.sweep = VUP_SWEEP_AUTO;
  mm.reserved = 0;
  mm.magic = vup::kMagic;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = vup::launch_clear_counters(static_cast<char*>(ws) + L.off_counters, s);
  if (e != hipSuccess) return launched(e, "vup_bin (clear counters)");
  e = vup::launch_bin(mm, f, edges, bin, s);
  if (e != hipSuccess) return launched(e, "vup_bin");
  *mm_out = mm;
  return ok();
}

int vup_windows(const vup_grid* g, const vup_dists* d, int32_t* win, void* stream) {
  int r = check_grid(g);
  if (r) return r;
  if ((r = check_dists(d, g->ndim))) return r;
  if (d->K > 0 && !win) return fail(VUP_EINVAL, "win is NULL");
  if ((r = check_device())) return r;
  return launched(vup::launch_windows(*g, *d, win, (hipStream_t)stream), "vup_windows");
}

int vup_propagate(const vup_mm* mm, const vup_dists* d, int32_t precision, float* P, double* Z,
                  void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if ((r = check_dists(d, mm->grid.ndim))) return r;
  if (precision < VUP_FP32 || precision > VUP_FP8E4M3)
    return fail(VUP_EINVAL, "unknown precision %d", precision);
  if (d->K > 0 && !P) return fail(VUP_EINVAL, "P is NULL");
  if ((r = check_sweep(mm, vup::kSweepPropagate))) return r;
  if ((r = check_device())) return r;
  return launched(vup::launch_propagate(*mm, *d, precision, P, Z, (hipStream_t)stream),
                  "vup_propagate");
}

size_t vup_separable_workspace_bytes(const vup_mm* mm, int32_t Mx, int32_t My) {
  if (check_mm(mm) || mm->grid.ndim != 2 || Mx < 1 || My < 1) return 0;
  return vup::sep_workspace_bytes(mm->grid, mm->B, Mx, My);
}

int vup_propagate_separable(const vup_mm* mm, const vup_sepdists* s, void* ws, size_t ws_bytes,
                            float* P, double* Z, void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if (mm->grid.ndim != 2) return fail(VUP_EUNSUPPORTED, "separable form needs a 2-D grid");
  if (mm->B > 512 && mm->grid.n[1] > 65534)
    return fail(VUP_EUNSUPPORTED, "separable form needs B <= 512 when n[1] > 65534");
  if (!s) return fail(VUP_EINVAL, "sepdists is NULL");
  if (s->M[0] < 1 || s->M[1] < 1 || s->M[0] > 65535 || s->M[1] > 65535)
    return fail(VUP_EINVAL, "M must be in [1, 65535]");
  if (!(s->n_sigma > 0.0) || !std::isfinite(s->n_sigma))
    return fail(VUP_EINVAL, "n_sigma must be finite and > 0");
  if (!s->mu[0] || !s->mu[1] || !s->sigma[0] || !s->sigma[1] || !P)
    return fail(VUP_EINVAL, "mu, sigma or P is NULL");
  if (s->precision != VUP_FP32 && s->precision != VUP_BF16 && s->precision != VUP_BF16X2)
    return fail(VUP_EINVAL, "separable precision %d: VUP_FP32, VUP_BF16 or VUP_BF16X2",
                s->precision);
  if (!ws) return fail(VUP_EWORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(VUP_EWORKSPACE, "workspace not 256-byte aligned");
  const size_t need = vup::sep_workspace_bytes(mm->grid, mm->B, s->M[0], s->M[1]);
  if (ws_bytes < need) return fail(VUP_EWORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, need);
  // families with fewer than 16 locations along y go through the general sweep
  if (s->M[1] < 16 && (r = check_sweep(mm, vup::kSweepPropagate))) return r;
  if ((r = check_device())) return r;
  return launched(vup::launch_separable(*mm, s->M[0], s->M[1], s->mu[0], s->mu[1], s->sigma[0],
                                        s->sigma[1], s->n_sigma, s->precision, ws, P, Z,
                                        (hipStream_t)stream),
                  "vup_propagate_separable");
}

int vup_moments(const vup_mm* mm, const vup_dists* d, const vup_model* model, double* mean,
                double* var, double* delta2, void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if ((r = check_dists(d, mm->grid.ndim))) return r;
  if (d->K > 0 && (!mean || !var)) return fail(VUP_EINVAL, "mean or var is NULL");
  if (delta2) {
    if (d->ncomp != 1) return fail(VUP_EUNSUPPORTED, "delta2 needs single-component pdfs");
    if (!model) return fail(VUP_EINVAL, "delta2 needs the built-in model");
    // the kernel evaluates the model at mu with the grid's ndim coordinates
    if ((r = check_model(model, mm->grid.ndim))) return r;
  }
  if ((r = check_sweep(mm, vup::kSweepMoments))) return r;
  if ((r = check_device())) return r;
  return launched(vup::launch_moments(*mm, *d, delta2 ? model : nullptr, mean, var, delta2,
                                      (hipStream_t)stream),
                  "vup_moments");
}

size_t vup_moments_tiled_workspace_bytes(const vup_mm* mm, const vup_dists* d) {
  if (check_mm(mm) || check_dists(d, mm->grid.ndim)) return 0;
  if (!vup::moments_tiled_applies(*mm, *d)) return 0;
  return vup::moments_tiled_ws_bytes(*mm, d->K);
}

int vup_moments_tiled(const vup_mm* mm, const vup_dists* d, const vup_model* model, void* ws,
                      size_t ws_bytes, double* mean, double* var, double* delta2, void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if ((r = check_dists(d, mm->grid.ndim))) return r;
  if (!vup::moments_tiled_applies(*mm, *d))
    return vup_moments(mm, d, model, mean, var, delta2, stream);
  if (d->K > 0 && (!mean || !var)) return fail(VUP_EINVAL, "mean or var is NULL");
  if (delta2) {
    if (!model) return fail(VUP_EINVAL, "delta2 needs the built-in model");
    if ((r = check_model(model, mm->grid.ndim))) return r;
  }
  const size_t need = vup::moments_tiled_ws_bytes(*mm, d->K);
  if (d->K > 0) {
    if (!ws) return fail(VUP_EWORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(VUP_EWORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < need) return fail(VUP_EWORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, need);
  }
  if ((r = check_device())) return r;
  return launched(vup::launch_moments_tiled(*mm, *d, delta2 ? model : nullptr, ws, mean, var,
                                            delta2, (hipStream_t)stream),
                  "vup_moments_tiled");
}

int vup_ipsa(const vup_mm* mm, int64_t K, const float* P, double* mean_hist, double* var,
             double* entropy, void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if (K < 0) return fail(VUP_EINVAL, "K < 0");
  if (K > 0 && !P) return fail(VUP_EINVAL, "P is NULL");
  if ((r = check_device())) return r;
  const double* edges =
      reinterpret_cast<const double*>(static_cast<const char*>(mm->ws) + mm->off_edges);
  return launched(
      vup::launch_ipsa_stats(edges, mm->B, K, P, mean_hist, var, entropy, (hipStream_t)stream),
      "vup_ipsa");
}

int vup_ipsa_backward(const vup_mm* mm, const vup_dists* d, const float* P,
                      const double* mean_hist, const double* g_var, const double* g_ent,
                      double* g_mu, double* g_sigma, double* g_weight, void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if ((r = check_dists(d, mm->grid.ndim))) return r;
  if (d->K > 0 && (!P || !mean_hist || !g_mu || !g_sigma))
    return fail(VUP_EINVAL, "P, mean_hist, g_mu or g_sigma is NULL");
  if ((r = check_sweep(mm, vup::kSweepBackward))) return r;
  if ((r = check_device())) return r;
  return launched(vup::launch_backward(*mm, *d, P, mean_hist, g_var, g_ent, g_mu, g_sigma, g_weight,
                                       (hipStream_t)stream),
                  "vup_ipsa_backward");
}

int vup_set_sweep_mode(vup_mm* mm, int32_t mode, void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if (mode < VUP_SWEEP_AUTO || mode > VUP_SWEEP_RUNS) return fail(VUP_EINVAL, "unknown mode %d", mode);
  if ((r = check_device())) return r;
  hipStream_t s = (hipStream_t)stream;
  if (mode == VUP_SWEEP_AUTO) {
    // resolve now from the run count vup_bin left in the counters
    const char* c = static_cast<const char*>(mm->ws) + mm->off_counters;
    int64_t nruns = 0;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess)
      e = hipMemcpy(&nruns, c + vup::kCntRuns * sizeof(int64_t), sizeof(nruns),
                    hipMemcpyDeviceToHost);
    if (e != hipSuccess) return launched(e, "vup_set_sweep_mode");
    const bool runs = vup::runs_allowed(*mm) && nruns > 0 && nruns * vup::kRunMinLength <= mm->N;
    mode = runs ? VUP_SWEEP_RUNS : VUP_SWEEP_CELLS;
  }
  mm->sweep = mode;
  return launched(vup::launch_set_mode(*mm, mode, s), "vup_set_sweep_mode");
}

int vup_eval_points(const vup_model* m, int32_t ndim, int64_t n, const double* x, int64_t ldx,
                    double* y, void* stream) {
  if (ndim < 1 || ndim > VUP_MAX_DIM) return fail(VUP_EINVAL, "ndim %d not in [1,4]", ndim);
  int r = check_model(m, ndim);
  if (r) return r;
  if (n < 0) return fail(VUP_EINVAL, "n < 0");
  if (ldx < ndim) return fail(VUP_EINVAL, "ldx %lld < ndim %d", (long long)ldx, ndim);
  if (n > 0 && (!x || !y)) return fail(VUP_EINVAL, "x or y is NULL");
  if (n > 0 && ldx > (int64_t)1 << 40) return fail(VUP_EUNSUPPORTED, "ldx too large");
  if ((r = check_device())) return r;
  return launched(vup::launch_eval_points(*m, ndim, n, x, ldx, y, (hipStream_t)stream),
                  "vup_eval_points");
}

int vup_ipsa_matrix(const vup_mm* mm, int64_t K, const float* P, const double* y_ref, double dy_lo,
                    double dy_width, int32_t n_dy, float* Q, double* lost, void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if (K < 0) return fail(VUP_EINVAL, "K < 0");
  if (n_dy < 1 || n_dy > VUP_MAX_DY) return fail(VUP_EINVAL, "n_dy %d not in [1,%d]", n_dy, VUP_MAX_DY);
  if (!std::isfinite(dy_lo) || !std::isfinite(dy_width) || !(dy_width > 0.0) ||
      !std::isfinite(dy_lo + (double)n_dy * dy_width))
    return fail(VUP_EINVAL, "Delta-y grid needs finite dy_lo and dy_width > 0");
  if (K > 0 && (!P || !y_ref || !Q)) return fail(VUP_EINVAL, "P, y_ref or Q is NULL");
  if ((r = check_device())) return r;
  const double* edges =
      reinterpret_cast<const double*>(static_cast<const char*>(mm->ws) + mm->off_edges);
  return launched(vup::launch_ipsa_matrix(edges, mm->B, K, P, y_ref, dy_lo, dy_width, n_dy, Q, lost,
                                          (hipStream_t)stream),
                  "vup_ipsa_matrix");
}

int vup_ipsa_fields(const vup_mm* mm, int64_t K, const float* P, const double* y_ref,
                    int32_t n_levels, const double* levels, double* y_mode, double* p_max,
                    double* quant, double* dev, double* delta2, void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if (K < 0) return fail(VUP_EINVAL, "K < 0");
  if (n_levels < 0 || n_levels > VUP_MAX_LEVELS)
    return fail(VUP_EINVAL, "n_levels %d not in [0,%d]", n_levels, VUP_MAX_LEVELS);
  if (quant && n_levels == 0) return fail(VUP_EINVAL, "quant given but n_levels == 0");
  if (n_levels > 0 && !levels) return fail(VUP_EINVAL, "levels is NULL");
  for (int q = 0; q < n_levels; ++q)
    if (!(levels[q] > 0.0 && levels[q] <= 1.0))
      return fail(VUP_EINVAL, "level %d = %g not in (0, 1]", q, levels[q]);
  if ((dev || delta2) && !y_ref) return fail(VUP_EINVAL, "dev and delta2 need y_ref");
  if (K > 0 && !P) return fail(VUP_EINVAL, "P is NULL");
  if ((r = check_device())) return r;
  const double* edges =
      reinterpret_cast<const double*>(static_cast<const char*>(mm->ws) + mm->off_edges);
  return launched(vup::launch_ipsa_fields(edges, mm->B, K, P, y_ref, n_levels, levels, y_mode, p_max,
                                          quant, dev, delta2, (hipStream_t)stream),
                  "vup_ipsa_fields");
}

size_t vup_marginal_workspace_bytes(int64_t K, int32_t n) {
  if (K < 0 || n < 1 || n > VUP_MAX_MARGINAL_COLS) return 0;
  return vup::marginal_workspace_bytes(K, n);
}

int vup_marginalize(int64_t K, int32_t n, const float* A, const double* rho, void* ws,
                    size_t ws_bytes, double* out, void* stream) {
  if (K < 0) return fail(VUP_EINVAL, "K < 0");
  if (n < 1 || n > VUP_MAX_MARGINAL_COLS)
    return fail(VUP_EINVAL, "n %d not in [1,%d]", n, VUP_MAX_MARGINAL_COLS);
  if (!out || (K > 0 && !A)) return fail(VUP_EINVAL, "A or out is NULL");
  const size_t need = vup::marginal_workspace_bytes(K, n);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(VUP_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  int r = check_device();
  if (r) return r;
  return launched(vup::launch_marginalize(K, n, A, rho, ws, out, (hipStream_t)stream),
                  "vup_marginalize");
}

int vup_marginalize_noalloc(int64_t K, int32_t n, const float* A, const double* rho,
                            double* out, void* stream) {
  if (K < 0) return fail(VUP_EINVAL, "K < 0");
  if (n < 1 || n > VUP_MAX_MARGINAL_COLS)
    return fail(VUP_EINVAL, "n %d not in [1,%d]", n, VUP_MAX_MARGINAL_COLS);
  if (!out || (K > 0 && !A)) return fail(VUP_EINVAL, "A or out is NULL");
  const size_t need = vup::marginal_workspace_bytes(K, n);
  if (need > VUP_NOALLOC_SCRATCH_BYTES)
    return fail(VUP_EUNSUPPORTED,
                "partial sums of %zu bytes exceed the library's %d-byte scratch array "
                "(use vup_marginalize with a workspace)",
                need, VUP_NOALLOC_SCRATCH_BYTES);
  int r = check_device();
  if (r) return r;
  return launched(vup::launch_marginalize_static(K, n, A, rho, out, (hipStream_t)stream),
                  "vup_marginalize_noalloc");
}

int vup_posterior(const vup_mm* mm, const vup_dists* d, int64_t n_sel, const int64_t* sel,
                  const float* P, const double* Z, float* post, double* mean, void* stream) {
  int r = check_mm(mm);
  if (r) return r;
  if ((r = check_dists(d, mm->grid.ndim))) return r;
  if (n_sel < 0) return fail(VUP_EINVAL, "n_sel < 0");
  if (n_sel > 65535) return fail(VUP_EUNSUPPORTED, "n_sel %lld > 65535", (long long)n_sel);
  if (n_sel > 0 && (!sel || !P || !Z || !post))
    return fail(VUP_EINVAL, "sel, P, Z or post is NULL");
  if ((r = check_device())) return r;
  return launched(vup::launch_posterior(*mm, *d, n_sel, sel, P, Z, post, mean, (hipStream_t)stream),
                  "vup_posterior");
}

int vup_counters(const vup_mm* mm, void* stream, int64_t* out) {
  int r = check_mm(mm);
  if (r) return r;
  if (!out) return fail(VUP_EINVAL, "out is NULL");
  if ((r = check_device())) return r;
  hipStream_t s = (hipStream_t)stream;
  char* c = static_cast<char*>(mm->ws) + mm->off_counters;
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(out, c, 4 * sizeof(int64_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemsetAsync(c, 0, 4 * sizeof(int64_t), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return launched(e, "vup_counters");
}

}  // extern "C"
