/*
 * Plain FP64 CPU oracle for Vectorized Uncertainty Propagation (VUP) and
 * Input Probability Sensitivity Analysis (IPSA), arXiv:1908.11246.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path links, loads or calls
 * this file; it exists so the GPU library can be checked against a slow,
 * obviously correct computation written straight from the paper. It shares no
 * source, header, table or helper with the GPU library.
 *
 * Conventions (each one is restated where it is used):
 *  - Grid: uniform, cell centred (composite midpoint rule, Sec. 3 and Alg. VUP
 *    "generate a uniform grid"): x_{d,j} = lo_d + (j + 1/2) * ((hi_d - lo_d)/n_d).
 *    Flat cell index is row major, axis 0 slowest.
 *  - Bins partition the output range (Sec. 3, eq. (4): the bin widths
 *    "uniformly partition" the output; one nonzero per model-matrix column):
 *    bin(i) = largest b < B with e_b <= f_i, provided f_i <= e_B; otherwise -1
 *    (also for NaN). The last bin is closed.
 *  - Input pdf: Gaussian (Sec. 5.2, eq. gaussh) evaluated at cell centres and
 *    normalised over the kept cells (Alg. VUP, "evaluate the input pdf ... and
 *    normalize"); kept cells = per-axis box |x_d - mu_d| <= n_sigma*sigma_d,
 *    intersected with the grid (truncation as in Sec. 5.3).
 *  - Propagation: P[b,k] = sum_i [bin(i) = b] p_k(x_i)  (eq. (5), eq. VUP).
 *  - Floating point: FP64 everywhere, built with -ffp-contract=off, sums use
 *    Neumaier compensation.
 *
 * Parity of every function here is pinned by tests/test_oracle_pins.py against
 * closed forms, brute force and library routines.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* compensated summation                                                     */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;

static inline void ks_add(ksum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static inline double ks_val(const ksum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* grid                                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int ndim;
  int n[4];
  double lo[4], hi[4];
} og_grid;

static og_grid make_grid(int ndim, const int *n, const double *lo, const double *hi) {
  og_grid g;
  memset(&g, 0, sizeof g);
  g.ndim = ndim;
  for (int d = 0; d < ndim; ++d) { g.n[d] = n[d]; g.lo[d] = lo[d]; g.hi[d] = hi[d]; }
  return g;
}

/* cell width of axis d */
static inline double cell_h(const og_grid *g, int d) { return (g->hi[d] - g->lo[d]) / g->n[d]; }

/* cell centre x_{d,j} (composite midpoint rule) */
static inline double cell_x(const og_grid *g, int d, int j) {
  return g->lo[d] + (j + 0.5) * cell_h(g, d);
}

static long grid_cells(const og_grid *g) {
  long N = 1;
  for (int d = 0; d < g->ndim; ++d) N *= g->n[d];
  return N;
}

/* ------------------------------------------------------------------------ */
/* models  M(x) = y  (Sec. 2, eq. modelfunction). Scalar outputs only.       */
/* ------------------------------------------------------------------------ */
enum {
  OM_LINEAR = 0,  /* theta0 + sum_d theta_{d+1} x_d                           */
  OM_SINCOS2 = 1, /* sin x0 + 0.5 cos(2 x1) + x0 x1 / 4                        */
  OM_DAMPED3 = 2, /* exp(-0.1 x2) sin x0 cos x1 + 0.1 x0 x1 x2                 */
  OM_RING4 = 3,   /* sum_j sin(x_j) x_{j+1 mod 4} + 0.05 (sum_j x_j)^2         */
  OM_TIMING2 = 4, /* 1.1 sin x + 7 sin^2 alpha   (Sec. 4.1 timing model)       */
  OM_IPSA2 = 5    /* x^2 + 5 sin 3x + alpha      (Sec. 5.3 IPSA example)       */
};

/* evaluate model at point x[ndim]; returns NaN for an unknown model/ndim pair */
double orc_model_at(int kind, int ndim, const double *theta, const double *x) {
  switch (kind) {
    case OM_LINEAR: {
      double y = theta[0];
      for (int d = 0; d < ndim; ++d) y += theta[d + 1] * x[d];
      return y;
    }
    case OM_SINCOS2:
      if (ndim != 2) break;
      return sin(x[0]) + 0.5 * cos(2.0 * x[1]) + x[0] * x[1] / 4.0;
    case OM_DAMPED3:
      if (ndim != 3) break;
      return exp(-0.1 * x[2]) * sin(x[0]) * cos(x[1]) + 0.1 * x[0] * x[1] * x[2];
    case OM_RING4: {
      if (ndim != 4) break;
      double s = 0.0, t = 0.0;
      for (int j = 0; j < 4; ++j) s += sin(x[j]) * x[(j + 1) % 4];
      for (int j = 0; j < 4; ++j) t += x[j];
      return s + 0.05 * (t * t);
    }
    case OM_TIMING2:
      if (ndim != 2) break;
      {
        double sa = sin(x[1]);
        return 1.1 * sin(x[0]) + 7.0 * (sa * sa);
      }
    case OM_IPSA2:
      if (ndim != 2) break;
      return x[0] * x[0] + 5.0 * sin(3.0 * x[0]) + x[1];
    default:
      break;
  }
  return NAN;
}

/* decode flat index into per-axis indices (row major, axis 0 slowest) */
static inline void unflatten(const og_grid *g, long i, int *j) {
  for (int d = g->ndim - 1; d >= 0; --d) { j[d] = (int)(i % g->n[d]); i /= g->n[d]; }
}

/* Alg. VUP: "generate a uniform grid", "evaluate the model" -> f[N] */
int orc_eval_grid(int ndim, const int *n, const double *lo, const double *hi,
                  int kind, const double *theta, double *f) {
  og_grid g = make_grid(ndim, n, lo, hi);
  long N = grid_cells(&g);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    int j[4];
    double x[4];
    unflatten(&g, i, j);
    for (int d = 0; d < ndim; ++d) x[d] = cell_x(&g, d, j[d]);
    f[i] = orc_model_at(kind, ndim, theta, x);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* bins                                                                      */
/* ------------------------------------------------------------------------ */

/* B uniform bins over [min f, max f] (the harness's edge rule):
 * e_b = lo + b * ((hi - lo) / B) for b < B and e_B = hi exactly. */
void orc_uniform_edges(const double *f, long N, int B, double *edges) {
  double lo = INFINITY, hi = -INFINITY;
  for (long i = 0; i < N; ++i) {
    if (f[i] != f[i]) continue;
    if (f[i] < lo) lo = f[i];
    if (f[i] > hi) hi = f[i];
  }
  double w = (hi - lo) / B;
  for (int b = 0; b < B; ++b) edges[b] = lo + b * w;
  edges[B] = hi;
}

/* indicator Theta of eq. (4) as a bin index: largest b < B with e_b <= y,
 * valid when e_0 <= y <= e_B; -1 otherwise (NaN included). Linear scan. */
static int bin_of(double y, const double *e, int B) {
  if (!(y >= e[0] && y <= e[B])) return -1;
  int b = 0;
  while (b + 1 < B && e[b + 1] <= y) ++b;
  return b;
}

void orc_bin(const double *f, long N, const double *edges, int B, int *bin) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) bin[i] = bin_of(f[i], edges, B);
}

/* Sparse model matrix of eq. (5)/(MUP) in compressed form: for each bin b the
 * list of cells in increasing cell order (one nonzero per column).
 * offsets[B+1], perm[number of binned cells]. Cells with bin -1 are absent. */
void orc_model_matrix(const int *bin, long N, int B, long *offsets, long *perm) {
  for (int b = 0; b <= B; ++b) offsets[b] = 0;
  for (long i = 0; i < N; ++i)
    if (bin[i] >= 0) offsets[bin[i] + 1]++;
  for (int b = 0; b < B; ++b) offsets[b + 1] += offsets[b];
  long *fill = (long *)malloc(sizeof(long) * (size_t)B);
  for (int b = 0; b < B; ++b) fill[b] = offsets[b];
  for (long i = 0; i < N; ++i)
    if (bin[i] >= 0) perm[fill[bin[i]]++] = i;
  free(fill);
}

/* ------------------------------------------------------------------------ */
/* truncation windows                                                        */
/* ------------------------------------------------------------------------ */

/* Kept cells of one axis for a Gaussian centred at mu with deviation sigma:
 * all j with |x_j - mu| <= ns*sigma, evaluated as
 *   t_lo = ((mu - ns*sigma) - lo)/h - 1/2,   j_lo = max(0, ceil(t_lo))
 *   t_hi = ((mu + ns*sigma) - lo)/h - 1/2,   j_hi = min(n-1, floor(t_hi))
 * If that range is empty but mu lies in [lo, hi], the window is the single
 * cell containing mu (a pdf narrower than a cell, e.g. the delta input of
 * eq. (1)). Otherwise the window is empty (j_lo = 0, j_hi = -1).
 * Returns 0 on success, 1 for invalid parameters (sigma <= 0 or non-finite). */
static int axis_window(double lo, double hi, int n, double mu, double sigma, double ns,
                       int *jlo, int *jhi) {
  if (!(sigma > 0.0) || !isfinite(sigma) || !isfinite(mu)) { *jlo = 0; *jhi = -1; return 1; }
  double h = (hi - lo) / n;
  double tlo = ((mu - ns * sigma) - lo) / h - 0.5;
  double thi = ((mu + ns * sigma) - lo) / h - 0.5;
  double a = ceil(tlo), b = floor(thi);
  if (a < 0.0) a = 0.0;
  if (b > (double)(n - 1)) b = (double)(n - 1);
  if (a > b) {
    if (mu >= lo && mu <= hi) {
      double c = floor((mu - lo) / h);
      if (c < 0.0) c = 0.0;
      if (c > (double)(n - 1)) c = (double)(n - 1);
      a = b = c;
    } else {
      *jlo = 0; *jhi = -1; return 0;
    }
  }
  *jlo = (int)a;
  *jhi = (int)b;
  return 0;
}

/* windows for all (k, c): win[((k*C + c)*ndim + d)*2 + {0,1}], bad[k*C+c].
 * Returns the number of cell-distribution pairs sum_{k,c} |W_{k,c}|. */
long orc_windows(int ndim, const int *n, const double *lo, const double *hi,
                 long K, int C, const double *mu, const double *sigma, double ns,
                 int *win, int *bad) {
  long U = 0;
  for (long kc = 0; kc < K * C; ++kc) {
    int isbad = 0;
    long cells = 1;
    for (int d = 0; d < ndim; ++d) {
      int a, b;
      isbad |= axis_window(lo[d], hi[d], n[d], mu[kc * ndim + d], sigma[kc * ndim + d], ns, &a, &b);
      win[(kc * ndim + d) * 2 + 0] = a;
      win[(kc * ndim + d) * 2 + 1] = b;
      cells *= (b >= a) ? (long)(b - a + 1) : 0;
    }
    if (bad) bad[kc] = isbad;
    if (!isbad) U += cells;
  }
  return U;
}

/* ------------------------------------------------------------------------ */
/* density quantisers for the reduced-precision variants                     */
/* ------------------------------------------------------------------------ */
enum { OP_FP64 = -1, OP_FP32 = 0, OP_BF16 = 1, OP_BF16X2 = 2, OP_FP8E4M3 = 3 };

/* round to the nearest bfloat16 (8 significant bits), ties to even */
double orc_round_bf16(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  double m = frexp(x, &e);            /* x = m 2^e, 0.5 <= |m| < 1 */
  double r = nearbyint(ldexp(m, 8));  /* 8 significant bits, default RNE */
  return ldexp(r, e - 8);
}

/* round a value in [0, 448] to the nearest OCP FP8 E4M3 value, ties to even:
 * normals have 4 significant bits and exponent >= -6; below 2^-6 the
 * spacing is the subnormal quantum 2^-9. Values above 448 saturate. */
double orc_round_e4m3(double x) {
  if (x <= 0.0) return 0.0;
  if (x < 0.015625) return nearbyint(x * 512.0) / 512.0;
  int e;
  double m = frexp(x, &e);
  double r = ldexp(nearbyint(ldexp(m, 4)), e - 4);
  return r > 448.0 ? 448.0 : r;
}

/* density value actually used by a precision variant, from the exact w in (0,1]
 * bf16:   round(w);  bf16x2: hi + round(w - hi), hi = round(w);
 * e4m3:   round(448 w)/448  (scaled so the peak uses the top of the range). */
static inline double quantize(double w, int prec) {
  switch (prec) {
    case OP_BF16: return orc_round_bf16(w);
    case OP_BF16X2: {
      double h = orc_round_bf16(w);
      return h + orc_round_bf16(w - h);
    }
    case OP_FP8E4M3: return orc_round_e4m3(448.0 * w) / 448.0;
    case OP_FP32: return (double)(float)w;
    default: return w;
  }
}

/* ------------------------------------------------------------------------ */
/* propagation  (eq. (5), eq. VUP, Alg. VUP)                                 */
/* ------------------------------------------------------------------------ */

/* iterate the cells of a box window: returns flat cell index; j[] holds the
 * per-axis indices. Caller initialises j[d] = lo[d]. */
static inline int next_cell(int ndim, const int *wlo, const int *whi, int *j) {
  for (int d = ndim - 1; d >= 0; --d) {
    if (j[d] < whi[d]) { j[d]++; return 1; }
    j[d] = wlo[d];
  }
  return 0;
}

static inline long flat_index(const og_grid *g, const int *j) {
  long i = 0;
  for (int d = 0; d < g->ndim; ++d) i = i * g->n[d] + j[d];
  return i;
}

/* exact Gaussian weight exp(-1/2 sum_d ((x_d - mu_d)/sigma_d)^2), eq. gaussh */
static inline double gauss_w(const og_grid *g, const int *j, const double *mu, const double *sg) {
  double s = 0.0;
  for (int d = 0; d < g->ndim; ++d) {
    double t = (cell_x(g, d, j[d]) - mu[d]) / sg[d];
    s += t * t;
  }
  return exp(-0.5 * s);
}

/* P[k*B + b] (FP64), Z[k*C + c] = sum of the (quantised) weights over window
 * W_{k,c}. Mixture components are truncated and normalised separately, then
 * combined with their weights. Invalid parameters give a NaN column; an empty
 * window contributes nothing (Z = 0).
 * win may be NULL (computed here) or hold frozen windows. */
int orc_propagate(int ndim, const int *n, const double *lo, const double *hi,
                  const int *bin, int B, long K, int C,
                  const double *mu, const double *sigma, const double *weight, double ns,
                  int prec, const int *win_in, double *P, double *Z, int nthreads) {
  og_grid g = make_grid(ndim, n, lo, hi);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    ksum *hist = (ksum *)malloc(sizeof(ksum) * (size_t)B);
#pragma omp for schedule(dynamic, 1)
    for (long k = 0; k < K; ++k) {
      double *Pk = P + k * (long)B;
      for (int b = 0; b < B; ++b) Pk[b] = 0.0;
      int anybad = 0;
      for (int c = 0; c < C; ++c) {
        long kc = k * C + c;
        const double *m = mu + kc * ndim, *s = sigma + kc * ndim;
        int wlo[4], whi[4], bad = 0, empty = 0;
        for (int d = 0; d < ndim; ++d) {
          if (win_in) {
            wlo[d] = win_in[(kc * ndim + d) * 2];
            whi[d] = win_in[(kc * ndim + d) * 2 + 1];
            if (!(s[d] > 0.0) || !isfinite(s[d]) || !isfinite(m[d])) bad = 1;
          } else {
            bad |= axis_window(lo[d], hi[d], n[d], m[d], s[d], ns, &wlo[d], &whi[d]);
          }
          if (whi[d] < wlo[d]) empty = 1;
        }
        if (bad) { anybad = 1; Z[kc] = NAN; continue; }
        if (empty) { Z[kc] = 0.0; continue; }
        for (int b = 0; b < B; ++b) hist[b].s = hist[b].c = 0.0;
        ksum z = {0.0, 0.0};
        int j[4];
        for (int d = 0; d < ndim; ++d) j[d] = wlo[d];
        do {
          double q = quantize(gauss_w(&g, j, m, s), prec);
          ks_add(&z, q);
          int bb = bin[flat_index(&g, j)];
          if (bb >= 0) ks_add(&hist[bb], q);
        } while (next_cell(ndim, wlo, whi, j));
        double zc = ks_val(&z);
        Z[kc] = zc;
        double pc = (C > 1) ? weight[kc] : 1.0;
        for (int b = 0; b < B; ++b) Pk[b] += pc * (ks_val(&hist[b]) / zc);
      }
      if (anybad)
        for (int b = 0; b < B; ++b) Pk[b] = NAN;
    }
    free(hist);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* rounding sensitivity of the reduced-precision variants (for test bars)    */
/* ------------------------------------------------------------------------ */

/* Largest change of a rounded density when the value handed to the rounding
 * is off by a relative amount up to eps: the rounding is monotone, so every
 * value in [w(1-eps), w(1+eps)] rounds to a value between the roundings of
 * the two ends. The BF16 pair stays within 2^-17 of its argument on either
 * side of a change of its high part, so there the change is bounded by the
 * ends' difference plus 2^-16 w. FP32 and FP64 are not rounded to a coarser
 * grid here: no change. */
static double rounding_spread(double w, double eps, int prec) {
  if (prec != OP_BF16 && prec != OP_BF16X2 && prec != OP_FP8E4M3) return 0.0;
  double a = quantize(w * (1.0 - eps), prec);
  double b = quantize(w, prec);
  double c = quantize(w * (1.0 + eps), prec);
  double m = fmax(fabs(c - b), fabs(b - a));
  if (prec == OP_BF16X2 && orc_round_bf16(w * (1.0 - eps)) != orc_round_bf16(w * (1.0 + eps)))
    m += ldexp(w, -16);
  return m;
}

/* Bound on the column L1 distance between this oracle's reduced-precision P
 * (orc_propagate with prec) and any computation that rounds each density
 * from a value within relative eps of the exact one and normalises by the
 * sum of its own rounded values. Per component: M = sum over window cells of
 * rounding_spread, Z = sum of the rounded densities; a change of the rounded
 * values totalling at most M moves the normalised column by at most
 * 2 M / (Z - M) in L1. F[k] = sum_c pi_c 2 M_c / (Z_c - M_c); NaN for an
 * invalid component, 0 for an empty one. */
int orc_rounding_l1_bound(int ndim, const int *n, const double *lo, const double *hi, long K,
                          int C, const double *mu, const double *sigma, const double *weight,
                          double ns, int prec, double eps, double *F, int nthreads) {
  og_grid g = make_grid(ndim, n, lo, hi);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (long k = 0; k < K; ++k) {
    double f = 0.0;
    for (int c = 0; c < C; ++c) {
      long kc = k * C + c;
      const double *m = mu + kc * ndim, *s = sigma + kc * ndim;
      int wlo[4], whi[4], bad = 0, empty = 0;
      for (int d = 0; d < ndim; ++d) {
        bad |= axis_window(lo[d], hi[d], n[d], m[d], s[d], ns, &wlo[d], &whi[d]);
        if (whi[d] < wlo[d]) empty = 1;
      }
      if (bad) { f = NAN; break; }
      if (empty) continue;
      ksum z = {0.0, 0.0}, mm = {0.0, 0.0};
      int j[4];
      for (int d = 0; d < ndim; ++d) j[d] = wlo[d];
      do {
        double w = gauss_w(&g, j, m, s);
        ks_add(&z, quantize(w, prec));
        ks_add(&mm, rounding_spread(w, eps, prec));
      } while (next_cell(ndim, wlo, whi, j));
      double zc = ks_val(&z), mc = ks_val(&mm);
      double pc = (C > 1) ? weight[kc] : 1.0;
      f += pc * (mc < zc ? 2.0 * mc / (zc - mc) : 2.0);
    }
    F[k] = f;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* moments of the propagated output (exact f, quadrature form)               */
/* ------------------------------------------------------------------------ */

/* E_k = sum_c pi_c sum_i q_{c,i} f_i ;  Var_k = sum_c pi_c sum_i q_{c,i}(f_i - E_k)^2
 * (two passes). delta2 (optional, C == 1 only): the local expected squared
 * deviation of eq. IPSAvar, 1/2 sum_i q_i (f_i - M(mu_k))^2, with M(mu_k)
 * supplied in fmu[k]. NaN when any component is invalid or every window empty. */
int orc_moments(int ndim, const int *n, const double *lo, const double *hi,
                const double *f, long K, int C,
                const double *mu, const double *sigma, const double *weight, double ns,
                const double *fmu, double *mean, double *var, double *delta2, int nthreads) {
  og_grid g = make_grid(ndim, n, lo, hi);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (long k = 0; k < K; ++k) {
    int wlo[4][4], whi[4][4], bad = 0, allempty = 1, empty[4] = {0, 0, 0, 0};
    double zc[4] = {0, 0, 0, 0};
    for (int c = 0; c < C; ++c) {
      long kc = k * C + c;
      for (int d = 0; d < ndim; ++d) {
        bad |= axis_window(lo[d], hi[d], n[d], mu[kc * ndim + d], sigma[kc * ndim + d], ns,
                           &wlo[c][d], &whi[c][d]);
        if (whi[c][d] < wlo[c][d]) empty[c] = 1;
      }
      if (!empty[c]) allempty = 0;
    }
    if (bad || allempty) {
      mean[k] = var[k] = NAN;
      if (delta2) delta2[k] = NAN;
      continue;
    }
    /* normalisers */
    for (int c = 0; c < C; ++c) {
      if (empty[c]) continue;
      long kc = k * C + c;
      ksum z = {0, 0};
      int j[4];
      for (int d = 0; d < ndim; ++d) j[d] = wlo[c][d];
      do ks_add(&z, gauss_w(&g, j, mu + kc * ndim, sigma + kc * ndim));
      while (next_cell(ndim, wlo[c], whi[c], j));
      zc[c] = ks_val(&z);
    }
    /* pass 1: mean; pass 2: variance about it; delta2 about M(mu) */
    ksum e = {0, 0}, v = {0, 0}, dd = {0, 0};
    for (int pass = 0; pass < 2; ++pass) {
      double E = ks_val(&e);
      for (int c = 0; c < C; ++c) {
        if (empty[c]) continue;
        long kc = k * C + c;
        double pc = (C > 1) ? weight[kc] : 1.0;
        int j[4];
        for (int d = 0; d < ndim; ++d) j[d] = wlo[c][d];
        do {
          double q = pc * gauss_w(&g, j, mu + kc * ndim, sigma + kc * ndim) / zc[c];
          double fi = f[flat_index(&g, j)];
          if (pass == 0) {
            ks_add(&e, q * fi);
          } else {
            ks_add(&v, q * ((fi - E) * (fi - E)));
            if (delta2 && fmu) ks_add(&dd, q * ((fi - fmu[k]) * (fi - fmu[k])));
          }
        } while (next_cell(ndim, wlo[c], whi[c], j));
      }
    }
    mean[k] = ks_val(&e);
    var[k] = ks_val(&v);
    if (delta2) delta2[k] = (fmu && C == 1) ? 0.5 * ks_val(&dd) : NAN;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* IPSA coarse-grained quantities per column (Sec. 5.2)                      */
/* ------------------------------------------------------------------------ */

/* Bin centres c_b = (e_b + e_{b+1})/2. mean_hist = sum_b P_b c_b,
 * var = sum_b P_b (c_b - mean)^2 (two passes), entropy = -sum_{P_b>0} P_b ln P_b. */
int orc_ipsa(const double *P, long K, int B, const double *edges,
             double *mean_hist, double *var, double *entropy) {
#pragma omp parallel for schedule(static)
  for (long k = 0; k < K; ++k) {
    const double *Pk = P + k * (long)B;
    ksum m = {0, 0}, v = {0, 0}, h = {0, 0};
    for (int b = 0; b < B; ++b) ks_add(&m, Pk[b] * ((edges[b] + edges[b + 1]) / 2.0));
    double E = ks_val(&m);
    for (int b = 0; b < B; ++b) {
      double dc = (edges[b] + edges[b + 1]) / 2.0 - E;
      ks_add(&v, Pk[b] * (dc * dc));
      if (Pk[b] > 0.0) ks_add(&h, -Pk[b] * log(Pk[b]));
    }
    mean_hist[k] = E;
    var[k] = ks_val(&v);
    entropy[k] = ks_val(&h);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* IPSA sensitivity: gradient of Q_k = g_var Var_k + g_ent H_k                */
/* ------------------------------------------------------------------------ */

/* With P_b = sum_c pi_c sum_{i in b} q_{c,i}, q = w/Z, w the Gaussian weight
 * (eq. gaussh) on frozen windows:
 *   dQ/dP_b = g_var((c_b - E)^2 - 2 c_b S) - g_ent(ln P_b + 1) =: v_b,
 *   S = sum_b P_b (c_b - E)  (zero when the column sums to one),
 *   dq_{c,i}/dtheta = q_{c,i} (s_theta(i) - sum_j q_{c,j} s_theta(j)),
 *   s_mu_d = (x_d - mu_d)/sigma_d^2,  s_sigma_d = (x_d - mu_d)^2/sigma_d^3,
 * so dQ/dtheta_c = pi_c sum_i q_{c,i} v_{bin(i)} (s(i) - sbar), and
 *   dQ/dpi_c = sum_i q_{c,i} v_{bin(i)}.
 * Everything is summed cell by cell here (no separable shortcut).
 * P is the FP64 forward result of orc_propagate (prec = FP64) on the same
 * windows. Outputs g_mu/g_sigma [K][C][d], g_weight [K][C] (may be NULL). */
int orc_ipsa_grad(int ndim, const int *n, const double *lo, const double *hi,
                  const int *bin, int B, const double *edges, long K, int C,
                  const double *mu, const double *sigma, const double *weight,
                  const int *win, const double *P, const double *g_var, const double *g_ent,
                  double *g_mu, double *g_sigma, double *g_weight, int nthreads) {
  og_grid g = make_grid(ndim, n, lo, hi);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    double *v = (double *)malloc(sizeof(double) * (size_t)B);
#pragma omp for schedule(dynamic, 1)
    for (long k = 0; k < K; ++k) {
      const double *Pk = P + k * (long)B;
      double gv = g_var ? g_var[k] : 0.0, ge = g_ent ? g_ent[k] : 0.0;
      ksum m = {0, 0}, sacc = {0, 0};
      for (int b = 0; b < B; ++b) ks_add(&m, Pk[b] * ((edges[b] + edges[b + 1]) / 2.0));
      double E = ks_val(&m);
      for (int b = 0; b < B; ++b) ks_add(&sacc, Pk[b] * ((edges[b] + edges[b + 1]) / 2.0 - E));
      double S = ks_val(&sacc);
      for (int b = 0; b < B; ++b) {
        double cb = (edges[b] + edges[b + 1]) / 2.0;
        double vb = gv * ((cb - E) * (cb - E) - 2.0 * cb * S);
        if (Pk[b] > 0.0) vb -= ge * (log(Pk[b]) + 1.0);
        v[b] = vb;
      }
      for (int c = 0; c < C; ++c) {
        long kc = k * C + c;
        const double *mk = mu + kc * ndim, *sk = sigma + kc * ndim;
        int wlo[4], whi[4], empty = 0, bad = 0;
        for (int d = 0; d < ndim; ++d) {
          wlo[d] = win[(kc * ndim + d) * 2];
          whi[d] = win[(kc * ndim + d) * 2 + 1];
          if (whi[d] < wlo[d]) empty = 1;
          if (!(sk[d] > 0.0) || !isfinite(sk[d]) || !isfinite(mk[d])) bad = 1;
        }
        double pc = (C > 1) ? weight[kc] : 1.0;
        if (bad || empty) {
          for (int d = 0; d < ndim; ++d) {
            g_mu[kc * ndim + d] = bad ? NAN : 0.0;
            g_sigma[kc * ndim + d] = bad ? NAN : 0.0;
          }
          if (g_weight) g_weight[kc] = bad ? NAN : 0.0;
          continue;
        }
        ksum z = {0, 0}, a0 = {0, 0}, a1[4], a2[4], m1[4], m2[4];
        for (int d = 0; d < 4; ++d) a1[d] = a2[d] = m1[d] = m2[d] = (ksum){0, 0};
        int j[4];
        for (int d = 0; d < ndim; ++d) j[d] = wlo[d];
        do {
          double w = gauss_w(&g, j, mk, sk);
          int bb = bin[flat_index(&g, j)];
          double vi = (bb >= 0) ? v[bb] : 0.0;
          ks_add(&z, w);
          ks_add(&a0, w * vi);
          for (int d = 0; d < ndim; ++d) {
            double u = cell_x(&g, d, j[d]) - mk[d];
            double sm = u / (sk[d] * sk[d]);
            double ss = (u * u) / (sk[d] * sk[d] * sk[d]);
            ks_add(&a1[d], w * vi * sm);
            ks_add(&a2[d], w * vi * ss);
            ks_add(&m1[d], w * sm);
            ks_add(&m2[d], w * ss);
          }
        } while (next_cell(ndim, wlo, whi, j));
        double Zc = ks_val(&z), A0 = ks_val(&a0) / Zc;
        for (int d = 0; d < ndim; ++d) {
          g_mu[kc * ndim + d] = pc * (ks_val(&a1[d]) / Zc - (ks_val(&m1[d]) / Zc) * A0);
          g_sigma[kc * ndim + d] = pc * (ks_val(&a2[d]) / Zc - (ks_val(&m2[d]) / Zc) * A0);
        }
        if (g_weight) g_weight[kc] = A0;
      }
    }
    free(v);
  }
  return 0;
}
