/*
 * Sanitizer harness for the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Built together with vup_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only, gcc) by oracle/build.py's
 * build_sanitized(); tests/test_oracle_pins.py runs the executable. It calls
 * every exported oracle function on small grids of one to four axes, with
 * mixtures, every density precision, frozen windows, and the degenerate inputs
 * the oracle defines outputs for (NaN and out-of-range model values, invalid
 * and empty windows, a delta input, all-zero columns). Any out-of-bounds
 * access, use of freed memory or undefined arithmetic aborts the run; a clean
 * run prints "san_check ok" and exits 0. The values themselves are checked by
 * the Python pins, not here (only a few invariants are asserted).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double orc_model_at(int kind, int ndim, const double *theta, const double *x);
int orc_eval_grid(int ndim, const int *n, const double *lo, const double *hi, int kind,
                  const double *theta, double *f);
void orc_uniform_edges(const double *f, long N, int B, double *edges);
void orc_bin(const double *f, long N, const double *edges, int B, int *bin);
void orc_model_matrix(const int *bin, long N, int B, long *offsets, long *perm);
long orc_windows(int ndim, const int *n, const double *lo, const double *hi, long K, int C,
                 const double *mu, const double *sigma, double ns, int *win, int *bad);
double orc_round_bf16(double x);
double orc_round_e4m3(double x);
int orc_propagate(int ndim, const int *n, const double *lo, const double *hi, const int *bin,
                  int B, long K, int C, const double *mu, const double *sigma,
                  const double *weight, double ns, int prec, const int *win_in, double *P,
                  double *Z, int nthreads);
int orc_moments(int ndim, const int *n, const double *lo, const double *hi, const double *f,
                long K, int C, const double *mu, const double *sigma, const double *weight,
                double ns, const double *fmu, double *mean, double *var, double *delta2,
                int nthreads);
int orc_rounding_l1_bound(int ndim, const int *n, const double *lo, const double *hi, long K,
                          int C, const double *mu, const double *sigma, const double *weight,
                          double ns, int prec, double eps, double *F, int nthreads);
int orc_ipsa(const double *P, long K, int B, const double *edges, double *mean_hist,
             double *var, double *entropy);
int orc_ipsa_grad(int ndim, const int *n, const double *lo, const double *hi, const int *bin,
                  int B, const double *edges, long K, int C, const double *mu,
                  const double *sigma, const double *weight, const int *win, const double *P,
                  const double *g_var, const double *g_ent, double *g_mu, double *g_sigma,
                  double *g_weight, int nthreads);

/* models of each dimension count: linear, sincos2, damped3, ring4, timing2, ipsa2 */
static const int kModelDim[6] = {0, 2, 3, 4, 2, 2};

static unsigned long long g_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* splitmix64 -> [0, 1) */
  unsigned long long z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static void *xmalloc(size_t n) {
  void *p = malloc(n ? n : 1);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return p;
}

static int fails = 0;
static void expect(int cond, const char *what) {
  if (!cond) {
    fprintf(stderr, "san_check: %s\n", what);
    ++fails;
  }
}

/* one grid, one model, B bins, K distributions of C components */
static void run_case(int ndim, const int *n, int kind, int B, long K, int C, int nthreads) {
  double lo[4], hi[4], theta[8];
  long N = 1;
  for (int d = 0; d < ndim; ++d) {
    lo[d] = -2.0 - 0.1 * d;
    hi[d] = 2.0 + 0.3 * d;
    N *= n[d];
  }
  for (int t = 0; t < 8; ++t) theta[t] = 0.25 + 0.5 * t;
  double *f = xmalloc(sizeof(double) * N);
  orc_eval_grid(ndim, n, lo, hi, kind, theta, f);
  double *edges = xmalloc(sizeof(double) * (B + 1));
  orc_uniform_edges(f, N, B, edges);
  /* a few cells outside the bins and a NaN value */
  f[0] = edges[B] + 1.0;
  if (N > 2) f[N / 2] = NAN;
  int *bin = xmalloc(sizeof(int) * N);
  orc_bin(f, N, edges, B, bin);
  long *offsets = xmalloc(sizeof(long) * (B + 1));
  long *perm = xmalloc(sizeof(long) * N);
  orc_model_matrix(bin, N, B, offsets, perm);
  expect(offsets[B] <= N, "model matrix holds at most N cells");

  size_t nkc = (size_t)K * C, npar = nkc * ndim;
  double *mu = xmalloc(sizeof(double) * npar), *sg = xmalloc(sizeof(double) * npar);
  double *w = C > 1 ? xmalloc(sizeof(double) * nkc) : NULL;
  for (size_t i = 0; i < npar; ++i) {
    int d = (int)(i % ndim);
    mu[i] = lo[d] - 0.5 + urand() * (hi[d] - lo[d] + 1.0);
    sg[i] = 0.02 + 0.8 * urand();
  }
  if (w)
    for (long k = 0; k < K; ++k) {
      double a = urand();
      w[k * C] = a;
      w[k * C + 1] = 1.0 - a;
    }
  /* degenerate inputs: invalid sigma, a window outside the grid, a delta input
   * at a cell centre, a window covering the whole grid */
  sg[0] = 0.0;
  if (K > 1) mu[(size_t)1 * C * ndim] = hi[0] + 50.0;
  if (K > 2)
    for (int d = 0; d < ndim; ++d) {
      mu[(size_t)2 * C * ndim + d] = lo[d] + 1.5 * (hi[d] - lo[d]) / n[d];
      sg[(size_t)2 * C * ndim + d] = 1e-9;
    }
  if (K > 3)
    for (int d = 0; d < ndim; ++d) sg[(size_t)3 * C * ndim + d] = 1e6;

  int *win = xmalloc(sizeof(int) * npar * 2), *bad = xmalloc(sizeof(int) * nkc);
  long U = orc_windows(ndim, n, lo, hi, K, C, mu, sg, 4.0, win, bad);
  expect(U >= 0, "window cell count is non-negative");

  double *P = xmalloc(sizeof(double) * K * B), *Z = xmalloc(sizeof(double) * nkc);
  for (int prec = -1; prec <= 3; ++prec) {
    orc_propagate(ndim, n, lo, hi, bin, B, K, C, mu, sg, w, 4.0, prec, NULL, P, Z, nthreads);
    orc_propagate(ndim, n, lo, hi, bin, B, K, C, mu, sg, w, 4.0, prec, win, P, Z, nthreads);
  }
  double *F = xmalloc(sizeof(double) * K);
  for (int prec = -1; prec <= 3; ++prec)
    orc_rounding_l1_bound(ndim, n, lo, hi, K, C, mu, sg, w, 4.0, prec, 0x1p-19, F, nthreads);
  free(F);
  double *fmu = xmalloc(sizeof(double) * K), *mean = xmalloc(sizeof(double) * K);
  double *var = xmalloc(sizeof(double) * K), *d2 = xmalloc(sizeof(double) * K);
  for (long k = 0; k < K; ++k) fmu[k] = orc_model_at(kind, ndim, theta, mu + (size_t)k * C * ndim);
  orc_moments(ndim, n, lo, hi, f, K, C, mu, sg, w, 4.0, fmu, mean, var, d2, nthreads);
  orc_moments(ndim, n, lo, hi, f, K, C, mu, sg, w, 4.0, NULL, mean, var, NULL, nthreads);

  double *mh = xmalloc(sizeof(double) * K), *vh = xmalloc(sizeof(double) * K);
  double *hh = xmalloc(sizeof(double) * K);
  orc_propagate(ndim, n, lo, hi, bin, B, K, C, mu, sg, w, 4.0, -1, win, P, Z, nthreads);
  orc_ipsa(P, K, B, edges, mh, vh, hh);
  double *gv = xmalloc(sizeof(double) * K), *ge = xmalloc(sizeof(double) * K);
  for (long k = 0; k < K; ++k) {
    gv[k] = 0.5 + urand();
    ge[k] = 0.5 + urand();
  }
  double *gm = xmalloc(sizeof(double) * npar), *gs = xmalloc(sizeof(double) * npar);
  double *gw = xmalloc(sizeof(double) * nkc);
  orc_ipsa_grad(ndim, n, lo, hi, bin, B, edges, K, C, mu, sg, w, win, P, gv, ge, gm, gs,
                C > 1 ? gw : NULL, nthreads);
  orc_ipsa_grad(ndim, n, lo, hi, bin, B, edges, K, C, mu, sg, w, win, P, NULL, NULL, gm, gs,
                NULL, nthreads);
  /* a column of zeros and a one-hot column through the IPSA quantities */
  memset(P, 0, sizeof(double) * B);
  if (K > 1) {
    memset(P + B, 0, sizeof(double) * B);
    P[B + B / 2] = 1.0;
  }
  orc_ipsa(P, K, B, edges, mh, vh, hh);
  if (K > 1) expect(hh[1] == 0.0 && vh[1] == 0.0, "one-hot column: zero entropy and variance");

  free(f); free(edges); free(bin); free(offsets); free(perm); free(mu); free(sg); free(w);
  free(win); free(bad); free(P); free(Z); free(fmu); free(mean); free(var); free(d2);
  free(mh); free(vh); free(hh); free(gv); free(ge); free(gm); free(gs); free(gw);
}

int main(void) {
  static const int n1[1] = {97}, n2[2] = {23, 31}, n3[3] = {9, 11, 13}, n4[4] = {5, 6, 4, 7};
  const int *ns[5] = {NULL, n1, n2, n3, n4};
  for (int kind = 0; kind < 6; ++kind) {
    for (int ndim = 1; ndim <= 4; ++ndim) {
      if (kModelDim[kind] != 0 && kModelDim[kind] != ndim) continue;
      for (int C = 1; C <= 2; ++C) run_case(ndim, ns[ndim], kind, 1 + 7 * ndim, 9, C, 2);
    }
  }
  /* one bin, and more bins than cells */
  run_case(2, n2, 1, 1, 5, 1, 1);
  run_case(1, n1, 0, 300, 5, 2, 1);
  /* quantisers at the ends of their ranges */
  const double xs[] = {0.0, 1e-300, 1e-40, 0x1p-10, 0x1p-9, 0x1p-7, 0.0078125, 1.0, 448.0, 500.0};
  for (size_t i = 0; i < sizeof xs / sizeof xs[0]; ++i) {
    volatile double a = orc_round_bf16(xs[i]), b = orc_round_e4m3(xs[i]);
    (void)a;
    (void)b;
  }
  if (fails) return 1;
  printf("san_check ok\n");
  return 0;
}
