/*
 * vup.h - C ABI of the MI355X (gfx950) library for Vectorized Uncertainty
 * Propagation (VUP) and Input Probability Sensitivity Analysis (IPSA),
 * arXiv:1908.11246.
 *
 * The problem (Sec. 3, eq. (4), eq. (5), eq. VUP): a model y = M(x) is
 * evaluated ONCE on a uniform cell-centred grid; every cell gets the index of
 * the output bin its value falls in (the sparse one-hot "model matrix"); then
 * K input probability distributions are propagated together,
 *     P[k][b] = sum_i [bin(i) = b] p_k(x_i),
 * where p_k is a Gaussian (Sec. 5.2, eq. gaussh) or a mixture of Gaussians,
 * evaluated at cell centres, truncated per axis at n_sigma standard deviations
 * and renormalised over the kept cells. From P the library derives the
 * coarse-grained IPSA quantities (Sec. 5.2): per-location output variance and
 * entropy, and their gradients with respect to the pdf parameters.
 *
 * Conventions shared by every entry point
 *  - Grid: ndim in [1,4] axes, n[d] cells on [lo[d], hi[d]]; cell centre
 *    x_{d,j} = lo_d + (j + 1/2) (hi_d - lo_d)/n_d (composite midpoint rule,
 *    Sec. 3); flat cell index row major, axis 0 slowest.
 *  - Memory: the caller owns all memory. Pointers marked "dev" are device
 *    (HBM) pointers of the current HIP device; "host" pointers are ordinary
 *    host memory. No call allocates device memory; the buffers the library
 *    needs are workspaces the caller passes (vup_bin, the separable form,
 *    the marginal). The one exception to caller-owned memory is the fixed
 *    device array behind vup_marginalize_noalloc (VUP_NOALLOC_SCRATCH_BYTES
 *    per GPU, part of the loaded code object, never allocated by a call).
 *  - Streams: every kernel is enqueued on `stream` (a hipStream_t; NULL = the
 *    default stream). No call synchronises except vup_counters.
 *  - Errors: every call returns VUP_OK (0) or a negative status. Arguments
 *    that can be checked on the host are checked before anything is enqueued;
 *    on failure nothing is enqueued and vup_last_error() (thread-local)
 *    explains why. Problems only visible on the device never fail a call:
 *    they give defined outputs (NaN or zero columns, bin -1) and raise the
 *    counters read by vup_counters.
 *  - Determinism: no cross-workgroup floating-point atomics; repeated calls
 *    with the same inputs give bit-identical outputs.
 */
#ifndef VUP_H
#define VUP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define VUP_OK 0
#define VUP_EINVAL (-1)       /* invalid argument (see vup_last_error)          */
#define VUP_ENODEV (-2)       /* no usable HIP device                            */
#define VUP_EDEVICE (-3)      /* a HIP runtime call failed                       */
#define VUP_EUNSUPPORTED (-4) /* valid but unsupported combination / size       */
#define VUP_EWORKSPACE (-5)   /* workspace too small or not built by vup_bin    */

/* density precision of vup_propagate (Sec. 3 leaves it open; all variants
 * accumulate in FP32 and normalise with an FP64 sum of the same values) */
#define VUP_FP32 0      /* density in FP32                                          */
#define VUP_BF16 1      /* density rounded to bfloat16 (nearest even)               */
#define VUP_BF16X2 2    /* hi + lo bfloat16 pair: hi = bf16(w), lo = bf16(w - hi)    */
#define VUP_FP8E4M3 3   /* OCP FP8 E4M3 of 448*w (nearest even); the scale cancels  */

/* built-in models for vup_eval_grid (Sec. 2, eq. modelfunction: any model can
 * instead be evaluated by the caller into f[N] and passed to vup_bin) */
#define VUP_MODEL_LINEAR 0   /* theta[0] + sum_d theta[d+1] x_d              any ndim */
#define VUP_MODEL_SINCOS2 1  /* sin x0 + 0.5 cos(2 x1) + x0 x1 / 4            ndim 2  */
#define VUP_MODEL_DAMPED3 2  /* exp(-0.1 x2) sin x0 cos x1 + 0.1 x0 x1 x2      ndim 3  */
#define VUP_MODEL_RING4 3    /* sum_j sin(x_j) x_{j+1 mod 4} + 0.05 (sum x)^2  ndim 4  */
#define VUP_MODEL_TIMING2 4  /* 1.1 sin x + 7 sin^2 alpha (Sec. 4.1)           ndim 2  */
#define VUP_MODEL_IPSA2 5    /* x^2 + 5 sin 3x + alpha (Sec. 5.3)              ndim 2  */

/* limits */
#define VUP_MAX_DIM 4
#define VUP_MAX_BINS 4096     /* B; the per-workgroup histograms live in LDS     */
#define VUP_MAX_COMP 2        /* mixture components per distribution            */
#define VUP_MAX_AXIS 65536    /* n[d]                                            */
#define VUP_MAX_DY (1 << 24)  /* n_dy of vup_ipsa_matrix                         */
#define VUP_MAX_LEVELS 16     /* quantile levels of vup_ipsa_fields              */
#define VUP_MAX_MARGINAL_COLS (1 << 24)  /* row length n of vup_marginalize      */

typedef struct vup_grid {
  int32_t ndim;      /* 1..4                                                   */
  int32_t n[4];      /* cells per axis, n[d] >= 1; entries >= ndim ignored     */
  double lo[4];      /* domain lower edge per axis (finite)                    */
  double hi[4];      /* domain upper edge per axis (finite, > lo)              */
} vup_grid;

typedef struct vup_model {
  int32_t kind;      /* VUP_MODEL_*                                            */
  int32_t reserved;
  double theta[8];   /* model parameters (VUP_MODEL_LINEAR only)               */
} vup_model;

/* K input distributions, each a mixture of ncomp diagonal Gaussians
 * (eq. gaussh per axis). Arrays are dev, FP64, row major:
 *   mu[K][ncomp][ndim], sigma[K][ncomp][ndim], weight[K][ncomp].
 * Each component is truncated to the box |x_d - mu_d| <= n_sigma sigma_d
 * intersected with the grid and normalised separately; the column is
 * sum_c weight_c * component_c (weights are used as given). */
typedef struct vup_dists {
  int64_t K;             /* number of distributions, >= 0                      */
  int32_t ncomp;         /* 1 or 2                                              */
  int32_t ndim;          /* must equal the grid's ndim                          */
  double n_sigma;        /* truncation half-width in standard deviations, > 0   */
  const double* mu;      /* dev [K][ncomp][ndim]                                */
  const double* sigma;   /* dev [K][ncomp][ndim]; <= 0 or non-finite -> NaN column */
  const double* weight;  /* dev [K][ncomp]; NULL iff ncomp == 1                 */
} vup_dists;

/* Host-side descriptor of a model matrix built by vup_bin. Plain data: copy
 * it freely. The arrays it refers to live inside the caller's workspace. */
typedef struct vup_mm {
  vup_grid grid;
  int32_t B;            /* number of bins                                       */
  int32_t pitch;        /* padded length of the fastest axis in the bin map     */
  int64_t N;            /* cells                                                */
  int64_t rows;         /* N / n[ndim-1]                                        */
  void* ws;             /* dev workspace base                                   */
  size_t ws_bytes;
  /* byte offsets inside ws */
  size_t off_edges;     /* double[B+1]      bin edges                           */
  size_t off_binmap;    /* uint16[rows*pitch] 4*bin (4*B for no bin), padded    */
  size_t off_f32;       /* float[rows*pitch] model values in FP32, padded: a    */
                        /* column c with c % 8 == 0 holds f, any other column  */
                        /* f - f(c - c % 8) (padding columns: 0)               */
  size_t off_counts;    /* int64[B+1]       cells per bin; [B] = outside        */
  size_t off_offsets;   /* int64[B+1]       CSR row starts of the model matrix  */
  size_t off_perm;      /* int32[N]         cells sorted by bin (stable)        */
  size_t off_scratch;   /* int32 scratch for the sort and the run count         */
  size_t off_counters;  /* int64[8]         device-side event counters          */
  size_t off_runs;      /* uint32[]  runs of equal bin along the fastest axis:
                           (first cell) | (4*bin << 16), one terminator per row */
  size_t off_rowptr;    /* int32[rows+1]    first run of each row               */
  size_t off_runidx;    /* uint16[rows*pitch] run of each cell, relative to row */
  int32_t sweep;        /* form of vup_propagate's FP32 sweep (VUP_SWEEP_*)     */
  int32_t reserved;
  uint64_t magic;
} vup_mm;

/* --------------------------------------------------------------------------
 * vup_eval_grid - Alg. VUP steps "generate a uniform grid" and "evaluate the
 * model" (Sec. 2 eq. modelfunction; Appendix A, Alg. VUP). Writes f[i] =
 * M(x_i) in FP64 for every cell, row major. f: dev [N].
 * EINVAL: bad grid, unknown model, model/ndim mismatch.
 * ------------------------------------------------------------------------ */
int vup_eval_grid(const vup_grid* g, const vup_model* m, double* f, void* stream);

/* --------------------------------------------------------------------------
 * vup_uniform_edges - B uniform bins over [min f, max f] (the output
 * partition of eq. (4), whose bin widths "uniformly partition" the output).
 * edges[b] = lo + b*((hi - lo)/B) for b < B, edges[B] = hi, with lo/hi the
 * min/max of the non-NaN f. f: dev [N]; edges: dev [B+1].
 * A constant f gives non-increasing edges, which vup_bin then flags.
 * EINVAL: N < 1, B outside [1, VUP_MAX_BINS], NULL pointers.
 * ------------------------------------------------------------------------ */
int vup_uniform_edges(const double* f, int64_t N, int32_t B, double* edges, void* stream);

/* --------------------------------------------------------------------------
 * vup_bin_workspace_bytes - bytes of device workspace vup_bin needs.
 * Returns 0 for an invalid grid or B.
 * ------------------------------------------------------------------------ */
size_t vup_bin_workspace_bytes(const vup_grid* g, int32_t B);

/* --------------------------------------------------------------------------
 * vup_bin - builds the model matrix (eq. (5), eq. MUP; Alg. VUP
 * "UniqueSorted ... set indexed model matrix elements to 1"): the indicator
 * Theta of eq. (4) as bin(i) = largest b < B with edges[b] <= f[i], valid when
 * edges[0] <= f[i] <= edges[B] (the last bin is closed); -1 for values
 * outside or NaN. Also stores, inside ws: the edges, a padded FP32 copy of f,
 * the bin map used by the propagation kernels, per-bin cell counts and the
 * compressed-by-bin form (cells of each bin in increasing order).
 *   f: dev [N] FP64;  edges: dev [B+1] FP64, finite and strictly increasing
 *   (checked on the device: if violated every bin is -1 and the `bad_edges`
 *   counter is raised);  bin: dev [N] int32 (may be NULL);  ws: dev,
 *   ws_bytes >= vup_bin_workspace_bytes(g, B), 256-byte aligned.
 * mm_out (host) receives the descriptor used by the calls below. The
 * workspace must stay allocated and unmodified while mm_out is in use.
 * EINVAL / EWORKSPACE before any launch.
 * ------------------------------------------------------------------------ */
int vup_bin(const vup_grid* g, const double* f, const double* edges, int32_t B, int32_t* bin,
            void* ws, size_t ws_bytes, vup_mm* mm_out, void* stream);

/* --------------------------------------------------------------------------
 * vup_windows - truncation windows of every (distribution, component), the
 * kept cells of eq. gaussh after truncation (Sec. 5.3): per axis
 *   t_lo = ((mu - ns*sigma) - lo)/h - 1/2, j_lo = max(0, ceil(t_lo)),
 *   t_hi = ((mu + ns*sigma) - lo)/h - 1/2, j_hi = min(n-1, floor(t_hi)),
 * h = (hi - lo)/n, all in FP64 without contraction; if j_lo > j_hi and mu is
 * inside [lo, hi] the window is the cell holding mu, else empty (0, -1).
 * Invalid parameters give (0, -1) as well.
 *   win: dev int32 [K][ncomp][ndim][2] (inclusive bounds).
 * ------------------------------------------------------------------------ */
int vup_windows(const vup_grid* g, const vup_dists* d, int32_t* win, void* stream);

/* --------------------------------------------------------------------------
 * vup_propagate - eq. VUP: P = M . P_in for all K input pdfs at once, with
 * the input probability matrix never materialised: densities are generated in
 * the kernel from (mu, sigma) as products of per-axis Gaussian factors over
 * the truncation window and accumulated per bin in on-chip histograms.
 *   P: dev FP32 [K][B] (row k = output pdf of distribution k; the paper's
 *      N_y x L output matrix stored column-major);
 *   Z: dev FP64 [K][ncomp] or NULL: sum of the (precision-rounded) weights of
 *      each component over its window, including cells with no bin. An axis
 *      whose largest weight factor in the window would be below 2^-20 (a pdf
 *      far narrower than a cell) has its factors scaled by a power of two
 *      inside the kernels; Z is scaled back exactly, and P does not depend
 *      on the scale.
 * precision: VUP_FP32 / VUP_BF16 / VUP_BF16X2 / VUP_FP8E4M3. FP32 densities
 * are accumulated per run of equal bin along the fastest axis (prefix sums of
 * the fastest-axis factors) or per cell, as vup_set_sweep_mode selects; the
 * reduced precisions round every cell's density and always go per cell.
 * Invalid parameters -> NaN row (counter bad_param); every window empty ->
 * zero row (counter empty). Column sums are 1 up to FP32 rounding unless some
 * cells of the window have bin -1.
 * EINVAL: bad descriptors; EWORKSPACE: mm not from vup_bin.
 * ------------------------------------------------------------------------ */
int vup_propagate(const vup_mm* mm, const vup_dists* d, int32_t precision, float* P, double* Z,
                  void* stream);

/* Tensor-product family of 2-D Gaussians for vup_propagate_separable:
 * distribution k = mx * M[1] + my has mean (mu[0][mx], mu[1][my]) and
 * deviations (sigma[0][mx], sigma[1][my]); e.g. measurement locations on a
 * subgrid of the input domain (Sec. 5.3 evaluates one pdf per location). */
typedef struct vup_sepdists {
  int32_t M[2];            /* locations per axis, >= 1                          */
  double n_sigma;          /* truncation half-width in standard deviations, > 0 */
  const double* mu[2];     /* dev [M[d]] FP64                                    */
  const double* sigma[2];  /* dev [M[d]] FP64; <= 0 or non-finite -> NaN rows    */
  int32_t precision;       /* operands of the contraction: VUP_FP32 (0), VUP_BF16,
                              VUP_BF16X2 (see vup_propagate_separable)           */
} vup_sepdists;

/* --------------------------------------------------------------------------
 * vup_separable_workspace_bytes - device workspace for vup_propagate_separable
 * (factor matrices, per-axis sums, prefix sums along y and the partial
 * contraction T, whose size is n[0] * B * M[1] floats). 0 for invalid
 * arguments.
 * ------------------------------------------------------------------------ */
size_t vup_separable_workspace_bytes(const vup_mm* mm, int32_t Mx, int32_t My);

/* --------------------------------------------------------------------------
 * vup_propagate_separable - eq. VUP for a tensor-product family on a 2-D grid,
 * with the input probability matrix factorised into per-axis truncated
 * Gaussian factors A_x[ix][mx], A_y[iy][my]:
 *   P[k][b] = sum_ix A_x[ix][mx] T[ix][b][my] / (Zx[mx] Zy[my]),
 *   T[ix][b][my] = sum_{iy : bin(ix,iy) = b} A_y[iy][my].
 * T is a scatter over one axis; the contraction over the other is a banded
 * dense product evaluated on the matrix cores. s->precision picks its
 * operands: VUP_FP32 (FP32 MFMA), VUP_BF16 (A_x and T rounded to bfloat16,
 * nearest even; BF16 MFMA with FP32 accumulation; each term within
 * (1 + 2^-8)^2 - 1 of the FP32 operands' product, so a column's L1 error
 * grows by at most about 2^-7) or VUP_BF16X2 (each operand as hi + lo
 * bfloat16, the product as hi*hi + hi*lo + lo*hi: within 3 * 2^-16 per
 * term). T stays FP32 in the workspace either way. Same outputs and
 * conventions as vup_propagate with K = M[0]*M[1], ncomp = 1 (Z[k] =
 * Zx[mx] * Zy[my], the window mass). T is built from the model matrix's runs
 * of equal bin along y (one difference of FP64 prefix sums per run). Families
 * with M[1] < 16 (e.g. one shared alpha factor) are too narrow for the
 * contraction's tiles and are propagated by the general sweep of
 * vup_propagate (FP32 densities, whatever s->precision) instead, with the
 * same outputs. Needs ndim == 2, and B <= 512 when n[1] > 65534.
 * EINVAL: precision other than VUP_FP32, VUP_BF16, VUP_BF16X2.
 *   ws: dev, 256-byte aligned, ws_bytes >= vup_separable_workspace_bytes.
 * ------------------------------------------------------------------------ */
int vup_propagate_separable(const vup_mm* mm, const vup_sepdists* s, void* ws, size_t ws_bytes,
                            float* P, double* Z, void* stream);

/* --------------------------------------------------------------------------
 * vup_moments - output moments of each propagated pdf from the exact model
 * values (quadrature form of the marginalisation integral, eq. UP):
 *   mean[k] = sum_i p_k(x_i) f_i,  var[k] = sum_i p_k(x_i) (f_i - mean_k)^2,
 * with FP32 per-row partial sums of shifted values and FP64 accumulation.
 * delta2 (optional, ncomp == 1 and a built-in model only): the local expected
 * squared deviation of eq. IPSAvar, 1/2 sum_i p_k(x_i)(f_i - M(mu_k))^2,
 * computed as (var + (mean - M(mu_k))^2)/2 with M evaluated at mu_k. The
 * reference value is the model at the pdf's maximum, y(l) = M(mu_k), the same
 * reference the IPSA probability matrix is translated by (Sec. 5.3). Eq.
 * IPSAvar keeps parameter-like axes (alpha) at the cell's own value inside the
 * reference, M(l, alpha); both readings agree when every axis is data-like,
 * and for a model additive in alpha with a window symmetric about mu_alpha
 * the y(l) reading exceeds eq. IPSAvar's by half the pdf's alpha variance.
 *   mean, var: dev FP64 [K]; delta2: dev FP64 [K] or NULL; model: host, used
 *   only for delta2 (may be NULL when delta2 is NULL); it must be a model of
 *   the grid's ndim (EINVAL otherwise).
 * Moments are of the f given to vup_bin (its FP32 copy, held in the model
 * matrix). NaN for invalid parameters or all-empty windows. The kernel sums
 * strips of 8 fastest-axis cells (columns 8m .. 8m+7) over the window's rows,
 * so a non-finite model value gives NaN for every window whose rows hold it
 * and whose columns meet its strip (vup_moments_tiled: only for windows that
 * hold it).
 * ------------------------------------------------------------------------ */
int vup_moments(const vup_mm* mm, const vup_dists* d, const vup_model* model, double* mean,
                double* var, double* delta2, void* stream);

/* --------------------------------------------------------------------------
 * vup_moments_tiled_workspace_bytes - device workspace of vup_moments_tiled
 * for K pdfs: 80 + 8 + 16 bytes per pdf and 32 per tile of 64 x 64 cells
 * (each part rounded up to 256 bytes). 0 when the tiled form does not apply
 * (see below); then vup_moments_tiled needs no workspace.
 * ------------------------------------------------------------------------ */
size_t vup_moments_tiled_workspace_bytes(const vup_mm* mm, const vup_dists* d);

/* --------------------------------------------------------------------------
 * vup_moments_tiled - the outputs of vup_moments (same arguments, meaning and
 * NaN rules) by tiles of the model values on the int8 matrix cores. For a
 * separable pdf the moment sums over one 64 x 64 tile are bilinear forms in
 * the tile's model values, sum_ij gx(i) (f_ij - a)^q gy(j), q = 1, 2 (eq. UP
 * with the Gaussian of eq. gaussh, which factors over the axes): 16 pdfs
 * whose windows meet a tile share its model values as one matrix operand.
 * The tile's f - a and (f - a)^2 (a: the tile's mid-range value) are 33-bit
 * fixed-point integers relative to the tile's range, the column factors
 * 27-bit integers; their products are summed exactly as base-128 digit
 * products in int32 (v_mfma_i32_16x16x64_i8), combined in FP64 with the row
 * factors, and the tiles' contributions are added per pdf as 64-bit
 * fixed-point integers: the sums carry no accumulation error and results are
 * bit-identical from run to run. The per-axis factors are exp2(-(c t)^2) in
 * FP32 (v_exp_f32) rather than the FP64-argument factors of vup_moments: the
 * two agree to a few 1e-7 relative. A window holding a non-finite model value
 * gives NaN (mean and variance).
 * Applies to 2-D grids with single-component pdfs (ncomp == 1), at most
 * 65 535 tiles of 64 cells per axis and 2^20 tiles in all, and K < 2^26;
 * other calls run vup_moments' kernel and ignore ws.
 *   ws: dev, 256-byte aligned, ws_bytes >= vup_moments_tiled_workspace_bytes
 *   (may be NULL when that is 0). EWORKSPACE: workspace too small.
 * ------------------------------------------------------------------------ */
int vup_moments_tiled(const vup_mm* mm, const vup_dists* d, const vup_model* model, void* ws,
                      size_t ws_bytes, double* mean, double* var, double* delta2, void* stream);

/* --------------------------------------------------------------------------
 * vup_ipsa - coarse-grained IPSA quantities per column (Sec. 5.2): with bin
 * centres c_b = (e_b + e_{b+1})/2,
 *   mean_hist[k] = sum_b P[k][b] c_b,
 *   var[k]       = sum_b P[k][b] (c_b - mean_hist[k])^2   (two passes),
 *   entropy[k]   = -sum_{b: P>0} P[k][b] ln P[k][b]        (nats),
 * all accumulated in FP64. Variance and entropy are invariant under the
 * per-column translation y -> y - y(l) that turns the output matrix into the
 * IPSA probability matrix.
 *   P: dev FP32 [K][B]; mean_hist, var, entropy: dev FP64 [K] (any may be NULL).
 * ------------------------------------------------------------------------ */
int vup_ipsa(const vup_mm* mm, int64_t K, const float* P, double* mean_hist, double* var,
             double* entropy, void* stream);

/* --------------------------------------------------------------------------
 * vup_ipsa_backward - sensitivity of Q_k = g_var[k] var[k] + g_ent[k] entropy[k]
 * (the IPSA outputs of vup_ipsa) to the pdf parameters, by an adjoint sweep
 * over the same truncation windows (windows are held fixed: cells entering or
 * leaving a window are not differentiated). With v_b = dQ/dP_b =
 * g_var((c_b - E)^2 - 2 c_b S) - g_ent(ln P_b + 1), S = sum_b P_b (c_b - E):
 *   dQ/dmu_{c,d}    = pi_c Cov_{q_c}(v_bin, (x_d - mu_d)/sigma_d^2)
 *   dQ/dsigma_{c,d} = pi_c Cov_{q_c}(v_bin, (x_d - mu_d)^2/sigma_d^3)
 *   dQ/dpi_c        = E_{q_c}[v_bin]
 * where q_c is component c's normalised truncated density.
 *   P: dev FP32 [K][B] from vup_propagate (VUP_FP32); mean_hist: dev FP64 [K]
 *   from vup_ipsa; g_var, g_ent: dev FP64 [K] or NULL (= 0);
 *   g_mu, g_sigma: dev FP64 [K][ncomp][ndim]; g_weight: dev FP64 [K][ncomp] or NULL.
 * The sweep goes per run of equal bin (prefix sums of g, g t, g t^2 along the
 * fastest axis) or per cell, with the form vup_set_sweep_mode selects.
 * Invalid parameters give NaN gradients.
 * ------------------------------------------------------------------------ */
int vup_ipsa_backward(const vup_mm* mm, const vup_dists* d, const float* P,
                      const double* mean_hist, const double* g_var, const double* g_ent,
                      double* g_mu, double* g_sigma, double* g_weight, void* stream);

/* --------------------------------------------------------------------------
 * vup_eval_points - the model at arbitrary points: y[i] = M(x_i), FP64, with
 * x_i = x[i*ldx .. i*ldx + ndim). Gives the reference outputs y(l) of Sec. 5.3
 * (the model at the maximum of each input pdf, e.g. x = mu with ldx =
 * ncomp*ndim for component 0).
 *   m: host; x: dev FP64 [n][ldx], ldx >= ndim; y: dev FP64 [n].
 * EINVAL: unknown model, model/ndim mismatch, n < 0, ldx < ndim, NULL arrays.
 * ------------------------------------------------------------------------ */
int vup_eval_points(const vup_model* m, int32_t ndim, int64_t n, const double* x, int64_t ldx,
                    double* y, void* stream);

/* --------------------------------------------------------------------------
 * vup_ipsa_matrix - the IPSA probability matrix (Sec. 5.2, eq. IPSA and the
 * per-column translation y -> Delta y = y - y(l)). Column k of P is read as a
 * histogram whose mass is spread evenly over each bin [e_b, e_{b+1}); it is
 * moved by y_ref[k] and integrated over the uniform grid
 * d_j = dy_lo + j*dy_width, j = 0..n_dy:
 *   Q[k][j] = sum_b P[k][b] |[e_b - y_k, e_{b+1} - y_k) n [d_j, d_{j+1})| / (e_{b+1} - e_b)
 *   lost[k] = mass that falls outside [d_0, d_{n_dy}).
 * Computed as differences of the column's piecewise-linear FP64 CDF at
 * d_j + y_k; Q is rounded to FP32 once.
 *   P: dev FP32 [K][B] (vup_propagate's layout); y_ref: dev FP64 [K];
 *   Q: dev FP32 [K][n_dy]; lost: dev FP64 [K] or NULL. Edges and B come
 *   from the model matrix.
 * A column holding a non-finite value gives NaN in Q and lost; a non-finite
 * y_ref[k] gives Q = 0 and lost = the column's mass.
 * EINVAL: K < 0, n_dy not in [1, VUP_MAX_DY], dy_lo or dy_width not finite,
 * dy_width <= 0, NULL arrays.
 * ------------------------------------------------------------------------ */
int vup_ipsa_matrix(const vup_mm* mm, int64_t K, const float* P, const double* y_ref, double dy_lo,
                    double dy_width, int32_t n_dy, float* Q, double* lost, void* stream);

/* --------------------------------------------------------------------------
 * vup_ipsa_fields - coarse-grained field lines of each column of P (Sec. 5.2:
 * the most probable output, confidence intervals, the expected deviation from
 * y(l) and the binned form of eq. IPSAvar). With c_b = (e_b + e_{b+1})/2,
 * C_b = sum_{b'<b} P[k][b'] (FP64) and T = C_B:
 *   p_max[k]  = max_b P[k][b];   y_mode[k] = c_b of the first bin attaining it
 *   quant[k][q] = smallest y with F(y) >= levels[q] * T, F the piecewise-linear
 *               CDF through (e_b, C_b) (levels in (0, 1], fractions of T)
 *   dev[k]    = sum_b P[k][b] (c_b - y_ref[k])
 *   delta2[k] = 1/2 sum_b P[k][b] (c_b - y_ref[k])^2
 *   P: dev FP32 [K][B]; y_ref: dev FP64 [K] (needed for dev and delta2);
 *   levels: host FP64 [n_levels], n_levels <= VUP_MAX_LEVELS;
 *   y_mode, p_max, dev, delta2: dev FP64 [K] or NULL; quant: dev FP64
 *   [K][n_levels] or NULL.
 * A column holding a non-finite value gives NaN everywhere; a column of zeros
 * gives p_max = dev = delta2 = 0 and NaN for y_mode and the quantiles.
 * EINVAL: K < 0, bad n_levels or a level outside (0, 1], dev/delta2 without
 * y_ref, NULL P.
 * ------------------------------------------------------------------------ */
int vup_ipsa_fields(const vup_mm* mm, int64_t K, const float* P, const double* y_ref,
                    int32_t n_levels, const double* levels, double* y_mode, double* p_max,
                    double* quant, double* dev, double* delta2, void* stream);

/* --------------------------------------------------------------------------
 * vup_marginalize - global values over locations (Sec. 5.2: marginalising
 * the per-location matrices with the measurement-location probability rho):
 *   out[j] = sum_k rho[k] A[k][j]       (rho NULL: rho_k = 1/K),
 * FP64, in a fixed order (repeatable bit for bit). A is any [K][n] FP32
 * matrix: P from vup_propagate (n = B) or Q from vup_ipsa_matrix (n = n_dy).
 *   A: dev FP32 [K][n]; rho: dev FP64 [K] or NULL; out: dev FP64 [n];
 *   ws: dev scratch of vup_marginal_workspace_bytes(K, n) bytes (may be
 *   NULL when that is 0), owned by the caller and reusable after the call's
 *   work on `stream` has finished.
 * EINVAL: K < 0, n not in [1, VUP_MAX_MARGINAL_COLS], NULL A or out;
 * EWORKSPACE: workspace too small.
 * ------------------------------------------------------------------------ */
size_t vup_marginal_workspace_bytes(int64_t K, int32_t n);
int vup_marginalize(int64_t K, int32_t n, const float* A, const double* rho, void* ws,
                    size_t ws_bytes, double* out, void* stream);

/* --------------------------------------------------------------------------
 * vup_marginalize_noalloc - vup_marginalize for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same result, bit for bit, with the partial sums
 * held in a device array the library owns (VUP_NOALLOC_SCRATCH_BYTES per GPU,
 * kept until the process ends) instead of a caller workspace. The call makes
 * no allocation of any kind; the caller still passes A, rho and out.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other host threads) race and must be serialised by the
 * caller. Nothing in the array needs clearing between calls.
 *   Arguments and errors as vup_marginalize, plus EUNSUPPORTED when
 *   vup_marginal_workspace_bytes(K, n) > VUP_NOALLOC_SCRATCH_BYTES, which
 *   happens exactly when n > 1048576 (any K), checked before anything is
 *   enqueued.
 * ------------------------------------------------------------------------ */
#define VUP_NOALLOC_SCRATCH_BYTES (8 << 20)
int vup_marginalize_noalloc(int64_t K, int32_t n, const float* A, const double* rho,
                            double* out, void* stream);

/* --------------------------------------------------------------------------
 * vup_posterior - Bayes inversion over the model matrix (Sec. 3, the Bayes
 * theorem paragraph and its footnote): columns of the "inverted model matrix"
 * for the selected distributions k = sel[t],
 *   post[t][i] = p_k(x_i) / P[k][bin(i)]   (0 for a cell without a bin, or
 *                                            whose bin has no mass),
 * the posterior over input cells given that the output fell in that cell's
 * bin, relative to the forward propagation that produced P and Z. Applied
 * after the model matrix it returns the input pdf (the footnote's identity:
 * sum_b post[i] P[k][b] [bin(i) = b] = p_k(x_i)), and over the cells of one
 * bin it sums to 1. p_k is the truncated, normalised mixture the propagation
 * uses (FP32 per-axis factors, normalised by Z in FP64; the factors of an axis
 * of a pdf far narrower than a cell are scaled by the same power of two as in
 * vup_propagate, and the scale is divided out of Z exactly).
 * Optional per-bin posterior means E[x_d | y in b, k] = sum over the bin's
 * cells of post x_d (FP64, summed in the compressed-by-bin order).
 *   d: the distributions given to vup_propagate; sel: dev int64 [n_sel]
 *   (an index outside [0, K) gives a NaN row); P: dev FP32 [K][B] and Z: dev
 *   FP64 [K][ncomp] from vup_propagate (VUP_FP32); post: dev FP32
 *   [n_sel][N]; mean: dev FP64 [n_sel][B][ndim] or NULL.
 * Invalid parameters or non-finite Z or evidence give NaN.
 * EINVAL: bad descriptor or dists, NULL arrays; EUNSUPPORTED: n_sel > 65535.
 * ------------------------------------------------------------------------ */
int vup_posterior(const vup_mm* mm, const vup_dists* d, int64_t n_sel, const int64_t* sel,
                  const float* P, const double* Z, float* post, double* mean, void* stream);

/* --------------------------------------------------------------------------
 * vup_counters - reads and clears the device-side event counters of a model
 * matrix's workspace. Synchronises `stream`.
 *   out (host int64[4]): [0] cells with no bin (set by vup_bin),
 *   [1] bad_edges (vup_bin), [2] components with invalid parameters,
 *   [3] distributions whose every window is empty (vup_propagate).
 * ------------------------------------------------------------------------ */
int vup_counters(const vup_mm* mm, void* stream, int64_t* out);

/* --------------------------------------------------------------------------
 * vup_set_sweep_mode - how vup_propagate (FP32 densities) accumulates over a
 * model matrix: per cell, or per run of equal bin along the fastest axis
 * (both give the same results up to rounding).
 *   VUP_SWEEP_CELLS / VUP_SWEEP_RUNS force one form; enqueued on `stream`.
 *   VUP_SWEEP_AUTO synchronises `stream`, reads the run statistics of the
 *   model matrix and fixes the form: runs when the mean run is at least 3
 *   cells, else cells. It is meant for set-up time.
 * Right after vup_bin, mm->sweep is VUP_SWEEP_AUTO and unresolved: each
 * vup_propagate then enqueues both forms and the device picks one by the
 * same rule (the other returns at once). The run form needs a fastest axis
 * of at most 65534 cells and fewer than 2^30 cells; otherwise cells are used.
 * ------------------------------------------------------------------------ */
#define VUP_SWEEP_AUTO 0
#define VUP_SWEEP_CELLS 1
#define VUP_SWEEP_RUNS 2
int vup_set_sweep_mode(vup_mm* mm, int32_t mode, void* stream);

/* last error message of the calling thread ("" if none). */
const char* vup_last_error(void);

/* library version string */
const char* vup_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VUP_H */
