"""Pins of the FP64 CPU oracle against things other than itself.

Each test names the paper passage (or the mathematics) that fixes the value.
None of them re-calls the oracle's own routine to produce the expectation:
expectations come from closed forms, brute force written differently
(dense matrices, per-axis sums, masks from the inequality itself), library
routines (numpy histogram / searchsorted / argsort, scipy truncnorm, torch
dtype conversions) or Monte Carlo sampling.
"""
import math
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_pairs(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([float(t) for t in line.split()])
    return rows


def _centres(n, lo, hi):
    """cell centres of each axis (composite midpoint rule, Sec. 3)."""
    return [lo[d] + (np.arange(n[d]) + 0.5) * ((hi[d] - lo[d]) / n[d]) for d in range(len(n))]


def _mesh(n, lo, hi):
    xs = _centres(n, lo, hi)
    return [m.ravel() for m in np.meshgrid(*xs, indexing="ij")]


def _dense_input_matrix(n, lo, hi, mu, sigma, ns=4.0):
    """N x K input probability matrix of eq. VUP, built densely from the
    definition: Gaussian (eq. gaussh) at cell centres, kept where
    |x_d - mu_d| <= ns*sigma_d on every axis, normalised per column."""
    X = _mesh(n, lo, hi)
    K = mu.shape[0]
    N = X[0].size
    Pin = np.zeros((N, K))
    for k in range(K):
        s = np.zeros(N)
        keep = np.ones(N, dtype=bool)
        for d in range(len(n)):
            t = (X[d] - mu[k, 0, d]) / sigma[k, 0, d]
            s += t * t
            keep &= np.abs(X[d] - mu[k, 0, d]) <= ns * sigma[k, 0, d]
        w = np.where(keep, np.exp(-0.5 * s), 0.0)
        Pin[:, k] = w / w.sum()
    return Pin


# --------------------------------------------------------------------------
# model evaluation and grid (Alg. VUP: uniform grid, evaluate the model)
# --------------------------------------------------------------------------
def test_model_special_values(orc):
    # values at points where the closed form is exact by hand
    assert orc.model_at("sincos2", [0.0, 0.0]) == 0.5
    assert orc.model_at("sincos2", [math.pi / 2, math.pi / 2]) == pytest.approx(
        1.0 - 0.5 + (math.pi / 2) ** 2 / 4, abs=1e-15)
    assert orc.model_at("damped3", [0.0, 1.0, 2.0]) == pytest.approx(0.0, abs=1e-15)
    assert orc.model_at("damped3", [math.pi / 2, 0.0, 0.0]) == pytest.approx(1.0, abs=1e-15)
    assert orc.model_at("ring4", [0.0, 0.0, 0.0, 0.0]) == 0.0
    assert orc.model_at("ring4", [1.0, 1.0, 1.0, 1.0]) == pytest.approx(
        4 * math.sin(1.0) + 0.05 * 16, abs=1e-14)
    assert orc.model_at("timing2", [math.pi / 2, math.pi / 2]) == pytest.approx(8.1, abs=1e-14)
    assert orc.model_at("ipsa2", [0.0, 0.25]) == 0.25
    assert orc.model_at("linear", [2.0, -1.0], theta=(0.5, 3.0, 4.0)) == 0.5 + 6.0 - 4.0


def test_grid_is_cell_centred_row_major(orc):
    # linear model returning x1 exposes the centre of axis 1 in flat order;
    # axis 0 slowest (row major)
    n, lo, hi = (3, 4), (0.0, -1.0), (3.0, 1.0)
    f0 = orc.eval_grid(n, lo, hi, "linear", (0.0, 1.0, 0.0))
    f1 = orc.eval_grid(n, lo, hi, "linear", (0.0, 0.0, 1.0))
    assert np.array_equal(f0.reshape(3, 4)[:, 0], np.array([0.5, 1.5, 2.5]))
    assert np.array_equal(f1.reshape(3, 4)[0], np.array([-0.75, -0.25, 0.25, 0.75]))


# --------------------------------------------------------------------------
# bins and model matrix (eq. (4), eq. (5), eq. MUP)
# --------------------------------------------------------------------------
def test_uniform_edges_and_bins_vs_numpy(orc):
    rng = np.random.default_rng(1)
    f = rng.normal(size=5000)
    f[17] = np.nan
    B = 37
    e = orc.uniform_edges(f, B)
    fin = f[np.isfinite(f)]
    assert e[0] == fin.min() and e[-1] == fin.max()
    assert np.allclose(e, np.linspace(fin.min(), fin.max(), B + 1), rtol=0, atol=4e-16 * 8)
    b = orc.bins(f, e)
    # library routine: searchsorted(side='right') - 1, last bin closed
    ref = np.searchsorted(e, f, side="right") - 1
    ref[f == e[-1]] = B - 1
    ref[(f < e[0]) | (f > e[-1]) | ~np.isfinite(f)] = -1
    assert np.array_equal(b, ref.astype(np.int32))
    # np.histogram uses the same half-open / last-closed partition
    cnt, _ = np.histogram(fin, bins=e)
    assert np.array_equal(np.bincount(b[b >= 0], minlength=B), cnt)


def test_bins_outside_and_nan(orc):
    e = np.array([0.0, 1.0, 2.0, 3.0])
    f = np.array([-1e-300, 0.0, 0.999, 1.0, 3.0, 3.0000000000000004, np.nan, np.inf])
    assert orc.bins(f, e).tolist() == [-1, 0, 0, 1, 2, -1, -1, -1]


def test_model_matrix_is_stable_sort_by_bin(orc):
    rng = np.random.default_rng(2)
    b = rng.integers(-1, 9, size=3000).astype(np.int32)
    off, perm = orc.model_matrix(b, 9)
    keep = np.nonzero(b >= 0)[0]
    ref = keep[np.argsort(b[keep], kind="stable")]
    assert np.array_equal(perm, ref)
    assert np.array_equal(np.diff(off), np.bincount(b[keep], minlength=9))
    # one nonzero per column: every binned cell appears exactly once
    assert np.array_equal(np.sort(perm), keep)


# --------------------------------------------------------------------------
# truncation windows (eq. gaussh truncated per axis; Sec. 5.3 truncation)
# --------------------------------------------------------------------------
def test_windows_match_inequality_mask(orc):
    n, lo, hi = (40, 23, 17), (-1.0, 0.0, -2.5), (1.0, 3.0, 0.5)
    rng = np.random.default_rng(3)
    K = 300
    mu = rng.uniform(-3, 3, size=(K, 1, 3))
    sigma = rng.uniform(0.01, 0.8, size=(K, 1, 3))
    win, bad, U = orc.windows(n, lo, hi, mu, sigma, 4.0)
    xs = _centres(n, lo, hi)
    total = 0
    for k in range(K):
        cells = 1
        for d in range(3):
            keep = np.nonzero(np.abs(xs[d] - mu[k, 0, d]) <= 4.0 * sigma[k, 0, d])[0]
            a, b = win[k, 0, d]
            if keep.size:
                assert (a, b) == (keep[0], keep[-1])
            else:
                # narrower than a cell: the cell holding mu, if mu is in the domain
                if lo[d] <= mu[k, 0, d] <= hi[d]:
                    j = min(int((mu[k, 0, d] - lo[d]) // ((hi[d] - lo[d]) / n[d])), n[d] - 1)
                    assert a == b == j
                else:
                    assert b < a
            cells *= max(0, b - a + 1)
        total += cells
    assert U == total and not bad.any()


def test_windows_bad_and_delta(orc):
    n, lo, hi = (10,), (0.0,), (1.0,)
    mu = np.array([[[0.55]], [[0.5]], [[5.0]], [[0.3]]])
    sigma = np.array([[[1e-7]], [[0.0]], [[0.1]], [[np.nan]]])
    win, bad, U = orc.windows(n, lo, hi, mu, sigma)
    assert tuple(win[0, 0, 0]) == (5, 5) and not bad[0, 0]
    assert bad[1, 0] and bad[3, 0]
    assert win[2, 0, 0, 1] < win[2, 0, 0, 0] and not bad[2, 0]
    assert U == 1


# --------------------------------------------------------------------------
# propagation: eq. (5) / eq. VUP
# --------------------------------------------------------------------------
def test_literal_vup_dense_matmul(orc):
    """P5: the dense one-hot model matrix (B x N) times the dense N x K input
    probability matrix, exactly as eq. VUP writes it."""
    n, lo, hi = (8, 8), (-1.0, -1.0), (1.0, 1.0)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    e = orc.uniform_edges(f, 5)
    b = orc.bins(f, e)
    rng = np.random.default_rng(4)
    mu = rng.uniform(-1, 1, size=(7, 1, 2))
    sigma = rng.uniform(0.1, 0.6, size=(7, 1, 2))
    M = np.zeros((5, b.size))
    M[b, np.arange(b.size)] = 1.0
    ref = M @ _dense_input_matrix(n, lo, hi, mu, sigma)
    P, Z = orc.propagate(n, lo, hi, b, 5, mu, sigma)
    assert np.allclose(P, ref.T, rtol=0, atol=1e-15)


def test_two_stage_alg_vup_equals_direct(orc):
    """P6: Alg. VUP as printed (UniqueSorted, sparse 1s, sparse multiply, then
    MarginalizeBin into B bins) gives the same column as direct binning."""
    import scipy.sparse as sp
    n, lo, hi = (24, 20), (-2.0, -2.0), (2.0, 2.0)
    f = orc.eval_grid(n, lo, hi, "timing2")
    B = 11
    e = orc.uniform_edges(f, B)
    rng = np.random.default_rng(5)
    mu = rng.uniform(-1.5, 1.5, size=(5, 1, 2))
    sigma = rng.uniform(0.2, 1.0, size=(5, 1, 2))
    yu, inv = np.unique(f, return_inverse=True)
    Mu = sp.csr_matrix((np.ones(f.size), (inv, np.arange(f.size))), shape=(yu.size, f.size))
    Pp = Mu @ _dense_input_matrix(n, lo, hi, mu, sigma)          # N_y x K
    jb = np.searchsorted(e, yu, side="right") - 1
    jb[yu == e[-1]] = B - 1
    ref = np.zeros((B, 5))
    np.add.at(ref, jb, Pp)
    P, _ = orc.propagate(n, lo, hi, orc.bins(f, e), B, mu, sigma)
    assert np.allclose(P, ref.T, rtol=0, atol=1e-14)


def test_columns_normalised_and_nonnegative(orc):
    """P1: each input column is normalised (Alg. VUP), the model matrix has one
    nonzero per column, so every output column sums to one."""
    wl = workloads.grid64()
    out = orc.run_workload(wl, with_moments=False)
    assert (out["P"] >= 0).all()
    assert np.allclose(out["P"].sum(axis=1), 1.0, rtol=0, atol=1e-13)


def test_delta_input_is_one_hot(orc):
    """P2: a certain input (eq. (1), the delta model propagator) lands in a
    single bin: bin(f(mu)), with E = f(mu), Var = 0 and zero entropy."""
    n, lo, hi = (30, 20), (-3.0, -3.0), (3.0, 3.0)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    e = orc.uniform_edges(f, 16)
    b = orc.bins(f, e)
    h = [(hi[d] - lo[d]) / n[d] for d in range(2)]
    cells = [(3, 7), (29, 0), (15, 19)]
    mu = np.array([[[lo[0] + (i + 0.5) * h[0], lo[1] + (j + 0.5) * h[1]]] for i, j in cells])
    sigma = np.array([[[1e-6 * h[0], 1e-6 * h[1]]]] * 3)
    P, Z = orc.propagate(n, lo, hi, b, 16, mu, sigma)
    mean, var, _ = orc.moments(n, lo, hi, f, mu, sigma)
    mh, vh, ent = orc.ipsa(P, e)
    for r, (i, j) in enumerate(cells):
        onehot = np.zeros(16)
        onehot[b[i * 20 + j]] = 1.0
        assert np.array_equal(P[r], onehot)
        assert mean[r] == f[i * 20 + j] and var[r] == 0.0 and ent[r] == 0.0


def test_uniform_limit_is_numpy_histogram(orc):
    """P4: a pdf much wider than the domain weights every cell equally, so the
    output is the plain histogram of f over the grid divided by N."""
    n, lo, hi = (33, 41), (-3.0, -3.0), (3.0, 3.0)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    e = orc.uniform_edges(f, 13)
    mu = np.array([[[0.0, 0.0]]])
    sigma = np.array([[[1e7, 1e7]]])
    P, _ = orc.propagate(n, lo, hi, orc.bins(f, e), 13, mu, sigma)
    cnt, _ = np.histogram(f, bins=e)
    assert np.allclose(P[0], cnt / f.size, rtol=1e-12, atol=0)


def test_mixture_is_linear_in_components(orc):
    """P14: components are normalised separately and mixed with their weights."""
    n, lo, hi = (20, 18), (-2.0, -2.0), (2.0, 2.0)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    e = orc.uniform_edges(f, 9)
    b = orc.bins(f, e)
    rng = np.random.default_rng(6)
    mu = rng.uniform(-1.5, 1.5, size=(6, 2, 2))
    sigma = rng.uniform(0.1, 0.7, size=(6, 2, 2))
    wt = rng.dirichlet([1, 1], size=6)
    P, Z = orc.propagate(n, lo, hi, b, 9, mu, sigma, wt)
    P1, _ = orc.propagate(n, lo, hi, b, 9, mu[:, :1], sigma[:, :1])
    P2, _ = orc.propagate(n, lo, hi, b, 9, mu[:, 1:], sigma[:, 1:])
    assert np.allclose(P, wt[:, :1] * P1 + wt[:, 1:] * P2, rtol=0, atol=1e-15)
    one = np.tile([1.0, 0.0], (6, 1))
    Pr, _ = orc.propagate(n, lo, hi, b, 9, mu, sigma, one)
    assert np.allclose(Pr, P1, rtol=0, atol=1e-15)


def test_normaliser_is_product_of_axis_sums(orc):
    """P10: the truncated Gaussian is separable, Z = prod_d Z_d with 1-D sums."""
    n, lo, hi = (25, 31, 19), (-1.0, -2.0, 0.0), (1.0, 2.0, 3.0)
    rng = np.random.default_rng(7)
    mu = rng.uniform(-0.5, 0.5, size=(4, 1, 3)) + np.array([0, 0, 1.5])
    sigma = rng.uniform(0.1, 0.5, size=(4, 1, 3))
    f = orc.eval_grid(n, lo, hi, "damped3")
    e = orc.uniform_edges(f, 7)
    _, Z = orc.propagate(n, lo, hi, orc.bins(f, e), 7, mu, sigma)
    xs = _centres(n, lo, hi)
    for k in range(4):
        prod = 1.0
        for d in range(3):
            m, s = mu[k, 0, d], sigma[k, 0, d]
            keep = np.abs(xs[d] - m) <= 4 * s
            prod *= np.exp(-0.5 * ((xs[d][keep] - m) / s) ** 2).sum()
        assert Z[k, 0] == pytest.approx(prod, rel=1e-13)


# --------------------------------------------------------------------------
# moments (exact f) and the IPSA local deviation eq. IPSAvar
# --------------------------------------------------------------------------
def test_linear_model_closed_form_moments(orc):
    """P3: for a linear model the output mean and variance are fixed by the
    per-axis discrete moments of the truncated Gaussian (1-D sums)."""
    n, lo, hi = (64, 48, 40), (-3.0, -2.0, -1.0), (3.0, 2.0, 1.0)
    theta = (0.7, 1.5, -2.0, 0.25)
    f = orc.eval_grid(n, lo, hi, "linear", theta)
    rng = np.random.default_rng(8)
    mu = rng.uniform(-0.5, 0.5, size=(6, 1, 3))
    sigma = rng.uniform(0.05, 0.3, size=(6, 1, 3))
    mean, var, _ = orc.moments(n, lo, hi, f, mu, sigma)
    xs = _centres(n, lo, hi)
    for k in range(6):
        Em, V = theta[0], 0.0
        for d in range(3):
            m, s = mu[k, 0, d], sigma[k, 0, d]
            x = xs[d][np.abs(xs[d] - m) <= 4 * s]
            g = np.exp(-0.5 * ((x - m) / s) ** 2)
            md = (g * x).sum() / g.sum()
            Em += theta[d + 1] * md
            V += theta[d + 1] ** 2 * ((g * (x - md) ** 2).sum() / g.sum())
        assert mean[k] == pytest.approx(Em, abs=1e-13)
        assert var[k] == pytest.approx(V, rel=1e-11)


def test_fine_grid_variance_matches_truncated_normal(orc):
    """P3 continuous limit: on a fine 1-D grid the discrete variance of the
    4-sigma truncated Gaussian approaches the closed form (golden)."""
    from scipy.stats import truncnorm
    gold = _golden_pairs("truncnorm_4sigma.txt")[0][0]
    assert truncnorm(-4, 4).var() == pytest.approx(gold, rel=1e-12)
    n, lo, hi = (20000,), (-1.0,), (1.0,)
    f = orc.eval_grid(n, lo, hi, "linear", (0.0, 1.0))
    mu = np.array([[[0.0]]])
    sigma = np.array([[[0.2]]])
    _, var, _ = orc.moments(n, lo, hi, f, mu, sigma)
    assert var[0] / 0.04 == pytest.approx(gold, rel=1e-5)


def test_moments_match_continuous_monte_carlo(orc):
    """P7(ii): quadrature moments of a smooth model agree with Monte Carlo over
    the continuous truncated Gaussian (Alg. MC with random samples), within
    the sampling error."""
    from scipy.stats import truncnorm
    n, lo, hi = (400, 400), (-3.0, -3.0), (3.0, 3.0)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    mu = np.array([[[0.4, -0.7]]])
    sigma = np.array([[[0.3, 0.45]]])
    mean, var, _ = orc.moments(n, lo, hi, f, mu, sigma)
    rng = np.random.default_rng(9)
    S = 400000
    x0 = truncnorm(-4, 4, loc=0.4, scale=0.3).rvs(S, random_state=rng)
    x1 = truncnorm(-4, 4, loc=-0.7, scale=0.45).rvs(S, random_state=rng)
    y = np.sin(x0) + 0.5 * np.cos(2 * x1) + x0 * x1 / 4
    se = y.std() / math.sqrt(S)
    assert abs(mean[0] - y.mean()) < 5 * se
    assert var[0] == pytest.approx(y.var(), rel=0.02)


def test_histogram_matches_discrete_monte_carlo(orc):
    """P7(i): Alg. MC drawing grid cells from the discrete input pdf and binning
    their outputs agrees with VUP's column (chi-square at a fixed seed)."""
    from scipy.stats import chi2
    n, lo, hi = (50, 50), (-3.0, -3.0), (3.0, 3.0)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    B = 12
    e = orc.uniform_edges(f, B)
    b = orc.bins(f, e)
    mu = np.array([[[0.2, 0.9]]])
    sigma = np.array([[[0.6, 0.5]]])
    p = _dense_input_matrix(n, lo, hi, mu, sigma)[:, 0]
    rng = np.random.default_rng(10)
    S = 200000
    cells = rng.choice(p.size, size=S, p=p)
    obs = np.bincount(b[cells], minlength=B)
    P, _ = orc.propagate(n, lo, hi, b, B, mu, sigma)
    exp_ = P[0] * S
    m = exp_ > 5
    stat = ((obs[m] - exp_[m]) ** 2 / exp_[m]).sum()
    assert stat < chi2(m.sum() - 1).ppf(0.999)


def test_delta2_identity_and_sheppard(orc):
    """P9: Var >= 0; eq. IPSAvar carries 1/2, so Var = 2 Delta^2 - (E - M(mu))^2;
    for wide pdfs the binned variance exceeds the exact one by ~ w^2/12."""
    n, lo, hi = (120, 100), (-3.0, -3.0), (3.0, 3.0)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    rng = np.random.default_rng(11)
    mu = rng.uniform(-1, 1, size=(5, 1, 2))
    sigma = rng.uniform(0.3, 0.6, size=(5, 1, 2))
    fmu = np.array([orc.model_at("sincos2", mu[k, 0]) for k in range(5)])
    mean, var, d2 = orc.moments(n, lo, hi, f, mu, sigma, fmu=fmu)
    assert (var >= 0).all()
    assert np.allclose(var, 2 * d2 - (mean - fmu) ** 2, rtol=1e-10, atol=1e-14)
    # Sheppard: needs a smooth output density, so a linear model on a fine grid
    # with an irrational slope ratio (a rational one puts the output values on a
    # lattice that aliases against the bins)
    n2 = (500, 500)
    fl = orc.eval_grid(n2, lo, hi, "linear", (0.0, 1.0, 0.7071067811865476))
    B = 60
    e = orc.uniform_edges(fl, B)
    mus = rng.uniform(-1, 1, size=(40, 1, 2))
    sg = np.full((40, 1, 2), 0.6)
    _, varl, _ = orc.moments(n2, lo, hi, fl, mus, sg)
    P, _ = orc.propagate(n2, lo, hi, orc.bins(fl, e), B, mus, sg)
    _, vh, _ = orc.ipsa(P, e)
    w = e[1] - e[0]
    assert np.allclose(vh - varl, w * w / 12, rtol=0.01, atol=0)


# --------------------------------------------------------------------------
# IPSA coarse-grained quantities (Sec. 5.2)
# --------------------------------------------------------------------------
def test_entropy_closed_forms(orc):
    """P8: one-hot -> 0; uniform over m bins -> ln m; bounds; shift invariance."""
    B = 10
    e = np.linspace(0.0, 1.0, B + 1)
    P = np.zeros((4, B))
    P[0, 3] = 1.0
    P[1, 2:7] = 0.2
    P[2] = 1.0 / B
    rng = np.random.default_rng(12)
    q = rng.random(6)
    P[3, 1:7] = q / q.sum()
    m, v, h = orc.ipsa(P, e)
    assert h[0] == 0.0 and v[0] == 0.0 and m[0] == pytest.approx(0.35, abs=1e-15)
    assert h[1] == pytest.approx(math.log(5), rel=1e-14)
    assert h[2] == pytest.approx(math.log(B), rel=1e-14)
    Ps = np.roll(P[3:4], 2, axis=1)
    ms, vs, hs = orc.ipsa(Ps, e)
    assert hs[0] == pytest.approx(h[3], rel=1e-14) and vs[0] == pytest.approx(v[3], rel=1e-12)
    assert ms[0] == pytest.approx(m[3] + 0.2, abs=1e-14)
    # binned variance of a uniform column over m adjacent bins: (m^2 - 1) w^2 / 12
    assert v[1] == pytest.approx((25 - 1) * 0.01 / 12, rel=1e-12)


# --------------------------------------------------------------------------
# IPSA sensitivity gradient: analytic vs finite differences (frozen windows)
# --------------------------------------------------------------------------
def _fd_grad(orc, n, lo, hi, b, e, mu, sigma, wt, win, gv, ge, h=1e-4):
    K, C, d = mu.shape
    gm = np.zeros_like(mu)
    gs = np.zeros_like(sigma)
    for c in range(C):
        for a in range(d):
            for arr, out in ((mu, gm), (sigma, gs)):
                p = arr.copy()
                p[:, c, a] += h
                m = arr.copy()
                m[:, c, a] -= h
                args_p = (p, sigma, wt) if arr is mu else (mu, p, wt)
                args_m = (m, sigma, wt) if arr is mu else (mu, m, wt)
                qp = orc.objective(n, lo, hi, b, e, *args_p, win, gv, ge)
                qm = orc.objective(n, lo, hi, b, e, *args_m, win, gv, ge)
                out[:, c, a] = (qp - qm) / (2 * h)
    return gm, gs


@pytest.mark.parametrize("C", [1, 2])
def test_ipsa_gradient_vs_central_fd(orc, C):
    """P11: analytic gradient of g_var*Var + g_ent*H equals FP64 central finite
    differences (h = 1e-4) on frozen windows."""
    n, lo, hi = (40, 36), (-3.0, -3.0), (3.0, 3.0)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    B = 24
    e = orc.uniform_edges(f, B)
    b = orc.bins(f, e)
    rng = np.random.default_rng(13 + C)
    K = 5
    mu = rng.uniform(-2, 2, size=(K, C, 2))
    sigma = rng.uniform(0.25, 0.6, size=(K, C, 2))
    wt = rng.dirichlet(np.ones(C), size=K) if C > 1 else None
    win, _, _ = orc.windows(n, lo, hi, mu, sigma)
    gv = rng.uniform(0.5, 1.5, size=K)
    ge = rng.uniform(0.5, 1.5, size=K)
    P, _ = orc.propagate(n, lo, hi, b, B, mu, sigma, wt, win=win)
    gm, gs, gw = orc.ipsa_grad(n, lo, hi, b, e, mu, sigma, wt, win, P, gv, ge)
    fm, fs = _fd_grad(orc, n, lo, hi, b, e, mu, sigma, wt, win, gv, ge)
    scale = max(np.abs(gm).max(), np.abs(gs).max())
    assert np.allclose(gm, fm, rtol=1e-5, atol=1e-8 * scale)
    assert np.allclose(gs, fs, rtol=1e-5, atol=1e-8 * scale)
    if C > 1:
        # weights: FD along the simplex tangent (pi1 + h, pi2 - h) checks g1 - g2
        hh = 1e-5
        wp = wt.copy()
        wp[:, 0] += hh
        wp[:, 1] -= hh
        wm = wt.copy()
        wm[:, 0] -= hh
        wm[:, 1] += hh
        qp = orc.objective(n, lo, hi, b, e, mu, sigma, wp, win, gv, ge)
        qm = orc.objective(n, lo, hi, b, e, mu, sigma, wm, win, gv, ge)
        assert np.allclose(gw[:, 0] - gw[:, 1], (qp - qm) / (2 * hh), rtol=1e-5,
                           atol=1e-8 * np.abs(gw).max())


def test_ipsa_gradient_vs_central_fd_grid1024_subset(orc):
    """P11 at the full 1024^2 size: the 64 seeded locations of the gradient
    subset of the 1024^2 configuration (sigma ~ U[0.05, 0.5], B = 256), all
    four parameters each (mu and sigma per axis), FP64 central differences
    with h = 1e-4 on frozen windows against the analytic gradient. The central
    difference's truncation error is about (h/sigma)^2/6 <= 7e-7 of the
    derivative, so rtol 1e-5 holds with margin."""
    wl = workloads.grid1024()
    ks = workloads.fd_subset(wl.K, 64)
    sub = wl.subset(ks)
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model)
    e = orc.uniform_edges(f, wl.B)
    b = orc.bins(f, e)
    win, _, _ = orc.windows(wl.n, wl.lo, wl.hi, sub.mu, sub.sigma)
    rng = np.random.default_rng(41)
    gv = rng.uniform(0.5, 1.5, size=sub.K)
    ge = rng.uniform(0.5, 1.5, size=sub.K)
    P, _ = orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, sub.mu, sub.sigma, win=win)
    gm, gs, _ = orc.ipsa_grad(wl.n, wl.lo, wl.hi, b, e, sub.mu, sub.sigma, None, win, P, gv, ge)
    fm, fs = _fd_grad(orc, wl.n, wl.lo, wl.hi, b, e, sub.mu, sub.sigma, None, win, gv, ge)
    scale = max(np.abs(gm).max(), np.abs(gs).max())
    assert np.allclose(gm, fm, rtol=1e-5, atol=1e-9 * scale)
    assert np.allclose(gs, fs, rtol=1e-5, atol=1e-9 * scale)
    # the isotropic pdf's two sigma partials are not equal at a generic
    # location (the test would not notice an axis swap otherwise)
    assert np.abs(gs[:, 0, 0] - gs[:, 0, 1]).max() > 1e-3 * scale


def test_ipsa_gradient_with_mass_outside_the_bins(orc):
    """P11 with edges that leave part of the output range uncovered, so columns
    sum to less than one and the variance derivative keeps its -2 c_b S term."""
    n, lo, hi = (36, 30), (-3.0, -3.0), (3.0, 3.0)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    B = 16
    e = np.linspace(np.quantile(f, 0.2), np.quantile(f, 0.9), B + 1)
    b = orc.bins(f, e)
    assert (b < 0).any()
    rng = np.random.default_rng(31)
    K = 4
    mu = rng.uniform(-1.5, 1.5, size=(K, 1, 2))
    sigma = rng.uniform(0.4, 0.8, size=(K, 1, 2))
    win, _, _ = orc.windows(n, lo, hi, mu, sigma)
    gv = np.ones(K)
    ge = np.full(K, 0.5)
    P, _ = orc.propagate(n, lo, hi, b, B, mu, sigma, win=win)
    assert (P.sum(axis=1) < 0.999).all()
    gm, gs, _ = orc.ipsa_grad(n, lo, hi, b, e, mu, sigma, None, win, P, gv, ge)
    fm, fs = _fd_grad(orc, n, lo, hi, b, e, mu, sigma, None, win, gv, ge)
    scale = max(np.abs(gm).max(), np.abs(gs).max())
    assert np.allclose(gm, fm, rtol=1e-5, atol=1e-8 * scale)
    assert np.allclose(gs, fs, rtol=1e-5, atol=1e-8 * scale)


def test_gradient_symmetry_zero_for_even_model(orc):
    """P11 symmetry: for an output that is even about mu on every axis (here
    f = x0^2 + x1^2 centred on a grid symmetric about mu) the mu-gradient of
    both variance and entropy vanishes."""
    n, lo, hi = (40, 40), (-2.0, -2.0), (2.0, 2.0)
    X = _mesh(n, lo, hi)
    f = X[0] ** 2 + X[1] ** 2
    e = orc.uniform_edges(f, 16)
    b = orc.bins(f, e)
    mu = np.zeros((1, 1, 2))
    sigma = np.array([[[0.4, 0.3]]])
    win, _, _ = orc.windows(n, lo, hi, mu, sigma)
    P, _ = orc.propagate(n, lo, hi, b, 16, mu, sigma, win=win)
    gm, gs, _ = orc.ipsa_grad(n, lo, hi, b, e, mu, sigma, None, win, P, np.ones(1), np.ones(1))
    assert np.abs(gm).max() < 1e-12 * max(1.0, np.abs(gs).max())


# --------------------------------------------------------------------------
# density quantisers (reduced-precision variants)
# --------------------------------------------------------------------------
def test_quantisers_golden(orc):
    for x, y in _golden_pairs("bf16_rounding.txt"):
        assert orc.round_bf16(x) == y
    for x, y in _golden_pairs("e4m3_rounding.txt"):
        assert orc.round_e4m3(x) == y


def test_quantisers_vs_torch_conversion(orc):
    """library routine: torch's float32 -> bfloat16 / float8_e4m3fn casts (RNE)."""
    import torch
    rng = np.random.default_rng(14)
    x = np.concatenate([rng.random(3000), 10.0 ** rng.uniform(-12, 0, 3000)]).astype(np.float32)
    tb = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal([orc.round_bf16(float(v)) for v in x], tb)
    y = (x.astype(np.float64) * 448.0).astype(np.float32)
    t8 = torch.from_numpy(y).to(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    assert np.array_equal([orc.round_e4m3(float(v)) for v in y], t8)


def test_reduced_precision_columns_still_sum_to_one(orc):
    """Z is the sum of the same quantised values, so every variant normalises."""
    wl = workloads.random_workload("q", (30, 26), (-3, -3), (3, 3), "sincos2", 20, 9, 2,
                                   (0.1, 0.6), seed=15)
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model)
    e = orc.uniform_edges(f, wl.B)
    b = orc.bins(f, e)
    P64, _ = orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, wl.mu, wl.sigma, wl.weight)
    for prec, tol in (("bf16", 2 * 2.0 ** -8), ("bf16x2", 1e-4), ("fp8e4m3", 0.13)):
        P, _ = orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, wl.mu, wl.sigma, wl.weight,
                             precision=prec)
        assert np.allclose(P.sum(axis=1), 1.0, atol=1e-13)
        assert np.abs(P - P64).sum(axis=1).max() <= tol


@pytest.mark.parametrize("precision", ["bf16", "bf16x2", "fp8e4m3"])
def test_rounding_l1_bound_covers_perturbed_roundings(orc, precision):
    """The bar of the reduced-precision comparisons: a propagation that rounds
    each density from a value perturbed by a relative amount up to eps (and
    normalises by its own rounded sum) stays within F = rounding_l1_bound of
    the oracle's same-precision column, for random perturbations and for the
    adversarial one that pushes every cell to the side where its rounding
    changes most; the adversarial one reaches a good part of F, so the bound
    is not vacuous. Densities, windows and the histogram are written out here
    in numpy from their definitions (eq. gaussh, eq. (5))."""
    n, lo, hi = (30, 26), (-3.0, -3.0), (3.0, 3.0)
    wl = workloads.random_workload("flip", n, lo, hi, "sincos2", 20, 9, 2, (0.15, 0.6), seed=44)
    f = orc.eval_grid(n, lo, hi, "sincos2")
    e = orc.uniform_edges(f, wl.B)
    b = orc.bins(f, e).reshape(n)
    eps = 2.0 ** -10
    Pq, _ = orc.propagate(n, lo, hi, b.ravel(), wl.B, wl.mu, wl.sigma, wl.weight,
                          precision=precision)
    F = orc.rounding_l1_bound(n, lo, hi, wl.mu, wl.sigma, wl.weight, precision=precision,
                              eps=eps)
    win, _, _ = orc.windows(n, lo, hi, wl.mu, wl.sigma)
    x = [lo[d] + (np.arange(n[d]) + 0.5) * ((hi[d] - lo[d]) / n[d]) for d in range(2)]
    rb = np.vectorize(orc.round_bf16)
    r8 = np.vectorize(orc.round_e4m3)
    quant = {"bf16": rb, "bf16x2": lambda v: rb(v) + rb(v - rb(v)),
             "fp8e4m3": lambda v: r8(448.0 * v) / 448.0}[precision]
    rng = np.random.default_rng(45)

    def column(k, mode):
        col = np.zeros(wl.B)
        for c in range(wl.C):
            (a0, b0), (a1, b1) = win[k, c]
            t0 = (x[0][a0:b0 + 1] - wl.mu[k, c, 0]) / wl.sigma[k, c, 0]
            t1 = (x[1][a1:b1 + 1] - wl.mu[k, c, 1]) / wl.sigma[k, c, 1]
            w = np.exp(-0.5 * (t0[:, None] ** 2 + t1[None, :] ** 2))
            if mode == "adversarial":
                up, mid, dn = quant(w * (1 + eps)), quant(w), quant(w * (1 - eps))
                q = np.where(np.abs(up - mid) >= np.abs(mid - dn), up, dn)
            else:
                q = quant(w * (1 + eps * rng.uniform(-1, 1, size=w.shape)))
            h = np.bincount(b[a0:b0 + 1, a1:b1 + 1].ravel(), weights=q.ravel(),
                            minlength=wl.B)
            col += wl.weight[k, c] * h / q.sum()
        return col

    reach = 0.0
    for k in range(wl.K):
        for _ in range(3):
            assert np.abs(column(k, "random") - Pq[k]).sum() <= F[k]
        adv = np.abs(column(k, "adversarial") - Pq[k]).sum()
        assert adv <= F[k]
        reach = max(reach, adv / F[k])
    assert reach > 0.2, reach


def test_workload_generators_shapes():
    wl = workloads.grid1024()
    assert wl.mu.shape == (65536, 1, 2) and wl.sigma.min() >= 0.05 and wl.sigma.max() <= 0.5
    assert np.array_equal(wl.sigma[:, 0, 0], wl.sigma[:, 0, 1])
    w3 = workloads.grid128_3d()
    assert w3.mu.shape == (32768, 1, 3) and w3.B == 512
    w5 = workloads.grid48_4d()
    assert w5.mu.shape == (16384, 2, 4) and np.allclose(w5.weight.sum(axis=1), 1.0)
    w1 = workloads.grid64()
    # subgrid midpoints: 16 per axis, spacing 6/16
    assert np.allclose(np.unique(w1.mu[:, 0, 0]), -3 + (np.arange(16) + 0.5) * 0.375)


def test_oracle_clean_under_address_and_ub_sanitizers():
    """The oracle's C code, with a harness calling every exported function on
    1- to 4-D grids, mixtures, every density precision, frozen windows and the
    degenerate inputs it defines outputs for, built under AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only): any out-of-bounds access, use
    after free, leak or undefined arithmetic fails the run."""
    import subprocess
    from oracle import build as oracle_build
    exe = oracle_build.build_sanitized()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "san_check ok" in r.stdout, r.stderr[-4000:]



def test_narrow_workload_recipe(orc):
    """The narrow-pdf inputs are what their tests assume: a one-cell window
    along every narrow axis, its centre 14 .. t_max sigma from the mean (the
    factor below FP32's range), and an oracle normaliser inside FP64's."""
    import workloads
    sets = [(0,), (1,), (0, 1)]
    wl = workloads.narrow_workload("narrow2", (40, 30), (-3.0, -3.0), (3.0, 3.0), "sincos2", 24,
                                   90, 301, sets)
    win = orc.windows(wl.n, wl.lo, wl.hi, wl.mu, wl.sigma, 4.0)[0][:, 0]
    h = [(wl.hi[d] - wl.lo[d]) / wl.n[d] for d in range(2)]
    for k in range(wl.K):
        narrow = sets[k % len(sets)]
        tmax = 36.0 if len(narrow) == 1 else 25.0
        for d in narrow:
            assert win[k, d, 0] == win[k, d, 1]
            c = wl.lo[d] + (win[k, d, 0] + 0.5) * h[d]
            t = abs(c - wl.mu[k, 0, d]) / wl.sigma[k, 0, d]
            assert 14.0 - 1e-9 <= t <= tmax + 1e-9
            assert np.exp(-0.5 * t * t) < np.finfo(np.float32).tiny
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model)
    P, Z = orc.propagate(wl.n, wl.lo, wl.hi, orc.bins(f, orc.uniform_edges(f, wl.B)), wl.B,
                         wl.mu, wl.sigma)
    assert (Z > 0).all() and np.isfinite(P).all()
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
