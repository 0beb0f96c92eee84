"""GPU parity of the IPSA probability matrix, field lines, marginal over
locations and point evaluation (Sec. 5.2, Sec. 5.3) against the FP64 oracle.

The GPU is always fed the oracle's inputs (its P rounded to FP32, its edges,
its y(l)); the oracle reads the same FP32 values as FP64. Bars:
  y(l) = M(mu)                <= 8 ulp of max |y| (libm vs ocml)
  Q (IPSA matrix)             |dQ| <= 2^-23 |Q| + 4 B 2^-52 T   (FP64 CDF of B
                              FP32 values differenced, one FP32 rounding)
  lost                        the Q bar's absolute part + (n_dy + 1) 2^-52 T
                              (the oracle sums one kept part per target cell)
  p_max, y_mode               bit-exact (same FP32 values, same first-max rule)
  quantiles                   |dq| <= w_b (4 B 2^-52 T / P_b) + 1e-12 |q|
                              (CDF error moved through the bin's slope)
  dev, delta2                 rtol 1e-12 (FP64 sums of B terms)
  marginal                    rtol 1e-12 + 1e-15 max|out|
Full-size launches (grid1024, K = 65 536, and the Sec. 5.3 example) run on the
GPU's own P with sampled rows overwritten by the oracle's; those rows are
compared, and every column is checked for conservation of mass.
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads
from oracle import fields as ofields

pytestmark = pytest.mark.gpu

DEV = "cuda"
EPS = 2.0 ** -52


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_11246_amd as v
    v.lib()
    return v


def _cpu(t):
    return t.detach().cpu().numpy()


def _mm_from_edges(vup, edges, n=(16, 16)):
    """A model matrix whose only role is to carry `edges` (the column kernels
    read edges and B from it)."""
    g = vup.make_grid(n, (0.0,) * len(n), (1.0,) * len(n))
    B = len(edges) - 1
    f = torch.linspace(float(edges[0]), float(edges[-1]), int(np.prod(n)), dtype=torch.float64,
                       device=DEV)
    return vup.build_model_matrix(g, f, torch.from_numpy(np.asarray(edges, np.float64)).to(DEV))


def _check_matrix(Qg, lg, Qo, lo_, P32, label, e, y, dy_lo, dy_w):
    B = P32.shape[1]
    P = P32.astype(np.float64)
    T = P.sum(axis=1)
    fin = np.isfinite(T)
    Tf = np.where(fin, T, 0.0)
    # CDF rounding (B terms) plus the rounding of the translated positions
    # d_j + y moved through the steepest bin of the column
    R = np.abs(e).max() + np.where(np.isfinite(y), np.abs(y), 0.0) + \
        max(abs(dy_lo), abs(dy_lo + Qo.shape[1] * dy_w))
    slope = np.nan_to_num(P / np.diff(e)[None, :], nan=0.0).max(axis=1) if B else 0.0
    atol = (4 * B * EPS * Tf + 8 * EPS * R * slope)[:, None]
    err = np.abs(Qg.astype(np.float64) - Qo) - (2.0 ** -23 * np.abs(Qo) + atol)
    nan_o = np.isnan(Qo)
    assert np.array_equal(np.isnan(Qg), nan_o), label
    worst = np.where(nan_o, -1.0, err).max() if Qo.size else -1.0
    # the oracle's lost mass is its column sum minus one kept part per target
    # cell, so its own rounding grows with the number of target cells
    el = np.abs(lg - lo_) - (atol[:, 0] + (Qo.shape[1] + 1) * EPS * Tf)
    _say(f"  {label}: Q max excess over bar {worst:.3e}, lost max excess "
         f"{np.nanmax(el) if el.size else 0:.3e}")
    assert worst <= 0.0, label
    assert np.array_equal(np.isnan(lg), np.isnan(lo_)), label
    assert (np.where(np.isnan(lo_), -1.0, el) <= 0.0).all(), label


def _check_fields(out, o, P32, edges, label):
    P = P32.astype(np.float64)
    B = P.shape[1]
    for key in ("p_max", "y_mode"):
        g = _cpu(out[key])
        assert np.array_equal(np.isnan(g), np.isnan(o[key])), (label, key)
        m = ~np.isnan(g)
        assert np.array_equal(g[m], o[key][m]), (label, key)
    if out["quant"] is not None:
        qg = _cpu(out["quant"])
        qo = o["quant"]
        assert np.array_equal(np.isnan(qg), np.isnan(qo)), (label, "quant nan")
        T = P.sum(axis=1)
        worst = -1.0
        for k in range(P.shape[0]):
            for q in range(qo.shape[1]):
                if math.isnan(qo[k, q]):
                    continue
                b = min(max(int(np.searchsorted(edges, qo[k, q], side="right")) - 1, 0), B - 1)
                # the bin the oracle's quantile lies in, or its left neighbour at an edge
                pb = max(P[k, b], P[k, b - 1] if b > 0 else 0.0)
                w = edges[b + 1] - edges[b]
                bar = w * (4 * B * EPS * T[k] / pb) + 1e-12 * abs(qo[k, q])
                worst = max(worst, abs(qg[k, q] - qo[k, q]) - bar)
        _say(f"  {label}: quantile max excess over bar {worst:.3e}")
        assert worst <= 0.0, label
    for key in ("dev", "delta2"):
        if out[key] is None:
            continue
        g = _cpu(out[key])
        assert np.array_equal(np.isnan(g), np.isnan(o[key])), (label, key)
        m = ~np.isnan(g)
        scale = np.abs(o[key][m]).max() if m.any() else 0.0
        np.testing.assert_allclose(g[m], o[key][m], rtol=1e-12, atol=1e-15 * scale,
                                   err_msg=f"{label} {key}")


def _oracle_P32(orc, wl):
    """Oracle pipeline: f, edges, bins, FP64 P rounded to FP32, y(l) = M(mu)."""
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
    e = orc.uniform_edges(f, wl.B)
    b = orc.bins(f, e)
    P, _ = orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, wl.mu, wl.sigma, wl.weight, wl.n_sigma)
    y = np.array([orc.model_at(wl.model, wl.mu[k, 0], wl.theta) for k in range(wl.K)])
    return f, e, P.astype(np.float32), y


# ---------------------------------------------------------------------------
# y(l): the model at points
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("model,ndim", [("sincos2", 2), ("damped3", 3), ("ring4", 4),
                                        ("timing2", 2), ("ipsa2", 2), ("linear", 3)])
def test_eval_points(vup, orc, model, ndim):
    rng = np.random.Generator(np.random.PCG64(31 + ndim))
    theta = (0.5, -1.0, 2.0, 0.25) if model == "linear" else ()
    x = rng.uniform(-3, 3, size=(777, 2, ndim))          # strided view: component 0
    xt = torch.from_numpy(x).to(DEV)
    yg = _cpu(vup.eval_points(model, xt[:, 0, :], theta))
    yo = np.array([orc.model_at(model, x[i, 0], theta) for i in range(x.shape[0])])
    err = np.abs(yg - yo).max()
    ulp = np.spacing(np.abs(yo).max())
    _say(f"[eval_points {model}] max |dy| = {err / ulp:.2f} ulp of max|y|")
    assert err <= 8 * ulp
    assert vup.eval_points(model, xt[:0, 0, :], theta).numel() == 0


# ---------------------------------------------------------------------------
# IPSA matrix and field lines on propagated columns
# ---------------------------------------------------------------------------
GRIDS = [
    # (dy_lo, dy_width as a fraction of the bin width, n_dy)
    ("aligned", None, 1.0, 128),
    ("offset", -0.37, 0.7, 173),
    ("coarse", -1.3, 3.1, 1),
    ("fine_long", -0.9, 0.13, 5001),
]


@pytest.mark.parametrize("grid", GRIDS, ids=[g[0] for g in GRIDS])
def test_matrix_and_fields_grid64(vup, orc, grid):
    wl = workloads.grid64()
    f, e, P32, y = _oracle_P32(orc, wl)
    rng_f = e[-1] - e[0]
    w = rng_f / wl.B
    name, lo_frac, wfrac, n_dy = grid
    dy_lo = -rng_f if lo_frac is None else lo_frac * rng_f
    dy_w = wfrac * w
    _say(f"[matrix grid64 {name}] K={wl.K} B={wl.B} n_dy={n_dy}")
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    mm = vup.build_model_matrix(g, torch.from_numpy(f).to(DEV), torch.from_numpy(e).to(DEV))
    Pt = torch.from_numpy(P32).to(DEV)
    yt = torch.from_numpy(y).to(DEV)
    Qg, lg = vup.ipsa_matrix(mm, Pt, yt, dy_lo, dy_w, n_dy)
    Qo, lo_ = ofields.ipsa_matrix(P32, e, y, dy_lo, dy_w, n_dy)
    _check_matrix(_cpu(Qg), _cpu(lg), Qo, lo_, P32, f"grid64 {name}", e, y, dy_lo, dy_w)
    lv = (0.025, 0.16, 0.5, 0.84, 0.975, 1.0)
    out = vup.ipsa_fields(mm, Pt, yt, lv)
    o = ofields.ipsa_fields(P32, e, y, lv)
    _check_fields(out, o, P32, e, "grid64 fields")


def test_matrix_fields_edge_cases(vup, orc):
    """Zero and NaN columns, infinite / NaN y(l), a one-mass column, irregular
    edges, ragged K."""
    rng = np.random.Generator(np.random.PCG64(77))
    B = 37
    e = np.cumsum(np.concatenate([[-1.0], rng.uniform(0.01, 0.2, size=B)]))
    K = 67
    P32 = (rng.random((K, B)) * (rng.random((K, B)) < 0.6)).astype(np.float32)
    P32[3] = 0.0
    P32[5, 7] = np.nan
    P32[6] = 0.0
    P32[6, 11] = 1.0
    P32[8, :] = 0.25                                      # ties for the mode
    y = rng.uniform(e[0], e[-1], size=K)
    y[9], y[10], y[11] = np.inf, -np.inf, np.nan
    mm = _mm_from_edges(vup, e)
    Pt = torch.from_numpy(P32).to(DEV)
    yt = torch.from_numpy(y).to(DEV)
    for dy_lo, dy_w, n_dy in ((-0.8, 0.05, 47), (0.3, 0.011, 300), (-5.0, 10.0, 1)):
        Qg, lg = vup.ipsa_matrix(mm, Pt, yt, dy_lo, dy_w, n_dy)
        Qo, lo_ = ofields.ipsa_matrix(P32, e, y, dy_lo, dy_w, n_dy)
        _check_matrix(_cpu(Qg), _cpu(lg), Qo, lo_, P32, f"edge n_dy={n_dy}", e, y, dy_lo, dy_w)
    lv = (0.01, 0.5, 0.99)
    yfin = np.where(np.isfinite(y), y, 0.0)
    out = vup.ipsa_fields(mm, Pt, torch.from_numpy(yfin).to(DEV), lv)
    _check_fields(out, ofields.ipsa_fields(P32, e, yfin, lv), P32, e, "edge fields")
    # optional outputs off, no reference values
    out2 = vup.ipsa_fields(mm, Pt, None, ())
    assert out2["dev"] is None and out2["quant"] is None
    assert np.array_equal(_cpu(out2["p_max"]), _cpu(out["p_max"]), equal_nan=True)
    assert np.array_equal(_cpu(out2["y_mode"]), _cpu(out["y_mode"]), equal_nan=True)
    # K = 0 is a no-op
    Q0, l0 = vup.ipsa_matrix(mm, Pt[:0], yt[:0], 0.0, 0.1, 5)
    assert Q0.shape == (0, 5) and l0.shape == (0,)


@pytest.mark.parametrize("B", [1, 64, 300, 2000, 4096])
def test_matrix_fields_bin_count_extremes(vup, orc, B):
    """B = 4096 needs more than 64 KiB of LDS per workgroup (one wave)."""
    rng = np.random.Generator(np.random.PCG64(B))
    e = np.linspace(-2.0, 3.0, B + 1)
    K = 130
    P32 = rng.random((K, B)).astype(np.float32)
    P32 /= P32.sum(axis=1, keepdims=True)
    y = rng.uniform(-2.0, 3.0, size=K)
    mm = _mm_from_edges(vup, e, n=(40, 40))
    Pt = torch.from_numpy(P32).to(DEV)
    yt = torch.from_numpy(y).to(DEV)
    Qg, lg = vup.ipsa_matrix(mm, Pt, yt, -2.5, 5.0 / 700, 700)
    Qo, lo_ = ofields.ipsa_matrix(P32, e, y, -2.5, 5.0 / 700, 700)
    _check_matrix(_cpu(Qg), _cpu(lg), Qo, lo_, P32, f"B={B}", e, y, -2.5, 5.0 / 700)
    lv = (0.05, 0.5, 0.95)
    out = vup.ipsa_fields(mm, Pt, yt, lv)
    _check_fields(out, ofields.ipsa_fields(P32, e, y, lv), P32, e, f"fields B={B}")


# ---------------------------------------------------------------------------
# marginal over locations
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("K,n", [(1, 7), (9, 256), (1000, 1000), (4099, 65), (65536, 256),
                                 (3, 70000)])
def test_marginal(vup, K, n):
    rng = np.random.Generator(np.random.PCG64(K * 7 + n))
    A = rng.random((K, n)).astype(np.float32)
    rho = rng.random(K)
    At = torch.from_numpy(A).to(DEV)
    for r in (rho, None):
        og = _cpu(vup.marginalize(At, None if r is None else torch.from_numpy(r).to(DEV)))
        oo = ofields.marginalize(A, r)
        np.testing.assert_allclose(og, oo, rtol=1e-12, atol=1e-15 * np.abs(oo).max())
    a = vup.marginalize(At, torch.from_numpy(rho).to(DEV))
    b = vup.marginalize(At, torch.from_numpy(rho).to(DEV))
    assert torch.equal(a, b)
    _say(f"[marginal K={K} n={n}] ok, workspace {vup.marginal_workspace_bytes(K, n)} B")


def test_marginal_empty_and_workspace_errors(vup):
    out = vup.marginalize(torch.zeros((0, 5), dtype=torch.float32, device=DEV))
    assert torch.equal(out, torch.zeros(5, dtype=torch.float64, device=DEV))
    A = torch.ones((100, 9), dtype=torch.float32, device=DEV)
    need = vup.marginal_workspace_bytes(100, 9)
    assert need > 0
    small = torch.empty(need - 8, dtype=torch.uint8, device=DEV)
    import ctypes
    lib = vup.lib()
    out = torch.empty(9, dtype=torch.float64, device=DEV)
    rc = lib.vup_marginalize(100, 9, ctypes.c_void_p(A.data_ptr()), None,
                             ctypes.c_void_p(small.data_ptr()), small.numel(),
                             ctypes.c_void_p(out.data_ptr()), None)
    assert rc == -5


# ---------------------------------------------------------------------------
# full-size launches: grid1024 (K = 65 536, B = 256) and the Sec. 5.3 example
# ---------------------------------------------------------------------------
def _full_size(vup, orc, wl, n_dy, nsample, seed):
    _say(f"[full size {wl.name}] K={wl.K} B={wl.B} n_dy={n_dy}")
    # the model matrix is built on the oracle's f and edges (GPU fed oracle inputs)
    fo = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
    eo = orc.uniform_edges(fo, wl.B)
    bo = orc.bins(fo, eo)
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    mm = vup.build_model_matrix(g, torch.from_numpy(fo).to(DEV), torch.from_numpy(eo).to(DEV))
    P, _ = vup.propagate(mm, wl.mu, wl.sigma, wl.weight, "fp32", wl.n_sigma)
    mu = torch.from_numpy(wl.mu).to(DEV)
    y = vup.eval_points(wl.model, mu[:, 0, :], wl.theta)
    # overwrite sampled rows with the oracle's own P (FP32) and y(l)
    ks = workloads.sample_indices(wl.K, nsample, seed)
    sub = wl.subset(ks)
    Po, _ = orc.propagate(wl.n, wl.lo, wl.hi, bo, wl.B, sub.mu, sub.sigma, sub.weight, wl.n_sigma)
    P32 = Po.astype(np.float32)
    P[torch.from_numpy(ks).to(DEV)] = torch.from_numpy(P32).to(DEV)
    yo = np.array([orc.model_at(wl.model, sub.mu[i, 0], wl.theta) for i in range(len(ks))])
    y[torch.from_numpy(ks).to(DEV)] = torch.from_numpy(yo).to(DEV)
    rng_f = eo[-1] - eo[0]
    dy_lo, dy_w = -rng_f, 2 * rng_f / n_dy
    Q, lost = vup.ipsa_matrix(mm, P, y, dy_lo, dy_w, n_dy)
    lv = (0.025, 0.5, 0.975)
    fl = vup.ipsa_fields(mm, P, y, lv)
    g_all = vup.marginalize(Q)
    torch.cuda.synchronize()
    Qo, lo_ = ofields.ipsa_matrix(P32, eo, yo, dy_lo, dy_w, n_dy)
    _check_matrix(_cpu(Q)[ks], _cpu(lost)[ks], Qo, lo_, P32, f"{wl.name} sampled", eo, yo,
                  dy_lo, dy_w)
    o = ofields.ipsa_fields(P32, eo, yo, lv)
    sel = {k: (None if v is None else v[torch.from_numpy(ks).to(DEV)]) for k, v in fl.items()}
    _check_fields(sel, o, P32, eo, f"{wl.name} fields sampled")
    # every column: the translation keeps the mass (Q + lost = column sum)
    Pd = P.double()
    T = Pd.sum(dim=1)
    cons = (Q.double().sum(dim=1) + lost - T).abs().max().item()
    bar = 4 * wl.B * EPS + 2.0 ** -22 + n_dy * EPS
    _say(f"  {wl.name}: max |sum Q + lost - T| over all {wl.K} columns {cons:.3e} (bar {bar:.1e})")
    assert cons <= bar
    gsum = g_all.sum().item() + lost.mean().item()
    assert abs(gsum - T.mean().item()) <= bar


def test_full_size_grid1024(vup, orc):
    _full_size(vup, orc, workloads.grid1024(), 512, 24, 5)


@pytest.mark.parametrize("sigma_l", [0.05, 3.0])
def test_full_size_ipsa_example(vup, orc, sigma_l):
    _full_size(vup, orc, workloads.ipsa_example(sigma_l), 2000, 6, 6)
