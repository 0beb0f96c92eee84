"""GPU parity of the Bayes inversion (vup_posterior, Sec. 3 and its footnote)
against the FP64 oracle in oracle/inverse.py.

The GPU gets the oracle's inputs: its P rounded to FP32 and its Z (the
normalisation of each component), on a model matrix built from the oracle's
f and edges; the oracle computes with the same FP32 P values. Bars:
  post   |d| <= 2^-20 |post| + 1e-30: the kernel's density is the FP32
         product of d <= 4 FP32 factors (each within about one FP32 ulp of
         the FP64 value), normalised in FP64 and rounded to FP32 once
  means  |d| <= 2^-20 sum_i |post_i x_i| over the bin, per axis
Full size (grid1024, N = 10^6): selected rows of the GPU's own P and Z are
replaced by the oracle's before the call; on the GPU's own rows the
properties are checked: every bin's posterior sums to 1 (deviations weighted
by P_b within the propagation's L1 bar, 2e-5) and the footnote's identity
post * P[bin] reproduces the density.
"""
import sys

import numpy as np
import pytest
import torch

import workloads
from oracle import inverse as oinv

pytestmark = pytest.mark.gpu

DEV = "cuda"
REL = 2.0 ** -20


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


def _run(vup, orc, wl, ks, label, P_override=None):
    fo = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
    eo = orc.uniform_edges(fo, wl.B)
    bo = orc.bins(fo, eo)
    win, _, _ = orc.windows(wl.n, wl.lo, wl.hi, wl.mu, wl.sigma, wl.n_sigma)
    sub = wl.subset(ks)
    Po, Zo = orc.propagate(wl.n, wl.lo, wl.hi, bo, wl.B, sub.mu, sub.sigma, sub.weight,
                           wl.n_sigma)
    P32 = Po.astype(np.float32)
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    mm = vup.build_model_matrix(g, torch.from_numpy(fo).to(DEV), torch.from_numpy(eo).to(DEV))
    # full-size P/Z tensors with the oracle's rows at the selected distributions
    P = torch.zeros((wl.K, wl.B), dtype=torch.float32, device=DEV)
    Z = torch.ones((wl.K, wl.C), dtype=torch.float64, device=DEV)
    kt = torch.from_numpy(np.asarray(ks, dtype=np.int64)).to(DEV)
    P[kt] = torch.from_numpy(P32).to(DEV)
    Z[kt] = torch.from_numpy(Zo).to(DEV)
    post, mean = vup.posterior(mm, wl.mu, wl.sigma, wl.weight, kt, P, Z, wl.n_sigma)
    torch.cuda.synchronize()
    # oracle on the same FP32 evidence (rows of a K-sized array at ks)
    Pfull = np.zeros((wl.K, wl.B))
    Pfull[ks] = P32.astype(np.float64)
    po = oinv.posterior(wl.n, wl.lo, wl.hi, bo, Pfull, wl.mu, wl.sigma, wl.weight, win, ks)
    pg = _cpu(post).astype(np.float64)
    nan_o = np.isnan(po)
    assert np.array_equal(np.isnan(pg), nan_o), label
    err = np.where(nan_o, 0.0, np.abs(pg - po) - (REL * np.abs(po) + 1e-30))
    _say(f"  {label}: post max excess over bar {err.max():.3e}, "
         f"max |post| {np.nanmax(np.abs(po)) if (~nan_o).any() else 0:.3e}")
    assert err.max() <= 0.0, label
    mo = oinv.posterior_means(wl.n, wl.lo, wl.hi, bo, po, wl.B)
    xs = oinv.cell_centres(wl.n, wl.lo, wl.hi)
    grids = np.meshgrid(*[np.arange(wl.n[d]) for d in range(wl.ndim)], indexing="ij")
    X = [np.abs(xs[d][gg.ravel()]) for d, gg in enumerate(grids)]
    mg = _cpu(mean)
    for t in range(len(ks)):
        if np.isnan(po[t]).any():
            assert np.isnan(mg[t]).all()
            continue
        for d in range(wl.ndim):
            bound = np.zeros(wl.B)
            has = bo >= 0
            np.add.at(bound, bo[has], np.abs(po[t, has]) * X[d][has])
            assert np.all(np.abs(mg[t, :, d] - mo[t, :, d]) <= REL * bound + 1e-15), (label, t, d)
    return mm, post, mean, bo


def test_posterior_grid64(vup, orc):
    wl = workloads.grid64()
    ks = [0, 17, 100, 128, 255]
    _say(f"[posterior grid64] ks={ks}")
    _run(vup, orc, wl, ks, "grid64")


def test_posterior_3d_and_mixtures(vup, orc):
    wl3 = workloads.random_workload("inv3d", (19, 23, 17), (-2.0, -1.0, 0.0), (2.0, 1.5, 2.0),
                                    "damped3", 29, 40, 1, (0.1, 0.6), seed=71)
    _run(vup, orc, wl3, [0, 5, 39], "3-D")
    wl4 = workloads.random_workload("inv4d", (9, 11, 7, 13), (-2.0,) * 4, (2.0,) * 4, "ring4", 31,
                                    20, 2, (0.1, 0.9), seed=72)
    _run(vup, orc, wl4, [3, 11, 19], "4-D mixtures")


def test_posterior_narrow_pdfs(vup, orc):
    """Pdfs far narrower than a cell along some axes (their factors below
    FP32's range): the posterior scales each axis's factors to a largest of
    1 and divides by the normaliser scaled alike."""
    wl = workloads.narrow_workload("inv_narrow", (19, 23, 17), (-2.0, -1.0, 0.0), (2.0, 1.5, 2.0),
                                   "damped3", 29, 24, 304, [(2,), (0, 2), (0, 1, 2)])
    _run(vup, orc, wl, [0, 1, 2, 5, 13], "3-D narrow pdfs")


def test_posterior_edge_cases(vup, orc):
    n, lo, hi = (30, 26), (-3.0, -3.0), (3.0, 3.0)
    mu = np.array([[[0.3, -0.2]], [[9.0, 0.0]], [[0.0, 0.0]], [[2.9, 2.9]]])
    sigma = np.array([[[0.4, 0.3]], [[0.2, 0.2]], [[0.0, 0.5]], [[0.5, 0.25]]])
    wl = workloads.Workload("inv_edge", 2, n, lo, hi, "sincos2", (), 12, mu, sigma, None)
    mm, post, mean, bo = _run(vup, orc, wl, [0, 1, 2, 3, 0], "edge cases (empty, invalid, corner)")
    p = _cpu(post)
    assert np.all(p[1] == 0.0) and np.all(np.isnan(p[2]))
    # an index outside [0, K) gives a NaN row; n_sel = 0 is a no-op
    P = torch.zeros((4, 12), dtype=torch.float32, device=DEV)
    Z = torch.ones((4, 1), dtype=torch.float64, device=DEV)
    bad, _ = vup.posterior(mm, mu, sigma, None, [7, -1], P, Z, want_mean=False)
    assert torch.isnan(bad).all()
    none, m0 = vup.posterior(mm, mu, sigma, None, np.zeros(0, np.int64), P, Z)
    assert none.shape == (0, n[0] * n[1])


def test_posterior_full_size_grid1024(vup, orc):
    """N = 10^6, K = 65 536: oracle parity on planted rows, and the footnote's
    identity and per-bin normalisation on rows of the GPU's own P and Z."""
    wl = workloads.grid1024()
    ks = [7, 40000]
    _say(f"[posterior grid1024] planted rows {ks}")
    mm, _, _, bo = _run(vup, orc, wl, ks, "grid1024 planted rows")
    P, Z = vup.propagate(mm, wl.mu, wl.sigma, None, "fp32", wl.n_sigma)
    own = torch.tensor([3, 1234, 65535], dtype=torch.int64, device=DEV)
    post, _ = vup.posterior(mm, wl.mu, wl.sigma, None, own, P, Z, wl.n_sigma, want_mean=False)
    torch.cuda.synchronize()
    b = torch.from_numpy(bo.astype(np.int64)).to(DEV)
    has = b >= 0
    for t in range(3):
        k = int(own[t])
        s = torch.zeros(wl.B, dtype=torch.float64, device=DEV)
        s.index_add_(0, b[has], post[t][has].double())
        # each bin's posterior sums to 1 up to the evidence's own error: the
        # deviations, weighted by P_b, are the column's L1 error of P against
        # the exact density sums, bounded like every FP32 propagation (2e-5)
        Pk = P[k].double()
        live = Pk > 0
        dev = ((s[live] - 1.0).abs() * Pk[live]).sum().item()
        _say(f"  k={k}: sum_b P_b |sum over bin - 1| = {dev:.3e} over {int(live.sum())} bins")
        assert dev <= 2e-5
        # footnote identity: post * P[bin] is the density, which sums to 1 over the
        # window minus the mass of cells without a bin
        dens = post[t][has].double() * P[k].double()[b[has]]
        assert abs(dens.sum().item() - P[k].double().sum().item()) <= 2e-5


def test_posterior_long_fastest_axis(vup, orc):
    """A fastest axis of 17 000 cells: the fastest-axis factor table no longer
    fits the posterior kernel's 64 KB LDS budget and is evaluated per cell."""
    wl = workloads.random_workload("inv_long", (4, 17000), (-2.0, -3.0), (2.0, 3.0), "sincos2", 23,
                                   12, 1, (0.2, 0.9), seed=73)
    _say("[posterior] long fastest axis")
    _run(vup, orc, wl, [0, 5, 11], "long axis")


def test_timing_study_workload_small_L(vup, orc):
    """The Sec. 4.1 timing workload (N = 10^6, untruncated pdfs over the
    whole grid) at L = 3 against the oracle: the configuration bench.py times
    with L up to 1000."""
    wl = workloads.timing_study(3)
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    fo = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model)
    eo = orc.uniform_edges(fo, wl.B)
    mm = vup.build_model_matrix(g, torch.from_numpy(fo).to(DEV), torch.from_numpy(eo).to(DEV))
    P, _ = vup.propagate(mm, wl.mu, wl.sigma, None, "fp32", wl.n_sigma)
    Po, _ = orc.propagate(wl.n, wl.lo, wl.hi, orc.bins(fo, eo), wl.B, wl.mu, wl.sigma,
                          n_sigma=wl.n_sigma)
    l1 = np.abs(_cpu(P).astype(np.float64) - Po).sum(axis=1).max()
    _say(f"[timing study L=3] max column L1 {l1:.3e}")
    assert l1 <= 2e-5
