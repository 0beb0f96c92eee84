"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle,
element by element on the same seeded inputs.

Bars (per distribution k unless noted):
  bins, windows, model-matrix CSR, edges     bit-exact
  f (FP64 on both sides, libm vs ocml)       <= 8 ulp of max |f|
  P, FP32 density                            L1 column error <= 2e-5, |sum - 1| <= 1e-6
  P, BF16 / BF16x2 / E4M3                    against the same-precision oracle: L1 <= 2e-5
                                             + the column's rounding-flip bound F (see
                                             TOL_ACCUM); against FP64: the oracle's own
                                             rounding error + that bar
  exact-f mean                               <= 1e-6 * (max f - min f)
  exact-f variance                           <= 1e-5 * Var + 1e-9 * range^2
  binned mean / variance                     same as exact-f bars
  binned mean / variance, reduced precision  from the column's L1 bar (_binned_reduced)
  entropy                                    <= 1e-5 nats (FP32);
                                             the kernel alone on the oracle's P:
                                             2^-22 (H + 1) (FP32 logarithm per term)
  gradients (FP32 adjoint vs FP64 analytic)  rtol 2e-3 + atol 1e-5 max|g|
The oracle always computes its own f, edges and bins; when a kernel is tested
in isolation, the GPU is fed the oracle's inputs (never the other way round).
"""
import math
import sys
import zlib

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

DEV = "cuda"


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


def _gpu_pipeline(vup, wl, precision="fp32", moments=True):
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    f = vup.eval_grid(g, wl.model, wl.theta)
    e = vup.uniform_edges(f, wl.B)
    mm = vup.build_model_matrix(g, f, e)
    P, Z = vup.propagate(mm, wl.mu, wl.sigma, wl.weight, precision, wl.n_sigma)
    out = dict(grid=g, f=f, edges=e, mm=mm, P=P, Z=Z)
    if moments:
        out["mean"], out["var"], _ = vup.moments(mm, wl.mu, wl.sigma, wl.weight,
                                                 n_sigma=wl.n_sigma)
    out["mean_hist"], out["var_hist"], out["entropy"] = vup.ipsa(mm, P)
    torch.cuda.synchronize()
    return out


def _cpu(t):
    return t.detach().cpu().numpy()


def _check_P(Pg, Po, tol_l1, label, tol_sum=1e-6):
    Pg = Pg.astype(np.float64)
    l1 = np.abs(Pg - Po).sum(axis=1)
    sums = np.abs(Pg.sum(axis=1) - 1.0)
    _say(f"  {label}: max L1 {l1.max():.3e} (bar {tol_l1:.1e}), max |sum-1| {sums.max():.2e}")
    assert (Pg >= 0).all()
    assert l1.max() <= tol_l1, (label, l1.max())
    assert sums.max() <= tol_sum, (label, sums.max())
    return l1.max()


def _check_moments(mg, vg, mo, vo, rng_f, label, scale=1.0):
    em = np.abs(mg - mo).max()
    ev = np.abs(vg - vo) - (1e-5 * scale * np.abs(vo) + 1e-9 * scale * rng_f ** 2)
    _say(f"  {label}: max |dE| {em:.3e} (bar {1e-6 * scale * rng_f:.1e}), "
         f"max var excess over bar {ev.max():.3e}")
    assert em <= 1e-6 * scale * rng_f, label
    assert (ev <= 0).all(), label


# ---------------------------------------------------------------------------
# model matrix construction
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["grid64", "grid1024", "grid128_3d", "grid48_4d"])
def test_eval_edges_bins_model_matrix(vup, orc, name):
    wl = workloads.CONFIGS[name]()
    _say(f"[eval/bin] {name} n={wl.n} B={wl.B}")
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    fg = vup.eval_grid(g, wl.model, wl.theta)
    fo = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
    err = np.abs(_cpu(fg) - fo).max()
    ulp = np.spacing(np.abs(fo).max())
    _say(f"  f: max |df| = {err:.3e} = {err / ulp:.2f} ulp of max|f|")
    assert err <= 8 * ulp
    # edges and bins from the oracle's f on both sides: bit-exact
    f_in = torch.from_numpy(fo).to(DEV)
    eg = vup.uniform_edges(f_in, wl.B)
    eo = orc.uniform_edges(fo, wl.B)
    assert np.array_equal(_cpu(eg), eo)
    mm = vup.build_model_matrix(g, f_in, torch.from_numpy(eo).to(DEV))
    bo = orc.bins(fo, eo)
    assert np.array_equal(_cpu(mm.bin), bo)
    off, perm = orc.model_matrix(bo, wl.B)
    assert np.array_equal(_cpu(mm.offsets), off)
    assert np.array_equal(_cpu(mm.perm)[:off[-1]], perm)
    cnt = _cpu(mm.counts)
    assert np.array_equal(cnt[:-1], np.diff(off)) and cnt[-1] == (bo < 0).sum()
    assert mm.counters()["outside"] == (bo < 0).sum()
    # end to end: the GPU's own f -> edges -> bins agree with the oracle's
    e2 = vup.uniform_edges(fg, wl.B)
    mm2 = vup.build_model_matrix(g, fg, e2)
    mism = int((_cpu(mm2.bin) != bo).sum())
    _say(f"  end-to-end bin mismatches: {mism}")
    assert mism == 0


def test_bins_outside_nan_and_bad_edges(vup, orc):
    g = vup.make_grid((3, 4), (0.0, 0.0), (1.0, 1.0))
    f = np.array([-1.0, 0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 3.0000000000000004, np.nan, np.inf,
                  2.9999999999999996, 1.0000000000000002])
    e = np.array([0.0, 1.0, 2.0, 3.0])
    mm = vup.build_model_matrix(g, torch.from_numpy(f).to(DEV), torch.from_numpy(e).to(DEV))
    assert np.array_equal(_cpu(mm.bin), orc.bins(f, e))
    c = mm.counters()
    assert c["outside"] == (orc.bins(f, e) < 0).sum() and c["bad_edges"] == 0
    ebad = np.array([0.0, 1.0, 1.0, 3.0])
    mm2 = vup.build_model_matrix(g, torch.from_numpy(f).to(DEV), torch.from_numpy(ebad).to(DEV))
    assert (_cpu(mm2.bin) == -1).all() and mm2.counters()["bad_edges"] == 1


# ---------------------------------------------------------------------------
# windows
# ---------------------------------------------------------------------------
def test_windows_bitexact(vup, orc):
    rng = np.random.default_rng(20)
    for n, lo, hi in [((40, 23, 17), (-1.0, 0.0, -2.5), (1.0, 3.0, 0.5)),
                      ((1024, 1024), (-3.0, -3.0), (3.0, 3.0)),
                      ((48, 48, 48, 48), (-2.0,) * 4, (2.0,) * 4)]:
        K = 2000
        d = len(n)
        mu = rng.uniform(np.array(lo) - 1, np.array(hi) + 1, size=(K, 1, d))
        sigma = rng.uniform(1e-4, 0.8, size=(K, 1, d))
        sigma[::97] = 0.0
        wo, bad, _ = orc.windows(n, lo, hi, mu, sigma)
        wg = _cpu(vup.windows(vup.make_grid(n, lo, hi), mu, sigma))
        wo = wo.copy()
        wo[bad.astype(bool)] = np.array([0, -1])
        assert np.array_equal(wg, wo), n


# ---------------------------------------------------------------------------
# propagation, moments, IPSA: small configuration, every output
# ---------------------------------------------------------------------------
def test_grid64_all_outputs(vup, orc):
    wl = workloads.grid64()
    _say(f"[grid64] K={wl.K}")
    o = orc.run_workload(wl)
    gp = _gpu_pipeline(vup, wl)
    rng_f = o["edges"][-1] - o["edges"][0]
    _check_P(_cpu(gp["P"]), o["P"], 2e-5, "P fp32")
    assert np.allclose(_cpu(gp["Z"]), o["Z"], rtol=2e-6, atol=0)
    _check_moments(_cpu(gp["mean"]), _cpu(gp["var"]), o["mean"], o["var"], rng_f, "exact-f")
    _check_moments(_cpu(gp["mean_hist"]), _cpu(gp["var_hist"]), o["mean_hist"], o["var_hist"],
                   rng_f, "binned")
    dh = np.abs(_cpu(gp["entropy"]) - o["entropy"]).max()
    _say(f"  entropy max err {dh:.2e}")
    assert dh <= 1e-5
    # the IPSA kernel alone, fed the oracle's columns rounded to FP32 and the
    # oracle's edges (through a model matrix built from the oracle's f)
    P32 = o["P"].astype(np.float32)
    mm_o = vup.build_model_matrix(gp["grid"], torch.from_numpy(o["f"]).to(DEV),
                                  torch.from_numpy(o["edges"]).to(DEV))
    mg, vg, hg = vup.ipsa(mm_o, torch.from_numpy(P32).to(DEV))
    m2, v2, h2 = orc.ipsa(P32.astype(np.float64), o["edges"])
    assert np.allclose(_cpu(mg), m2, rtol=0, atol=1e-13)
    assert np.allclose(_cpu(vg), v2, rtol=1e-12, atol=1e-15)
    # each entropy term takes the FP32 base-2 logarithm of the FP32 value
    # (relative error below 2^-22), so |dH| <= 2^-22 (H + 1)
    assert (np.abs(_cpu(hg) - h2) <= 2.0 ** -22 * (np.abs(h2) + 1.0)).all()


RAGGED = [
    ("1d", (1000,), (-2.0,), (3.0,), "linear", (0.3, 1.7), 33, 1, (0.01, 0.9)),
    ("2d", (37, 53), (-3.0, -2.0), (3.0, 2.5), "sincos2", (), 29, 1, (0.05, 1.2)),
    ("2d_mix", (61, 45), (-3.0, -3.0), (3.0, 3.0), "timing2", (), 40, 2, (0.05, 0.8)),
    ("3d", (20, 17, 23), (-2.0, -1.0, 0.0), (2.0, 1.5, 2.0), "damped3", (), 17, 1, (0.05, 0.7)),
    ("4d_mix", (9, 11, 7, 13), (-2.0,) * 4, (2.0,) * 4, "ring4", (), 50, 2, (0.1, 0.9)),
    ("2d_wide", (300, 7), (-1.0, -1.0), (1.0, 1.0), "linear", (0.0, 1.0, 0.1), 64, 1, (0.2, 3.0)),
]


@pytest.mark.parametrize("case", RAGGED, ids=[c[0] for c in RAGGED])
@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x2", "fp8e4m3"])
def test_ragged_shapes(vup, orc, case, precision):
    name, n, lo, hi, model, theta, B, C, sr = case
    wl = workloads.random_workload(name, n, lo, hi, model, B, 150, C, sr, seed=zlib.crc32(name.encode()) % 100000,
                                   theta=theta)
    _say(f"[ragged {name} {precision}] n={n} B={B} C={C}")
    o = orc.run_workload(wl, precision="fp64" if precision == "fp32" else precision,
                         with_moments=(precision == "fp32"))
    gp = _gpu_pipeline(vup, wl, precision, moments=(precision == "fp32"))
    rng_f = o["edges"][-1] - o["edges"][0]
    if precision == "fp32":
        _check_P(_cpu(gp["P"]), o["P"], 2e-5, "P fp32")
        _check_moments(_cpu(gp["mean"]), _cpu(gp["var"]), o["mean"], o["var"], rng_f, "exact-f")
        _check_moments(_cpu(gp["mean_hist"]), _cpu(gp["var_hist"]), o["mean_hist"],
                       o["var_hist"], rng_f, "binned")
    else:
        # against the oracle's same-precision result (bars at TOL_ACCUM)
        P64, _ = orc.propagate(wl.n, wl.lo, wl.hi, o["bin"], wl.B, wl.mu, wl.sigma, wl.weight)
        F = orc.rounding_l1_bound(wl.n, wl.lo, wl.hi, wl.mu, wl.sigma, wl.weight, wl.n_sigma,
                                  precision, EPS_DENSITY)
        Pg = _cpu(gp["P"])
        bar = _check_reduced(Pg, o["P"], P64, F, f"P {precision}")
        _binned_reduced(_cpu(gp["mean_hist"]), _cpu(gp["var_hist"]), o["mean_hist"],
                        o["var_hist"], o["P"], Pg, bar, o["edges"], f"binned {precision}")


def test_edge_cases(vup, orc):
    n, lo, hi = (40, 30), (-3.0, -3.0), (3.0, 3.0)
    h = (6.0 / 40, 6.0 / 30)
    mu = np.array([
        [[0.3, -0.2]],                                   # ordinary
        [[9.0, 0.0]],                                    # more than 4 sigma outside: empty
        [[0.0, 0.0]],                                    # sigma = 0: invalid
        [[lo[0] + 7.5 * h[0], lo[1] + 11.5 * h[1]]],     # delta input at a cell centre
        [[0.0, 0.0]],                                    # covers the whole grid
        [[-2.99, 2.99]],                                 # corner, window clipped
    ])
    sigma = np.array([[[0.4, 0.3]], [[0.2, 0.2]], [[0.0, 0.5]], [[1e-6 * h[0], 1e-6 * h[1]]],
                      [[1e6, 1e6]], [[0.5, 0.25]]])
    wl = workloads.Workload("edge", 2, n, lo, hi, "sincos2", (), 12, mu, sigma, None)
    o = orc.run_workload(wl)
    gp = _gpu_pipeline(vup, wl)
    Pg = _cpu(gp["P"])
    ok = [0, 3, 4, 5]
    assert np.abs(Pg[ok] - o["P"][ok]).sum(axis=1).max() <= 2e-5
    assert (Pg[1] == 0).all() and np.isnan(Pg[2]).all()
    assert np.isnan(_cpu(gp["mean"])[[1, 2]]).all()
    onehot = np.zeros(12)
    onehot[o["bin"][7 * 30 + 11]] = 1.0
    assert np.array_equal(Pg[3].astype(np.float64), onehot)
    assert _cpu(gp["var"])[3] == 0.0 and _cpu(gp["entropy"])[3] == 0.0
    c = gp["mm"].counters()
    assert c["bad_param"] == 1 and c["empty"] == 1
    # K = 0 is a no-op
    P0, _ = vup.propagate(gp["mm"], np.zeros((0, 1, 2)), np.zeros((0, 1, 2)))
    assert P0.shape == (0, 12)


@pytest.mark.parametrize("B", [1, 4096])
def test_bin_count_extremes(vup, orc, B):
    wl = workloads.random_workload(f"B{B}", (70, 66), (-3.0, -3.0), (3.0, 3.0), "sincos2", B,
                                   40, 1, (0.1, 1.0), seed=B)
    o = orc.run_workload(wl)
    gp = _gpu_pipeline(vup, wl)
    _check_P(_cpu(gp["P"]), o["P"], 2e-5, f"P B={B}")


def test_determinism(vup):
    wl = workloads.grid48_4d().subset(np.arange(512))
    a = _gpu_pipeline(vup, wl)
    b = _gpu_pipeline(vup, wl)
    for key in ("P", "Z", "mean", "var", "var_hist", "entropy"):
        assert torch.equal(a[key], b[key]), key


# ---------------------------------------------------------------------------
# full-size configurations: every column against the oracle
# ---------------------------------------------------------------------------
# Reduced-precision bars. The oracle's reduced-precision variant rounds every
# density with the same rule as the kernel (RNE to BF16, the BF16 hi + lo
# pair, or E4M3 of 448 w) and normalises by the sum of the same rounded
# values. The kernel rounds an FP32 density built from per-axis factors that
# are each the FP64 exponential rounded once to FP32 (0.5 ulp): the row factor
# is their product over the slower axes taken in FP64 and rounded once, then
# multiplied by the fastest axis' factor in FP32 (and by 448 for E4M3), so the
# value rounded is within (d - 1)/2 + 1/2 + 1/2 + 1/2 + 1/2 <= 3.5 ulps
# (2.1e-7) of the exact density for d <= 4; EPS_DENSITY = 2^-21 (4.8e-7)
# leaves a factor of two. A cell can therefore round differently only if its
# exact density lies within EPS_DENSITY of a rounding midpoint;
# orc.rounding_l1_bound sums, per column, how far such cells can move the
# normalised column (pinned on the CPU against random and adversarial
# perturbations). The bar against the same-precision oracle is that bound
# plus the FP32 bar of the accumulation, 2e-5; against FP64, additionally the
# oracle's own rounding error of the column (itself pinned against the
# worst-case bound 2u).
TOL_ACCUM = 2e-5
EPS_DENSITY = 2.0 ** -21


def _binned_reduced(mg, vg, mq, vq, Pq, Pg, bar_l1, e, label):
    """binned mean and variance at a reduced precision against the oracle of
    the same precision. With both columns of unit mass, a column L1 distance
    L moves the mean by at most L S / 2 and the variance by at most 3 L S^2 / 4,
    S being the width of the bin centres the two columns occupy (shift the
    centres to the middle of that span: |c - s| <= S/2 and |E - s| <= S/2)."""
    c = 0.5 * (e[:-1] + e[1:])
    occ = (Pq > 0) | (Pg > 0)
    S = np.array([c[o].max() - c[o].min() if o.any() else 0.0 for o in occ])
    em = np.abs(mg - mq) - (0.5 * bar_l1 * S + 1e-12)
    ev = np.abs(vg - vq) - (0.75 * bar_l1 * S ** 2 + 1e-12)
    _say(f"  {label}: max |dE| {np.abs(mg - mq).max():.3e}, max |dVar| "
         f"{np.abs(vg - vq).max():.3e}; worst excess over bar {em.max():.2e} / {ev.max():.2e}")
    assert (em <= 0).all() and (ev <= 0).all(), label


def _check_reduced(Pg, Pq, P64, F, label):
    """P at a reduced precision: per column L1 <= F + 2e-5 against the same-
    precision oracle, <= own + F + 2e-5 against FP64; returns the bar."""
    Pg = Pg.astype(np.float64)
    bar = TOL_ACCUM + F
    l1 = np.abs(Pg - Pq).sum(axis=1)
    own = np.abs(Pq - P64).sum(axis=1)
    l64 = np.abs(Pg - P64).sum(axis=1)
    sums = np.abs(Pg.sum(axis=1) - 1.0)
    _say(f"  {label} vs same-precision oracle: max L1 {l1.max():.3e}, max L1 - bar "
         f"{(l1 - bar).max():.2e}, max rounding bound F {F.max():.2e} (nonzero in "
         f"{(F > 0).mean():.1%} of columns); vs FP64: max L1 {l64.max():.3e} (oracle's own "
         f"{own.max():.3e}); max |sum-1| {sums.max():.2e}")
    assert (Pg >= 0).all()
    assert (l1 <= bar).all(), label
    assert (l64 <= own + bar).all(), label
    assert sums.max() <= 1e-6, label
    return bar


def _binned_bars(mg, vg, hg, mo, vo, ho, rng_f, label):
    """binned mean, variance and entropy from the kernel's P against the
    oracle's, with the FP32 bars (mean 1e-6 range, variance 1e-5 Var +
    1e-9 range^2, entropy 1e-5 nats)."""
    _check_moments(mg, vg, mo, vo, rng_f, label)
    eh = np.abs(hg - ho).max()
    _say(f"  {label} entropy: max |dH| {eh:.3e} (bar 1e-5)")
    assert eh <= 1e-5, label


def _full_size(vup, orc, wl, precision, moments=True):
    """Every column of the configuration against the oracle (the oracle runs
    all K distributions, multi-threaded): P, the binned IPSA quantities and,
    at FP32, the exact-f moments."""
    _say(f"[{wl.name} {precision}] K={wl.K}, all columns")
    gp = _gpu_pipeline(vup, wl, precision, moments=moments)
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
    e = orc.uniform_edges(f, wl.B)
    b = orc.bins(f, e)
    rng_f = e[-1] - e[0]
    Pg = _cpu(gp["P"])
    P64, _ = orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, wl.mu, wl.sigma, wl.weight)
    mh, vh, hh = orc.ipsa(P64, e)
    if precision == "fp32":
        l1 = _check_P(Pg, P64, 2e-5, f"P {precision}")
        _binned_bars(_cpu(gp["mean_hist"]), _cpu(gp["var_hist"]), _cpu(gp["entropy"]), mh, vh,
                     hh, rng_f, "binned")
    else:
        Pq, _ = orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, wl.mu, wl.sigma, wl.weight,
                              precision=precision)
        F = orc.rounding_l1_bound(wl.n, wl.lo, wl.hi, wl.mu, wl.sigma, wl.weight, wl.n_sigma,
                                  precision, EPS_DENSITY)
        bar = _check_reduced(Pg, Pq, P64, F, f"P {precision}")
        l1 = np.abs(Pg.astype(np.float64) - P64).sum(axis=1).max()
        mq, vq, hq = orc.ipsa(Pq, e)
        mg, vg, hg = _cpu(gp["mean_hist"]), _cpu(gp["var_hist"]), _cpu(gp["entropy"])
        _binned_reduced(mg, vg, mq, vq, Pq, Pg, bar, e, f"binned {precision}")
        _say(f"  binned {precision} vs FP64: max |dE| {np.abs(mg - mh).max():.3e}, "
             f"max |dVar|/Var {(np.abs(vg - vh) / vh).max():.3e}, "
             f"max |dH| {np.abs(hg - hh).max():.3e}")
    if moments:
        mo, vo, _ = orc.moments(wl.n, wl.lo, wl.hi, f, wl.mu, wl.sigma, wl.weight)
        _check_moments(_cpu(gp["mean"]), _cpu(gp["var"]), mo, vo, rng_f, "exact-f")
    return gp, l1


def test_grid1024_fp32_all_columns(vup, orc):
    _full_size(vup, orc, workloads.grid1024(), "fp32")


@pytest.mark.parametrize("precision", ["bf16", "bf16x2", "fp8e4m3"])
def test_grid1024_reduced_precision_all_columns(vup, orc, precision):
    _full_size(vup, orc, workloads.grid1024(), precision, moments=False)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x2"])
def test_grid128_3d_all_columns(vup, orc, precision):
    _full_size(vup, orc, workloads.grid128_3d(), precision, moments=(precision == "fp32"))


@pytest.mark.parametrize("precision", ["fp32", "fp8e4m3"])
def test_grid48_4d_all_columns(vup, orc, precision):
    _full_size(vup, orc, workloads.grid48_4d(), precision, moments=(precision == "fp32"))


# ---------------------------------------------------------------------------
# exact-f moments (eq. UP) on 2-D grids: the matrix-core tiles
# (vup_moments_tiled) and the per-pdf kernel (vup_moments), each against the
# oracle with the exact-f bars
# ---------------------------------------------------------------------------
# name, n, lo, hi, model, theta, K, sigma range, n_sigma: a grid inside one
# ragged tile, tile edges at 64 and 128 cells with windows of 1 to ~400
# cells, windows wider than the grid, and the n_sigma = 8 truncation
TILED_CASES = [
    ("one_tile", (40, 30), (-3.0, -3.0), (3.0, 3.0), "sincos2", (), 200, (0.01, 2.0), 4.0),
    ("ragged", (200, 130), (-3.0, -2.0), (3.0, 2.5), "sincos2", (), 300, (0.005, 1.5), 4.0),
    ("tile_edges", (65, 129), (-2.0, -2.0), (2.0, 2.0), "timing2", (), 300, (0.002, 0.4), 4.0),
    ("wide", (96, 160), (-1.0, -1.0), (1.0, 1.0), "linear", (0.5, 1.0, -2.0), 150, (0.5, 5.0), 4.0),
    ("ns8", (128, 192), (-5.0, -1.0), (5.0, 5.0), "ipsa2", (), 200, (0.02, 0.6), 8.0),
]


def _tiled_case(case):
    name, n, lo, hi, model, theta, K, sr, ns = case
    wl = workloads.random_workload(name, n, lo, hi, model, 16, K, 1, sr,
                                   seed=zlib.crc32(name.encode()) % 100000, theta=theta)
    wl.n_sigma = ns
    return wl


def _moments_vs_oracle(vup, orc, wl, tiled, f=None, label="", nan_expected=None):
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    if f is None:
        f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
    fin = f[np.isfinite(f)]
    e = orc.uniform_edges(fin, wl.B)
    mm = vup.build_model_matrix(g, torch.from_numpy(f).to(DEV), torch.from_numpy(e).to(DEV))
    mg, vg, _ = vup.moments(mm, wl.mu, wl.sigma, wl.weight, n_sigma=wl.n_sigma, tiled=tiled)
    mo, vo, _ = orc.moments(wl.n, wl.lo, wl.hi, f, wl.mu, wl.sigma, wl.weight, wl.n_sigma)
    mg, vg = _cpu(mg), _cpu(vg)
    nan_o = np.isnan(mo) if nan_expected is None else (np.isnan(mo) | nan_expected)
    assert np.array_equal(np.isnan(mg), nan_o) and np.array_equal(np.isnan(vg), nan_o)
    ok = ~nan_o
    _check_moments(mg[ok], vg[ok], mo[ok], vo[ok], fin.max() - fin.min(),
                   f"exact-f {'tiled' if tiled else 'per-pdf'} {label}")
    return mm, mg, vg


@pytest.mark.parametrize("tiled", [True, False], ids=["tiled", "per_pdf"])
@pytest.mark.parametrize("case", TILED_CASES, ids=[c[0] for c in TILED_CASES])
def test_moments_2d_forms(vup, orc, case, tiled):
    wl = _tiled_case(case)
    _say(f"[moments {case[0]} {'tiled' if tiled else 'per-pdf'}] n={wl.n} K={wl.K}")
    _moments_vs_oracle(vup, orc, wl, tiled)


@pytest.mark.parametrize("tiled", [True, False], ids=["tiled", "per_pdf"])
def test_moments_long_grid(vup, orc, tiled):
    """A 16448 x 6 grid against the oracle. Tiled: 257 tiles along one axis
    (16-bit tile indices) and windows thousands of cells long. Per pdf: the
    six-cell fastest axis is steep, so a strip's anchor value lies far from
    those of the few window cells it meets (the case that needs the shifted
    value formed per cell)."""
    wl = workloads.random_workload("long", (16448, 6), (-4.0, -1.0), (4.0, 1.0), "sincos2", 16,
                                   200, 1, (0.01, 0.5), seed=5)
    _say(f"[moments long grid {'tiled' if tiled else 'per-pdf'}] n={wl.n} K={wl.K}")
    _moments_vs_oracle(vup, orc, wl, tiled)


def test_moments_tiled_hands_over_to_the_per_pdf_kernel(vup):
    """Outside the tiled form (a 2-D mixture here) vup_moments_tiled runs the
    per-pdf kernel of vup_moments: the same bits, and no workspace."""
    wl = workloads.random_workload("mix", (61, 45), (-3.0, -3.0), (3.0, 3.0), "timing2", 16,
                                   100, 2, (0.05, 0.8), seed=9)
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    f = vup.eval_grid(g, wl.model)
    mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, wl.B))
    assert vup.moments_workspace(mm, wl.mu, wl.sigma, wl.weight) is None
    m1, v1, _ = vup.moments(mm, wl.mu, wl.sigma, wl.weight, tiled=True)
    m0, v0, _ = vup.moments(mm, wl.mu, wl.sigma, wl.weight, tiled=False)
    assert torch.equal(m1, m0) and torch.equal(v1, v0)


def test_moments_tiled_many_parts(vup, orc):
    """Enough pdfs on a 2 x 2-tile grid that each tile's list is split in
    parts (part boundaries, partial last batches)."""
    wl = workloads.random_workload("parts", (128, 100), (-2.0, -2.0), (2.0, 2.0), "sincos2", 16,
                                   6000, 1, (0.01, 0.6), seed=77)
    _say(f"[moments parts] n={wl.n} K={wl.K}")
    _moments_vs_oracle(vup, orc, wl, True)


def test_moments_nonfinite_model_values(vup, orc):
    """NaN model values in a 3 x 3 block (one of them at an anchor column of
    the FP32 copy, column 64) and one cell: the tiled form gives NaN exactly
    for the pdfs whose windows hold one (as the oracle's sums do); the per-pdf
    kernel, which sums 8-column strips, for the windows whose rows hold one
    and whose 8-aligned column span meets it. The other pdfs are unaffected."""
    wl = _tiled_case(TILED_CASES[1])
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta).reshape(wl.n)
    f[100:103, 64:67] = np.nan
    f[7, 129] = np.nan
    bad = np.isnan(f)
    f = f.reshape(-1)
    win = orc.windows(wl.n, wl.lo, wl.hi, wl.mu, wl.sigma, wl.n_sigma)[0][:, 0]
    strip_nan = np.array([bad[w[0, 0]:w[0, 1] + 1, (w[1, 0] // 8) * 8:(w[1, 1] // 8) * 8 + 8].any()
                          for w in win])
    _, mt, _ = _moments_vs_oracle(vup, orc, wl, True, f=f, label="NaN cells")
    _, mp, _ = _moments_vs_oracle(vup, orc, wl, False, f=f, label="NaN cells",
                                  nan_expected=strip_nan)
    _say(f"  NaN: tiled {np.isnan(mt).sum()}, per-pdf {np.isnan(mp).sum()} of {wl.K}")
    assert 0 < np.isnan(mt).sum() < np.isnan(mp).sum() < wl.K


def test_moments_tiled_grid1024_all(vup, orc):
    """All 65 536 pdfs of grid1024 through both kernels against the oracle;
    the tiled result is bit-identical over repeated calls (integer
    accumulation), with a fresh and with a reused workspace."""
    wl = workloads.grid1024()
    _say(f"[moments grid1024 both forms] K={wl.K}")
    mm, m1, v1 = _moments_vs_oracle(vup, orc, wl, True)
    ws = vup.moments_workspace(mm, wl.mu, wl.sigma)
    for _ in range(2):
        m2, v2, _ = vup.moments(mm, wl.mu, wl.sigma, workspace=ws)
        assert np.array_equal(_cpu(m2), m1) and np.array_equal(_cpu(v2), v1)
    _, m3, v3 = _moments_vs_oracle(vup, orc, wl, False)
    _say(f"  tiled vs per-pdf: max |dE| {np.abs(m1 - m3).max():.2e}, "
         f"max |dVar|/Var {(np.abs(v1 - v3) / v3).max():.2e}")


def test_moments_tiled_edge_cases(vup, orc):
    """The edge-case pdfs of test_edge_cases through vup_moments_tiled: empty
    and invalid windows NaN, a point mass with variance exactly 0, a window
    over the whole grid, a clipped corner."""
    n, lo, hi = (40, 30), (-3.0, -3.0), (3.0, 3.0)
    h = (6.0 / 40, 6.0 / 30)
    mu = np.array([[[0.3, -0.2]], [[9.0, 0.0]], [[0.0, 0.0]],
                   [[lo[0] + 7.5 * h[0], lo[1] + 11.5 * h[1]]], [[0.0, 0.0]], [[-2.99, 2.99]]])
    sigma = np.array([[[0.4, 0.3]], [[0.2, 0.2]], [[0.0, 0.5]], [[1e-6 * h[0], 1e-6 * h[1]]],
                      [[1e6, 1e6]], [[0.5, 0.25]]])
    wl = workloads.Workload("edge", 2, n, lo, hi, "sincos2", (), 12, mu, sigma, None)
    _, mg, vg = _moments_vs_oracle(vup, orc, wl, True)
    assert np.isnan(mg[[1, 2]]).all() and np.isnan(vg[[1, 2]]).all()
    assert vg[3] == 0.0 and np.isfinite(mg[[0, 3, 4, 5]]).all()


# ---------------------------------------------------------------------------
# pdfs far narrower than a cell (truncation windows of one cell whose centre
# lies 14 to 36 sigma from the mean): each such axis's factor is below FP32's
# range, so the kernels scale every axis's factors to a largest of 1 and put
# the scale back into the reported normalisers in FP64
# ---------------------------------------------------------------------------
NARROW_2D = ("narrow2", (40, 30), (-3.0, -3.0), (3.0, 3.0), "sincos2", 24, 90, 301,
             [(0,), (1,), (0, 1)])
NARROW_3D = ("narrow3", (19, 23, 17), (-2.0, -1.0, 0.0), (2.0, 1.5, 2.0), "damped3", 29, 60, 302,
             [(2,), (0,), (0, 2), (0, 1, 2)])


def _narrow(case):
    name, n, lo, hi, model, B, K, seed, sets = case
    return workloads.narrow_workload(name, n, lo, hi, model, B, K, seed, sets)


@pytest.mark.parametrize("case", [NARROW_2D, NARROW_3D], ids=["2d", "3d"])
def test_narrow_pdfs_propagate(vup, orc, case):
    """Both sweep forms against the oracle: P within the FP32 bar, Z (the mass
    of the truncated densities, down to 1e-266 here) within rtol 2e-6."""
    wl = _narrow(case)
    _say(f"[narrow pdfs propagate] {wl.name} n={wl.n} K={wl.K}")
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model)
    e = orc.uniform_edges(f, wl.B)
    Po, Zo = orc.propagate(wl.n, wl.lo, wl.hi, orc.bins(f, e), wl.B, wl.mu, wl.sigma)
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    mm = vup.build_model_matrix(g, torch.from_numpy(f).to(DEV), torch.from_numpy(e).to(DEV))
    for mode in ("cells", "runs"):
        mm.set_sweep_mode(mode)
        P, Z = vup.propagate(mm, wl.mu, wl.sigma)
        _check_P(_cpu(P), Po, 2e-5, f"{wl.name} {mode} form")
        zg = _cpu(Z)[:, 0]
        _say(f"  Z: max rel err {np.max(np.abs(zg - Zo[:, 0]) / Zo[:, 0]):.2e}, "
             f"min Z {Zo[:, 0].min():.1e}")
        assert np.allclose(zg, Zo[:, 0], rtol=2e-6, atol=0)
    mm.set_sweep_mode("auto")


@pytest.mark.parametrize("case", [NARROW_2D, NARROW_3D], ids=["2d", "3d"])
def test_narrow_pdfs_moments(vup, orc, case):
    """Exact-f moments of the narrow pdfs against the oracle: the per-pdf
    kernel (2-D and 3-D) and the tiled form (2-D)."""
    wl = _narrow(case)
    _say(f"[narrow pdfs moments] {wl.name} n={wl.n} K={wl.K}")
    forms = (True, False) if wl.ndim == 2 else (False,)
    for tiled in forms:
        _moments_vs_oracle(vup, orc, wl, tiled, label="narrow pdfs")


@pytest.mark.parametrize("precision", ["bf16", "bf16x2"])
@pytest.mark.parametrize("case", [NARROW_2D, NARROW_3D], ids=["2d", "3d"])
def test_narrow_pdfs_reduced_precision(vup, orc, case, precision):
    """BF16 and split BF16 round each density. The narrow axes' factors are
    scaled by powers of two, which BF16 rounding (FP32's exponent range, 8
    significant bits) does not see, so P matches the same-precision oracle's
    roundings of the unscaled densities within the usual bar."""
    wl = _narrow(case)
    _say(f"[narrow pdfs {precision}] {wl.name} n={wl.n} K={wl.K}")
    o = orc.run_workload(wl, precision=precision, with_moments=False)
    gp = _gpu_pipeline(vup, wl, precision, moments=False)
    P64, _ = orc.propagate(wl.n, wl.lo, wl.hi, o["bin"], wl.B, wl.mu, wl.sigma, wl.weight)
    F = orc.rounding_l1_bound(wl.n, wl.lo, wl.hi, wl.mu, wl.sigma, wl.weight, wl.n_sigma,
                              precision, EPS_DENSITY)
    _check_reduced(_cpu(gp["P"]), o["P"], P64, F, f"P {precision} narrow")


@pytest.mark.parametrize("form", ["cells", "runs"])
@pytest.mark.parametrize("case", [NARROW_2D, NARROW_3D], ids=["2d", "3d"])
def test_narrow_pdfs_backward(vup, orc, case, form):
    """The adjoint on pdfs far narrower than a cell against the oracle's FP64
    analytic gradient: along a one-cell axis the derivatives are exactly 0
    (the output does not depend on that axis's mean or deviation within the
    window), the other axes' as for any pdf."""
    wl = _narrow(case)
    _say(f"[narrow pdfs backward {form}] {wl.name} n={wl.n} K={wl.K}")
    gm, gs, _ = _grad_case(vup, orc, wl, np.arange(wl.K), 45, form=form)
    win = orc.windows(wl.n, wl.lo, wl.hi, wl.mu, wl.sigma, wl.n_sigma)[0][:, 0]
    one = (win[:, :, 1] == win[:, :, 0])
    assert one.any() and np.all(_cpu(gm)[:, 0, :][one] == 0.0)
    assert np.all(_cpu(gs)[:, 0, :][one] == 0.0)


def test_scaled_multicell_windows(vup, orc):
    """n_sigma = 8 with means 5.5 to 7.5 sigma outside the grid along x: the
    windows hold several cells along x, all 5.5 to 8 sigma from the mean, so
    that axis is scaled (largest factor below 2^-20) while its factors still
    differ from cell to cell. P (both forms), Z and the moments (per pdf and
    tiled) against the oracle."""
    n, lo, hi = (40, 30), (-3.0, -3.0), (3.0, 3.0)
    K = 48
    rng = np.random.Generator(np.random.PCG64(305))
    mu = np.empty((K, 1, 2))
    sg = np.empty((K, 1, 2))
    sg[:, 0, 0] = rng.uniform(0.1, 0.3, K)
    side = np.where(np.arange(K) % 2 == 0, -1.0, 1.0)
    mu[:, 0, 0] = np.where(side < 0, lo[0], hi[0]) + side * rng.uniform(5.5, 7.5, K) * sg[:, 0, 0]
    mu[:, 0, 1] = rng.uniform(-2.5, 2.5, K)
    sg[:, 0, 1] = rng.uniform(0.05, 0.5, K)
    wl = workloads.Workload("scaled8", 2, n, lo, hi, "sincos2", (), 24, mu, sg, None)
    wl.n_sigma = 8.0
    _say(f"[scaled multi-cell windows] n={n} K={K} n_sigma=8")
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model)
    e = orc.uniform_edges(f, wl.B)
    win = orc.windows(wl.n, wl.lo, wl.hi, wl.mu, wl.sigma, 8.0)[0][:, 0]
    assert ((win[:, 0, 1] - win[:, 0, 0]) >= 1).sum() >= K // 2  # several cells along x
    Po, Zo = orc.propagate(wl.n, wl.lo, wl.hi, orc.bins(f, e), wl.B, wl.mu, wl.sigma, None, 8.0)
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    mm = vup.build_model_matrix(g, torch.from_numpy(f).to(DEV), torch.from_numpy(e).to(DEV))
    for mode in ("cells", "runs"):
        mm.set_sweep_mode(mode)
        P, Z = vup.propagate(mm, wl.mu, wl.sigma, None, "fp32", 8.0)
        _check_P(_cpu(P), Po, 2e-5, f"scaled8 {mode} form")
        assert np.allclose(_cpu(Z)[:, 0], Zo[:, 0], rtol=2e-6, atol=0)
    mm.set_sweep_mode("auto")
    for tiled in (True, False):
        _moments_vs_oracle(vup, orc, wl, tiled, label="n_sigma 8, scaled x")


def test_narrow_family_banded(vup, orc):
    """The banded form with locations whose x deviation is far below a cell:
    P and Z against the oracle (the columns of A_x are scaled to a largest
    factor of 1; k_sep_z puts the scale back into Z)."""
    n, lo, hi = (48, 40), (-3.0, -3.0), (3.0, 3.0)
    hx = 6.0 / 48
    centres = workloads.subgrid_midpoints(-3.0, 3.0, 48)
    rng = np.random.Generator(np.random.PCG64(303))
    idx = rng.choice(np.arange(2, 46), size=16, replace=False)
    u = rng.uniform(0.1, 0.45, 16) * np.where(rng.uniform(size=16) < 0.5, -1.0, 1.0)
    mux = centres[idx] + u * hx
    sgx = np.abs(u) * hx / rng.uniform(14.0, 36.0, 16)  # the cell centre 14 .. 36 sigma away
    muy = workloads.subgrid_midpoints(-2.5, 2.5, 16)
    sgy = np.full(16, 0.3)
    Pg, Zg, Po, Zo, mm, mu, sg = _sep_case(vup, orc, n, lo, hi, "sincos2", 32, mux, muy, sgx, sgy,
                                           "narrow x deviations")
    _check_P(Pg, Po, 2e-5, "P separable (narrow) vs oracle")
    assert np.allclose(Zg, Zo, rtol=2e-6, atol=0)


# ---------------------------------------------------------------------------
# eq. (IPSAvar): the local expected squared deviation of vup_moments
# ---------------------------------------------------------------------------
def _check_delta2(vup, orc, wl):
    """delta2 from vup_moments against the oracle's 1/2 sum p (f - M(mu))^2
    (the oracle evaluates M(mu) on the host). delta2 = (Var + (E - M)^2)/2,
    so its bar follows from the moment bars: half the variance bar plus
    |E - M| times the mean bar (and an ulp-level term for M(mu) itself)."""
    _say(f"[delta2 {wl.name}] K={wl.K}")
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
    e = orc.uniform_edges(f, wl.B)
    mm = vup.build_model_matrix(g, torch.from_numpy(f).to(DEV), torch.from_numpy(e).to(DEV))
    mg, vg, dg = vup.moments(mm, wl.mu, wl.sigma, wl.weight, model=wl.model, theta=wl.theta,
                             n_sigma=wl.n_sigma)
    fmu = np.array([orc.model_at(wl.model, wl.mu[k, 0], wl.theta) for k in range(wl.K)])
    mo, vo, do = orc.moments(wl.n, wl.lo, wl.hi, f, wl.mu, wl.sigma, wl.weight, wl.n_sigma,
                             fmu=fmu)
    rng_f = e[-1] - e[0]
    _check_moments(_cpu(mg), _cpu(vg), mo, vo, rng_f, "exact-f")
    dg = _cpu(dg)
    bar = (0.5 * (1e-5 * np.abs(vo) + 1e-9 * rng_f ** 2) + np.abs(mo - fmu) * 1e-6 * rng_f
           + 1e-14 * (1 + np.abs(fmu)) ** 2)
    err = np.abs(dg - do)
    _say(f"  delta2: max |err| {err.max():.3e}, max err/bar {(err / bar).max():.3f}")
    assert (err <= bar).all()
    # the identity the kernel uses, on its own outputs
    assert np.allclose(dg, 0.5 * (_cpu(vg) + (_cpu(mg) - fmu) ** 2), rtol=1e-12, atol=1e-15)


def test_delta2_grid64(vup, orc):
    _check_delta2(vup, orc, workloads.grid64())


def test_delta2_grid1024_all(vup, orc):
    _check_delta2(vup, orc, workloads.grid1024())


@pytest.mark.parametrize("case", [c for c in RAGGED if c[7] == 1], ids=[c[0] for c in RAGGED
                                                                         if c[7] == 1])
def test_delta2_ragged(vup, orc, case):
    name, n, lo, hi, model, theta, B, C, sr = case
    wl = workloads.random_workload(name, n, lo, hi, model, B, 150, C, sr, seed=91, theta=theta)
    _check_delta2(vup, orc, wl)


def test_delta2_rejects_model_of_other_ndim(vup):
    wl = workloads.grid64()
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    f = vup.eval_grid(g, wl.model)
    mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, wl.B))
    with pytest.raises(vup.VupError):
        vup.moments(mm, wl.mu, wl.sigma, model="ring4")


# ---------------------------------------------------------------------------
# backward: adjoint kernel vs FP64 analytic gradient (and the oracle's FD)
# ---------------------------------------------------------------------------
def _grad_case(vup, orc, wl, ks, seed, form=None):
    rng = np.random.default_rng(seed)
    g_var = rng.uniform(0.5, 1.5, size=wl.K)
    g_ent = rng.uniform(0.5, 1.5, size=wl.K)
    gp = _gpu_pipeline(vup, wl, moments=False)
    if form is not None:
        gp["mm"].set_sweep_mode(form)
    gm, gs, gw = vup.ipsa_backward(gp["mm"], wl.mu, wl.sigma, wl.weight, gp["P"],
                                   gp["mean_hist"], torch.from_numpy(g_var).to(DEV),
                                   torch.from_numpy(g_ent).to(DEV))
    sub = wl.subset(ks)
    f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
    e = orc.uniform_edges(f, wl.B)
    b = orc.bins(f, e)
    win, _, _ = orc.windows(wl.n, wl.lo, wl.hi, sub.mu, sub.sigma)
    P, _ = orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, sub.mu, sub.sigma, sub.weight, win=win)
    om, os_, ow = orc.ipsa_grad(wl.n, wl.lo, wl.hi, b, e, sub.mu, sub.sigma, sub.weight, win, P,
                                g_var[ks], g_ent[ks])
    for name, g, o in (("mu", _cpu(gm)[ks], om), ("sigma", _cpu(gs)[ks], os_),
                       ("weight", _cpu(gw)[ks], ow)):
        if name == "weight" and wl.weight is None:
            continue
        scale = np.abs(o).max()
        err = np.abs(g - o) - (2e-3 * np.abs(o) + 1e-5 * scale)
        _say(f"  d/d{name}: max |err| {np.abs(g - o).max():.3e}, scale {scale:.3e}")
        assert (err <= 0).all(), name
    return gm, gs, gw


def test_backward_grid64_all(vup, orc):
    wl = workloads.grid64()
    _say("[backward grid64]")
    _grad_case(vup, orc, wl, np.arange(wl.K), 40)


def test_backward_grid1024_fd_subset(vup, orc):
    """The 64 seeded locations of the finite-difference subset at 1024^2 (the
    oracle's analytic gradient there is pinned against central differences on
    the CPU)."""
    wl = workloads.grid1024()
    _say("[backward grid1024, 64-location subset]")
    ks = workloads.fd_subset(wl.K, 64)
    _grad_case(vup, orc, wl, ks, 41)


def test_backward_mixtures_4d_sampled(vup, orc):
    wl = workloads.grid48_4d()
    _say("[backward grid48_4d mixtures sampled]")
    _grad_case(vup, orc, wl, workloads.sample_indices(wl.K, 256, 42), 42)


def test_backward_ragged(vup, orc):
    for case in RAGGED:
        name, n, lo, hi, model, theta, B, C, sr = case
        wl = workloads.random_workload(name, n, lo, hi, model, B, 40, C, sr, seed=7, theta=theta)
        _say(f"[backward ragged {name}]")
        _grad_case(vup, orc, wl, np.arange(wl.K), 43)


@pytest.mark.parametrize("form", ["cells", "runs"])
def test_backward_both_forms(vup, orc, form):
    # the per-cell adjoint sweep and the run-form one, each against the FP64
    # analytic gradient, on 2-D and 3-D grids with long and short runs
    cases = [workloads.grid64(),
             workloads.random_workload("bwd2d", (57, 300), (-3, -3), (3, 3), "sincos2", 40, 60, 2,
                                       (0.05, 0.9), seed=35),
             workloads.random_workload("bwd3d", (20, 17, 90), (-2, -2, -2), (2, 2, 2), "damped3",
                                       30, 40, 1, (0.1, 0.8), seed=36)]
    for wl in cases:
        _say(f"[backward {form} form: {wl.name}]")
        _grad_case(vup, orc, wl, np.arange(wl.K), 44, form=form)


def test_autograd_function_matches_adjoint(vup):
    wl = workloads.grid64()
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    f = vup.eval_grid(g, wl.model)
    mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, wl.B))
    mu = torch.from_numpy(wl.mu).to(DEV).requires_grad_(True)
    sg = torch.from_numpy(wl.sigma).to(DEV).requires_grad_(True)
    var, ent = vup.IPSA.apply(mu, sg, None, mm)
    (var.sum() + 0.5 * ent.sum()).backward()
    P, _ = vup.propagate(mm, wl.mu, wl.sigma)
    mh, _, _ = vup.ipsa(mm, P)
    gm, gs, _ = vup.ipsa_backward(mm, wl.mu, wl.sigma, None, P, mh,
                                  torch.ones(wl.K, dtype=torch.float64, device=DEV),
                                  torch.full((wl.K,), 0.5, dtype=torch.float64, device=DEV))
    assert torch.equal(mu.grad, gm) and torch.equal(sg.grad, gs)


# ---------------------------------------------------------------------------
# separable (banded MFMA) form for tensor-product families
# ---------------------------------------------------------------------------
def _sep_case(vup, orc, n, lo, hi, model, B, mux, muy, sgx, sgy, label, precision="fp32"):
    _say(f"[separable {label}] n={n} B={B} M=({len(mux)},{len(muy)}) {precision}")
    g = vup.make_grid(n, lo, hi)
    f = vup.eval_grid(g, model)
    mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, B))
    P, Z, _ = vup.propagate_separable(mm, mux, muy, sgx, sgy, precision=precision)
    # the same K = Mx*My distributions through the general path and the oracle
    Mx, My = len(mux), len(muy)
    mu = np.zeros((Mx * My, 1, 2))
    sg = np.zeros((Mx * My, 1, 2))
    mu[:, 0, 0] = np.repeat(mux, My)
    mu[:, 0, 1] = np.tile(muy, Mx)
    sg[:, 0, 0] = np.repeat(sgx, My)
    sg[:, 0, 1] = np.tile(sgy, Mx)
    fo = orc.eval_grid(n, lo, hi, model)
    eo = orc.uniform_edges(fo, B)
    Po, Zo = orc.propagate(n, lo, hi, orc.bins(fo, eo), B, mu, sg)
    torch.cuda.synchronize()
    return _cpu(P), _cpu(Z), Po, Zo[:, 0], mm, mu, sg


def test_separable_grid64(vup, orc):
    wl = workloads.grid64()
    m = workloads.subgrid_midpoints(-3.0, 3.0, 16)
    s = np.full(16, 0.25)
    Pg, Zg, Po, Zo, mm, mu, sg = _sep_case(vup, orc, wl.n, wl.lo, wl.hi, wl.model, wl.B, m, m, s, s,
                                           "grid64")
    _check_P(Pg, Po, 2e-5, "P separable vs oracle")
    assert np.allclose(Zg, Zo, rtol=2e-6, atol=0)
    Pgen, _ = vup.propagate(mm, mu, sg)
    d = np.abs(Pg.astype(np.float64) - _cpu(Pgen)).sum(axis=1).max()
    _say(f"  separable vs general kernel: max L1 {d:.2e}")
    assert d <= 2e-5


SEP_PATHS = [
    # (label, n, Mx, My, B): rows over 4096 cells (T by read-modify-write),
    # rows over 65534 cells (T cell by cell), more than 256 x locations, and a
    # family with fewer than 16 y locations (propagated by the general sweep)
    ("long_rows", (6, 5000), 5, 300, 37),
    ("very_long_rows", (2, 65536), 2, 17, 20),
    ("wide_x", (300, 40), 300, 17, 64),
    ("narrow_y", (70, 90), 40, 5, 33),
]


def test_separable_shared_alpha_axis(vup, orc):
    """A family with one shared alpha factor (M_y = 1), as in the Sec. 5.3
    example (propagated by the general sweep, M_y < 16), against the oracle."""
    n, lo, hi = (200, 150), (-5.0, -1.0), (5.0, 1.0)
    mux = workloads.subgrid_midpoints(-5.0, 5.0, 40)
    for s_l in (0.05, 3.0):
        sgx = np.full(40, s_l)
        Pg, Zg, Po, Zo, mm, mu, sg = _sep_case(vup, orc, n, lo, hi, "ipsa2", 100, mux,
                                               np.array([0.0]), sgx, np.array([0.25]),
                                               f"shared alpha, sigma_l={s_l}")
        _check_P(Pg, Po, 2e-5, f"P separable shared alpha sigma_l={s_l}")
        assert np.allclose(Zg, Zo, rtol=2e-6, atol=0)


@pytest.mark.parametrize("s_l", [0.05, 3.0])
def test_separable_ipsa_example_full_size(vup, orc, s_l):
    """The Sec. 5.3 example at full size (N = 10^6, B = 1000, 1000 locations)
    through vup_propagate_separable with the shared alpha factor (M_y = 1, so
    the general sweep): every row against the oracle."""
    wl = workloads.ipsa_example(s_l)
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    fo = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model)
    eo = orc.uniform_edges(fo, wl.B)
    mm = vup.build_model_matrix(g, torch.from_numpy(fo).to(DEV), torch.from_numpy(eo).to(DEV))
    P, Z, _ = vup.propagate_separable(mm, wl.mu[:, 0, 0], [0.0], wl.sigma[:, 0, 0], [0.25],
                                      wl.n_sigma)
    Po, _ = orc.propagate(wl.n, wl.lo, wl.hi, orc.bins(fo, eo), wl.B, wl.mu, wl.sigma,
                          n_sigma=wl.n_sigma)
    _check_P(_cpu(P), Po, 2e-5, f"P separable Sec. 5.3 example sigma_l={s_l}")


# Bars of the BF16 contractions against the FP64 oracle. Every term a t of
# the contraction is non-negative (a = A_x factor, t = T sum of A_y factors)
# and the terms of a column sum to its mass 1. BF16 keeps 8 significant
# bits, so a and t rounded to nearest even are within 2^-8 of themselves and
# the product within (1 + 2^-8)^2 - 1 = 2^-7 + 2^-16 of a t; the column's L1
# error grows by at most that over the FP32 form's 2e-5 (FP32 operands and
# accumulation). Families with few x cells per window get close to it (a
# column then sums a handful of terms, so little of the rounding cancels:
# 4.8e-3 on 6 x cells). Split BF16: hi + lo is within 2^-16 of each operand
# and the dropped lo*lo term is below 2^-16 a t, so each term is within
# 3 * 2^-16 of a t. The same bounds hold for the column sums (|sum - 1|).
SEP_BARS = {"bf16": 2e-5 + 2.0 ** -7 + 2.0 ** -16, "bf16x2": 2e-5 + 3 * 2.0 ** -16}


@pytest.mark.parametrize("precision", ["bf16", "bf16x2"])
def test_separable_bf16_grid64(vup, orc, precision):
    wl = workloads.grid64()
    m = workloads.subgrid_midpoints(-3.0, 3.0, 16)
    s = np.full(16, 0.25)
    Pg, Zg, Po, Zo, mm, mu, sg = _sep_case(vup, orc, wl.n, wl.lo, wl.hi, wl.model, wl.B, m, m, s, s,
                                           "grid64", precision)
    bar = SEP_BARS[precision]
    _check_P(Pg, Po, bar, f"P separable {precision} vs oracle", tol_sum=bar)
    assert np.allclose(Zg, Zo, rtol=2e-6, atol=0)


@pytest.mark.parametrize("precision", ["bf16", "bf16x2"])
@pytest.mark.parametrize("case", [c for c in SEP_PATHS if c[3] >= 16],
                         ids=[c[0] for c in SEP_PATHS if c[3] >= 16])
def test_separable_bf16_paths(vup, orc, case, precision):
    """The BF16 contractions on rows over 4096 and over 65534 cells and on more
    than 256 x locations (chunks of 32 rows of ix, ragged at both ends)."""
    label, n, Mx, My, B = case
    lo, hi = (-2.0, -3.0), (2.5, 3.0)
    rng = np.random.default_rng(sum(n) + Mx)
    mux = rng.uniform(lo[0], hi[0], Mx)
    muy = rng.uniform(lo[1], hi[1], My)
    sgx = rng.uniform(0.1, 0.8, Mx)
    sgy = rng.uniform(0.01, 0.5, My)
    Pg, Zg, Po, Zo, mm, mu, sg = _sep_case(vup, orc, n, lo, hi, "sincos2", B, mux, muy, sgx, sgy,
                                           label, precision)
    bar = SEP_BARS[precision]
    _check_P(Pg, Po, bar, f"P separable {precision} {label}", tol_sum=bar)
    assert np.allclose(Zg, Zo, rtol=2e-6, atol=0)


@pytest.mark.parametrize("precision", ["bf16", "bf16x2"])
def test_separable_bf16_1024_family_all_rows(vup, orc, precision):
    """The BF16 contractions on the full-size 1024^2 family (256 x 256
    locations, shared sigma = 0.25): every row against the oracle."""
    n, lo, hi, B, M = (1024, 1024), (-3.0, -3.0), (3.0, 3.0), 256, 256
    m = workloads.subgrid_midpoints(lo[0], hi[0], M)
    s = np.full(M, 0.25)
    Pg, Zg, Po, Zo, mm, mu, sg = _sep_case(vup, orc, n, lo, hi, "sincos2", B, m, m, s, s,
                                           "1024^2 family, all rows", precision)
    bar = SEP_BARS[precision]
    _check_P(Pg, Po, bar, f"P separable {precision} 1024^2 family", tol_sum=bar)
    assert np.allclose(Zg, Zo, rtol=2e-6, atol=0)


def test_separable_1024_family_all_rows(vup, orc):
    """The banded form on the full-size tensor-product family: 1024^2 grid on
    [-3,3]^2, sincos model, B = 256, 256 x 256 locations on the midpoint
    subgrid with one shared sigma = 0.25 per axis (U = 6.4e9), every one of
    the 65 536 rows against the oracle, and against the general propagation
    of the same distributions."""
    n, lo, hi, B, M = (1024, 1024), (-3.0, -3.0), (3.0, 3.0), 256, 256
    m = workloads.subgrid_midpoints(lo[0], hi[0], M)
    s = np.full(M, 0.25)
    Pg, Zg, Po, Zo, mm, mu, sg = _sep_case(vup, orc, n, lo, hi, "sincos2", B, m, m, s, s,
                                           "1024^2 family, all rows")
    _check_P(Pg, Po, 2e-5, "P separable 1024^2 family")
    assert np.allclose(Zg, Zo, rtol=2e-6, atol=0)
    Pgen, _ = vup.propagate(mm, mu, sg)
    d = np.abs(Pg.astype(np.float64) - _cpu(Pgen)).sum(axis=1).max()
    _say(f"  separable vs general kernel: max L1 {d:.2e}")
    assert d <= 2e-5


@pytest.mark.parametrize("case", SEP_PATHS, ids=[c[0] for c in SEP_PATHS])
def test_separable_paths(vup, orc, case):
    label, n, Mx, My, B = case
    lo, hi = (-2.0, -3.0), (2.5, 3.0)
    rng = np.random.default_rng(sum(n) + Mx)
    mux = rng.uniform(lo[0], hi[0], Mx)
    muy = rng.uniform(lo[1], hi[1], My)
    sgx = rng.uniform(0.1, 0.8, Mx)
    sgy = rng.uniform(0.01, 0.5, My)
    Pg, Zg, Po, Zo, mm, mu, sg = _sep_case(vup, orc, n, lo, hi, "sincos2", B, mux, muy, sgx, sgy,
                                           label)
    _check_P(Pg, Po, 2e-5, f"P separable {label}")
    assert np.allclose(Zg, Zo, rtol=2e-6, atol=0)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16x2"])
def test_separable_ragged_and_edge_cases(vup, orc, precision):
    rng = np.random.default_rng(50)
    n, lo, hi = (61, 75), (-3.0, -2.0), (3.0, 2.5)
    mux = rng.uniform(-3.2, 3.2, 37)
    muy = rng.uniform(-2.2, 2.7, 21)
    sgx = rng.uniform(0.05, 1.0, 37)
    sgy = rng.uniform(0.05, 1.0, 21)
    mux[3] = 30.0          # empty window on x: whole row block of k is zero
    sgy[5] = 0.0           # invalid: NaN rows
    Pg, Zg, Po, Zo, mm, mu, sg = _sep_case(vup, orc, n, lo, hi, "timing2", 45, mux, muy, sgx,
                                           sgy, "ragged", precision)
    k = np.arange(37 * 21)
    bad = (k % 21) == 5
    empty = (k // 21) == 3
    ok = ~bad & ~empty
    bar = SEP_BARS.get(precision, 2e-5)
    _check_P(Pg[ok], Po[ok], bar, f"P separable ragged {precision}",
             tol_sum=SEP_BARS.get(precision, 1e-6))
    assert np.isnan(Pg[bad]).all() and np.isnan(Zg[bad]).all()
    assert (Pg[empty & ~bad] == 0).all() and (Zg[empty & ~bad] == 0).all()


# ---------------------------------------------------------------------------
# run form of the model matrix and the two accumulation forms
# ---------------------------------------------------------------------------
def _runs_reference(b2, B):
    """runs of equal bin along each row: (first cell, 4*bin or 4*B), terminator."""
    recs, ptr, idx = [], [0], []
    none = 4 * B
    for row in b2:
        code = np.where(row >= 0, 4 * row, none)
        starts = np.nonzero(np.r_[True, code[1:] != code[:-1]])[0]
        for s0 in starts:
            recs.append(int(s0) | (int(code[s0]) << 16))
        recs.append(len(row) | (none << 16))
        ptr.append(len(recs))
        idx.append(np.searchsorted(starts, np.arange(len(row)), side="right") - 1)
    return np.array(recs, dtype=np.int64), np.array(ptr), idx


@pytest.mark.parametrize("n", [(64, 64), (37, 53), (9, 96), (5, 7, 33)])
def test_run_structure_bitexact(vup, orc, n):
    d = len(n)
    lo, hi = (-3.0,) * d, (3.0,) * d
    model = {2: "timing2", 3: "damped3"}[d]
    fo = orc.eval_grid(n, lo, hi, model)
    B = 23
    eo = orc.uniform_edges(fo, B)
    bo = orc.bins(fo, eo)
    g = vup.make_grid(n, lo, hi)
    mm = vup.build_model_matrix(g, torch.from_numpy(fo).to(DEV), torch.from_numpy(eo).to(DEV))
    recs, ptr, idx = _runs_reference(bo.reshape(-1, n[-1]), B)
    got = _cpu(mm.runs).astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(_cpu(mm.rowptr), ptr)
    assert np.array_equal(got[:len(recs)], recs)
    ri = _cpu(mm.runidx).astype(np.int64).reshape(-1, mm.mm.pitch)
    for r, ref in enumerate(idx):
        assert np.array_equal(ri[r, :n[-1]], ref)


def test_run_and_cell_forms_agree(vup, orc):
    for wl in (workloads.grid64(), workloads.grid1024().subset(workloads.sample_indices(65536, 40, 9)),
               workloads.random_workload("runs2d", (57, 300), (-3, -3), (3, 3), "sincos2", 40, 60, 2,
                                         (0.05, 0.9), seed=33),
               workloads.random_workload("runs3d", (20, 17, 90), (-2, -2, -2), (2, 2, 2), "damped3",
                                         30, 40, 1, (0.1, 0.8), seed=34)):
        f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model)
        e = orc.uniform_edges(f, wl.B)
        Po, _ = orc.propagate(wl.n, wl.lo, wl.hi, orc.bins(f, e), wl.B, wl.mu, wl.sigma, wl.weight)
        g = vup.make_grid(wl.n, wl.lo, wl.hi)
        fg = vup.eval_grid(g, wl.model)
        mm = vup.build_model_matrix(g, fg, vup.uniform_edges(fg, wl.B))
        out = {}
        for mode in ("cells", "runs"):
            mm.set_sweep_mode(mode)
            P, Z = vup.propagate(mm, wl.mu, wl.sigma, wl.weight)
            out[mode] = _cpu(P)
            _check_P(out[mode], Po, 2e-5, f"{wl.name} {mode} form")
        mm.set_sweep_mode("auto")
        assert mm.sweep in ("cells", "runs")
        d = np.abs(out["runs"].astype(np.float64) - out["cells"]).sum(axis=1).max()
        _say(f"  runs vs cells: max L1 {d:.2e}; auto resolves to {mm.sweep}")
        # unresolved auto mode: both forms are enqueued and the device picks the
        # same one; results are bit-identical to the resolved form's
        mm_u = vup.build_model_matrix(g, fg, vup.uniform_edges(fg, wl.B), resolve_sweep=False)
        assert mm_u.sweep == "auto"
        Pu, _ = vup.propagate(mm_u, wl.mu, wl.sigma, wl.weight)
        assert np.array_equal(_cpu(Pu), out[mm.sweep])


def test_model_copy_is_anchored(vup):
    """The FP32 model copy inside the model matrix holds, per row, f at every
    eighth column and the FP64 difference f - f(anchor), rounded once, at the
    seven after it; padding columns hold 0 (the layout include/vup.h states).
    A fastest axis of 37 cells makes the last anchor block ragged."""
    g = vup.make_grid((5, 37), (-2.0, -1.0), (2.0, 1.5))
    f = vup.eval_grid(g, "sincos2")
    mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, 16))
    torch.cuda.synchronize()
    rows, pitch = int(mm.mm.rows), int(mm.mm.pitch)
    f32 = mm._view(mm.mm.off_f32, torch.float32, rows * pitch).cpu().numpy().reshape(rows, pitch)
    fh = f.cpu().numpy().reshape(5, 37)
    want = np.zeros((rows, pitch), dtype=np.float32)
    for c in range(37):
        c0 = c - c % 8
        want[:, c] = fh[:, c] if c == c0 else (fh[:, c] - fh[:, c0])
    assert np.array_equal(f32, want)


def test_step_graph_capture(vup):
    """The whole step (model evaluation, edges, model matrix with its sweep
    form set explicitly, propagation, tiled moments, IPSA statistics) captured
    in one HIP graph: nothing in these calls synchronises or records a memset,
    and every replay, with eager steps and synchronisations between replays
    and the outputs cleared before each, reproduces the eager results bit for
    bit (all accumulation is in integers)."""
    wl = workloads.grid64()
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    mu = torch.from_numpy(wl.mu).to(DEV)
    sg = torch.from_numpy(wl.sigma).to(DEV)
    f0 = vup.eval_grid(g, wl.model)
    mm0 = vup.build_model_matrix(g, f0, vup.uniform_edges(f0, wl.B), want_bin=False)
    form = mm0.sweep
    ws = vup.moments_workspace(mm0, mu, sg)
    assert ws is not None

    def step():
        f = vup.eval_grid(g, wl.model)
        e = vup.uniform_edges(f, wl.B)
        mm = vup.build_model_matrix(g, f, e, want_bin=False, resolve_sweep=False)
        mm.set_sweep_mode(form)
        P, _ = vup.propagate(mm, mu, sg, None, "fp32", want_Z=False)
        mean, var, _ = vup.moments(mm, mu, sg, workspace=ws)
        mh, vh, ent = vup.ipsa(mm, P)
        return P, mean, var, mh, vh, ent

    ref = [t.clone() for t in step()]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = step()
    for i in range(3):
        eager = step()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(eager, ref))
        for t in outs:
            t.zero_()
        graph.replay()
        torch.cuda.synchronize()
        _say(f"  replay {i}: " + ", ".join(str(torch.equal(a, b)) for a, b in zip(outs, ref)))
        assert all(torch.equal(a, b) for a, b in zip(outs, ref)), i
