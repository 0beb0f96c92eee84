"""Pins of the oracle's IPSA probability matrix, field lines and marginal
(Sec. 5.2 and Sec. 5.3) against things other than the oracle itself: exact
shifts, closed forms, a different formulation through a library routine
(numpy.interp of the piecewise-linear CDF), the exact per-cell CDF of the
translated statistic, the normal quantile function, the parallel-axis theorem
and the linearity of eq. VUP."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import fields


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# IPSA probability matrix
# ---------------------------------------------------------------------------
def test_matrix_whole_bin_shift_is_a_permutation():
    """y(l) a whole number of bins: translation moves each bin onto one target
    cell, so Q is P shifted by y/h places, exactly."""
    h = 0.25
    B = 16
    e = np.arange(B + 1) * h
    rng = _rng(1)
    P = rng.random((5, B))
    shifts = np.array([0, 3, -2, 7, 12])
    Q, lost = fields.ipsa_matrix(P, e, shifts * h, -(B + 4) * h, h, 2 * B + 8)
    for k, m in enumerate(shifts):
        want = np.zeros(2 * B + 8)
        want[B + 4 - m:2 * B + 4 - m] = P[k]
        assert np.array_equal(Q[k], want)
        assert lost[k] == 0.0


def test_matrix_half_bin_shift_averages_neighbours():
    """y(l) half a bin past a whole shift: each target cell takes half of two
    neighbouring bins."""
    h = 0.5
    B = 12
    e = 1.0 + np.arange(B + 1) * h
    P = _rng(2).random((3, B))
    y = np.array([1.0 + 0.25, 1.0 + 2 * h + 0.25, 1.0 - h + 0.25])
    # translated bin b is [(b-m)h - h/2, (b-m)h + h/2); target cells are
    # [(j-4)h, (j-3)h), so each bin splits evenly over cells b-m+3 and b-m+4
    Q, lost = fields.ipsa_matrix(P, e, y, -4 * h, h, B + 8)
    for k in range(3):
        m = int(round((y[k] - 1.0 - 0.25) / h))   # whole-bin part of the shift
        want = np.zeros(B + 8)
        for b in range(B):
            want[b - m + 3] += 0.5 * P[k, b]
            want[b - m + 4] += 0.5 * P[k, b]
        np.testing.assert_allclose(Q[k], want, rtol=0, atol=1e-15)
        assert abs(lost[k]) < 1e-15


def test_matrix_coarse_target_sums_consecutive_bins():
    """Aligned target cells three bins wide hold the sum of three bins."""
    h = 0.125
    B = 18
    e = np.arange(B + 1) * h
    P = _rng(3).random((2, B))
    Q, lost = fields.ipsa_matrix(P, e, np.zeros(2), 0.0, 3 * h, 6)
    np.testing.assert_allclose(Q, P.reshape(2, 6, 3).sum(axis=2), rtol=1e-15, atol=0)
    assert np.all(np.abs(lost) < 1e-15)


def test_matrix_equals_cdf_difference_on_irregular_edges():
    """Different formulation: Q_j = F(d_{j+1} + y) - F(d_j + y) with F the
    piecewise-linear CDF evaluated by numpy.interp; lost mass = T - sum Q."""
    rng = _rng(4)
    B = 40
    e = np.cumsum(np.concatenate([[-2.0], rng.uniform(0.02, 0.3, size=B)]))
    P = rng.random((6, B)) * (rng.random((6, B)) < 0.8)
    y = rng.uniform(-1.0, 1.0, size=6)
    J = 37
    d = fields.target_edges(-1.7, 0.09, J)
    Q, lost = fields.ipsa_matrix(P, e, y, -1.7, 0.09, J)
    for k in range(6):
        C = np.concatenate([[0.0], np.cumsum(P[k])])
        F = np.interp(d + y[k], e, C)
        np.testing.assert_allclose(Q[k], np.diff(F), rtol=1e-12, atol=1e-14)
        assert abs(lost[k] - (C[-1] - (F[-1] - F[0]))) < 1e-13
        assert abs(Q[k].sum() + lost[k] - P[k].sum()) < 1e-13


def test_matrix_tracks_the_per_cell_distribution_of_delta_y():
    """The quantity the matrix stands for is the distribution of
    S_lin = f_i - y(l) over cells (Sec. 5.2). Built from a weighted cell cloud,
    the cumulative sums of Q differ from the exact per-cell CDF of f - y by at
    most the mass of the bins that hold the two end points (within a bin the
    per-cell CDF lies between the bin's end values)."""
    rng = _rng(5)
    f = rng.normal(0.3, 1.0, size=20000)
    p = rng.random(f.size)
    p /= p.sum()
    B = 30
    e = np.linspace(f.min(), f.max(), B + 1)
    e[-1] = f.max()
    b = oracle.bins(f, e)
    P = np.bincount(b, weights=p, minlength=B)[None, :]
    for y in (-0.4, 0.0, 0.77):
        J = 50
        d = fields.target_edges(-2.5, 0.1, J)
        Q, _ = fields.ipsa_matrix(P, e, [y], -2.5, 0.1, J)
        cumQ = np.concatenate([[0.0], np.cumsum(Q[0])])
        order = np.argsort(f - y)
        fs = (f - y)[order]
        cs = np.concatenate([[0.0], np.cumsum(p[order])])
        G = cs[np.searchsorted(fs, d, side="left")]        # sum p [f - y < d]
        bin_at = np.clip(np.searchsorted(e, d + y, side="right") - 1, 0, B - 1)
        slack = P[0, bin_at] + P[0, bin_at[0]] + 1e-12
        assert np.all(np.abs(cumQ - (G - G[0])) <= slack)


def test_matrix_degenerate_columns():
    e = np.arange(5.0)
    P = np.array([[0.1, 0.2, 0.3, 0.4], [0.1, np.nan, 0.3, 0.4], [0.1, 0.2, 0.3, 0.4]])
    y = np.array([np.inf, 0.0, np.nan])
    Q, lost = fields.ipsa_matrix(P, e, y, -2.0, 0.5, 8)
    assert np.all(Q[0] == 0.0) and abs(lost[0] - 1.0) < 1e-15
    assert np.all(np.isnan(Q[1])) and math.isnan(lost[1])
    assert np.all(Q[2] == 0.0) and abs(lost[2] - 1.0) < 1e-15


def test_matrix_wrong_direction_would_fail():
    """A shift by +y instead of -y moves mass the other way: pins the sign."""
    h = 1.0
    e = np.arange(5) * h
    P = np.array([[0.0, 1.0, 0.0, 0.0]])
    Q, _ = fields.ipsa_matrix(P, e, [2.0], -4.0, 1.0, 8)
    # bin [1, 2) minus 2 -> [-1, 0): target cell 3 of the grid starting at -4
    assert Q[0, 3] == 1.0 and Q[0].sum() == 1.0


# ---------------------------------------------------------------------------
# field lines
# ---------------------------------------------------------------------------
def test_fields_uniform_column_quantiles_are_linear():
    B = 10
    e = np.linspace(-1.0, 4.0, B + 1)
    P = np.full((1, B), 0.1)
    lv = [0.025, 0.25, 0.5, 0.975, 1.0]
    out = fields.ipsa_fields(P, e, None, lv)
    np.testing.assert_allclose(out["quant"][0], -1.0 + 5.0 * np.array(lv), rtol=0, atol=1e-14)


def test_fields_quantiles_match_library_inverse_cdf():
    """Positive columns: the piecewise-linear CDF is strictly increasing, so the
    quantile is numpy.interp of the inverse."""
    rng = _rng(6)
    B = 33
    e = np.cumsum(np.concatenate([[0.5], rng.uniform(0.05, 0.4, size=B)]))
    P = rng.uniform(0.01, 1.0, size=(4, B))
    lv = [0.05, 0.3, 0.5, 0.95]
    out = fields.ipsa_fields(P, e, None, lv)
    for k in range(4):
        C = np.concatenate([[0.0], np.cumsum(P[k])])
        want = np.interp(np.array(lv) * C[-1], C, e)
        np.testing.assert_allclose(out["quant"][k], want, rtol=0, atol=1e-13)


def test_fields_quantiles_skip_empty_bins():
    """Smallest y reaching the level: a gap of empty bins is jumped over."""
    e = np.arange(7.0)
    P = np.array([[0.5, 0.0, 0.0, 0.0, 0.5, 0.0]])
    out = fields.ipsa_fields(P, e, None, [0.5, 0.75])
    # level 0.5 is reached at the right end of bin 0; 0.75 half-way through bin 4
    assert out["quant"][0, 0] == 1.0
    assert out["quant"][0, 1] == 4.5


def test_fields_gaussian_column_quantiles():
    """A finely binned normal: the quantiles approach the normal quantile
    function within a bin width."""
    mu, sd = 0.7, 0.4
    B = 2000
    e = np.linspace(mu - 6 * sd, mu + 6 * sd, B + 1)
    P = np.diff(stats.norm.cdf(e, mu, sd))[None, :]
    lv = [0.025, 0.16, 0.5, 0.84, 0.975]
    out = fields.ipsa_fields(P, e, None, lv)
    want = stats.norm.ppf(np.array(lv), mu, sd)
    assert np.all(np.abs(out["quant"][0] - want) < (e[1] - e[0]))
    assert abs(out["y_mode"][0] - mu) <= (e[1] - e[0])


def test_fields_mode_first_maximum_and_hand_values():
    e = np.array([0.0, 1.0, 2.0, 3.0])
    P = np.array([[0.25, 0.75, 0.0],
                  [0.4, 0.2, 0.4]])
    out = fields.ipsa_fields(P, e, np.array([0.0, 1.0]), [0.5])
    assert out["y_mode"][0] == 1.5 and out["p_max"][0] == 0.75
    assert out["y_mode"][1] == 0.5 and out["p_max"][1] == 0.4   # tie -> first bin
    # column 0 by hand: dev = .25*.5 + .75*1.5 ; delta2 = (.25*.25 + .75*2.25)/2
    assert out["dev"][0] == 1.25
    assert out["delta2"][0] == 0.875
    # column 1 is symmetric about its y_ref = 1.5 - 0.5: dev = 0.4*-0.5+0.2*0.5+0.4*1.5
    assert abs(out["dev"][1] - 0.5) < 1e-15
    # median of column 0: 0.5 = 0.25 + 0.75 * t on bin 1 -> 1 + 1/3
    assert abs(out["quant"][0, 0] - (1.0 + 1.0 / 3.0)) < 1e-15


def test_fields_delta2_parallel_axis_theorem():
    """For normalised columns, 1/2 sum P (c - y)^2 = 1/2 (Var + (E - y)^2)
    with E, Var the binned moments of the separately written C oracle."""
    rng = _rng(7)
    B = 25
    e = np.sort(rng.uniform(-3, 3, size=B + 1))
    P = rng.random((5, B))
    P /= P.sum(axis=1, keepdims=True)
    y = rng.normal(size=5)
    out = fields.ipsa_fields(P, e, y, [])
    m, v, _ = oracle.ipsa(P, e)
    np.testing.assert_allclose(out["delta2"], 0.5 * (v + (m - y) ** 2), rtol=1e-12)
    np.testing.assert_allclose(out["dev"], m - y, rtol=1e-12, atol=1e-14)


def test_fields_degenerate_columns():
    e = np.arange(5.0)
    P = np.array([[0.0, 0.0, 0.0, 0.0],
                  [0.1, np.nan, 0.2, 0.0]])
    out = fields.ipsa_fields(P, e, np.zeros(2), [0.5])
    assert out["p_max"][0] == 0.0 and math.isnan(out["y_mode"][0])
    assert math.isnan(out["quant"][0, 0])
    assert out["dev"][0] == 0.0 and out["delta2"][0] == 0.0
    for key in ("y_mode", "p_max", "dev", "delta2"):
        assert math.isnan(out[key][1])
    assert math.isnan(out["quant"][1, 0])


# ---------------------------------------------------------------------------
# marginal over locations
# ---------------------------------------------------------------------------
def test_marginal_hand_values():
    A = np.array([[1.0, 2.0, 3.0], [5.0, 7.0, 11.0]])
    np.testing.assert_array_equal(fields.marginalize(A, [0.25, 0.5]), [2.75, 4.0, 6.25])
    np.testing.assert_array_equal(fields.marginalize(A), [3.0, 4.5, 7.0])


def test_marginal_is_the_propagated_mixture():
    """Linearity of eq. VUP: marginalising two propagated columns with weights
    rho equals propagating the two-component mixture with those weights."""
    n, lo, hi = (24, 20), (-2.0, -1.5), (2.0, 1.5)
    f = oracle.eval_grid(n, lo, hi, "sincos2")
    B = 16
    e = oracle.uniform_edges(f, B)
    b = oracle.bins(f, e)
    mu = np.array([[[-0.5, 0.2]], [[0.8, -0.4]]])
    sg = np.array([[[0.4, 0.3]], [[0.25, 0.5]]])
    P, _ = oracle.propagate(n, lo, hi, b, B, mu, sg)
    rho = np.array([0.3, 0.7])
    mix_mu = mu[:, 0, :][None, :, :]
    mix_sg = sg[:, 0, :][None, :, :]
    Pm, _ = oracle.propagate(n, lo, hi, b, B, mix_mu, mix_sg, weight=rho[None, :])
    np.testing.assert_allclose(fields.marginalize(P, rho), Pm[0], rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("seed", [8, 9])
def test_matrix_then_marginal_conserves_mass(seed):
    rng = _rng(seed)
    B = 20
    e = np.linspace(0, 2, B + 1)
    P = rng.random((7, B))
    Q, lost = fields.ipsa_matrix(P, e, rng.uniform(0, 2, 7), -1.0, 0.05, 40)
    rho = rng.random(7)
    g = fields.marginalize(Q, rho)
    assert abs(g.sum() + rho @ lost - rho @ P.sum(axis=1)) < 1e-12
