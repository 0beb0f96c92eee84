"""Pins of the oracle's inverted model matrix (Bayes inversion, Sec. 3 and the
footnote to its Bayes paragraph) against things other than the oracle itself:
the footnote's identity with dense one-hot matrices, normalisation of every
conditional, Bayes' rule by hand, agreement of its input pdf with the
separately written C oracle's propagation, and closed-form posterior means."""
import math

import numpy as np
import pytest

import oracle
from oracle import inverse


def _case(n, lo, hi, model, B, mu, sigma, weight=None, ns=4.0):
    f = oracle.eval_grid(n, lo, hi, model)
    e = oracle.uniform_edges(f, B)
    b = oracle.bins(f, e)
    win, _, _ = oracle.windows(n, lo, hi, mu, sigma, ns)
    return f, e, b, win


def test_footnote_identity_with_dense_matrices():
    """Minv . M . P_in = P_in on every cell that has a bin (dense one-hot M and
    a dense matrix product for the evidence, not the oracle's propagation)."""
    n, lo, hi = (23, 17), (-2.0, -1.5), (2.0, 1.5)
    rng = np.random.default_rng(3)
    K = 4
    mu = rng.uniform(-1.5, 1.5, (K, 2, 2))
    sg = rng.uniform(0.2, 0.9, (K, 2, 2))
    wt = rng.dirichlet([1.0, 1.0], K)
    f, e, b, win = _case(n, lo, hi, "sincos2", 11, mu, sg)
    N = b.size
    M = np.zeros((11, N))
    M[b[b >= 0], np.nonzero(b >= 0)[0]] = 1.0
    for k in range(K):
        pin = inverse.input_pdf(n, lo, hi, mu[k], sg[k], wt[k], win[k])
        P = M @ pin
        post = inverse.posterior(n, lo, hi, b, P[None, :], mu[k:k + 1], sg[k:k + 1],
                                 wt[k:k + 1], win[k:k + 1], [0])[0]
        Minv = np.zeros((N, 11))
        Minv[np.nonzero(b >= 0)[0], b[b >= 0]] = post[b >= 0]
        back = Minv @ (M @ pin)
        has = b >= 0
        np.testing.assert_allclose(back[has], pin[has], rtol=1e-13, atol=1e-17)


def test_each_conditional_sums_to_one():
    n, lo, hi = (40, 31), (-3.0, -3.0), (3.0, 3.0)
    mu = np.array([[[0.3, -0.4]], [[1.2, 0.9]]])
    sg = np.array([[[0.6, 0.5]], [[0.3, 1.1]]])
    f, e, b, win = _case(n, lo, hi, "timing2", 17, mu, sg)
    P, _ = oracle.propagate(n, lo, hi, b, 17, mu, sg)
    post = inverse.posterior(n, lo, hi, b, P, mu, sg, None, win, [0, 1])
    for t in range(2):
        s = np.bincount(b[b >= 0], weights=post[t, b >= 0], minlength=17)
        np.testing.assert_allclose(s[P[t] > 0], 1.0, rtol=1e-12)
        assert np.all(s[P[t] == 0] == 0.0)


def test_bayes_rule_by_hand():
    """1-D, 4 cells, a flat pdf over all of them (huge sigma, whole-grid
    window), model y = x: bins [0,2) -> cells 0,1 and [2,4] -> cells 2,3, so each
    cell's posterior within its bin is 1/2."""
    n, lo, hi = (4,), (0.0,), (4.0,)
    mu = np.array([[[2.0]]])
    sg = np.array([[[1e6]]])
    f = oracle.eval_grid(n, lo, hi, "linear", (0.0, 1.0))
    e = np.array([0.0, 2.0, 4.0])
    b = oracle.bins(f, e)
    assert list(b) == [0, 0, 1, 1]
    win, _, _ = oracle.windows(n, lo, hi, mu, sg)
    P = np.array([[0.5, 0.5]])
    post = inverse.posterior(n, lo, hi, b, P, mu, sg, None, win, [0])
    np.testing.assert_allclose(post[0], [0.5, 0.5, 0.5, 0.5], rtol=1e-12)
    means = inverse.posterior_means(n, lo, hi, b, post, 2)
    np.testing.assert_allclose(means[0, :, 0], [1.0, 3.0], rtol=1e-12)


def test_input_pdf_matches_the_c_oracle_propagation():
    """Binning this module's input pdf reproduces the C oracle's P (two
    independent implementations of the truncated, normalised Gaussian)."""
    n, lo, hi = (15, 12, 9), (-2.0, -1.0, 0.0), (2.0, 1.5, 2.0)
    rng = np.random.default_rng(9)
    mu = rng.uniform(-0.5, 1.0, (3, 1, 3))
    sg = rng.uniform(0.2, 0.8, (3, 1, 3))
    f, e, b, win = _case(n, lo, hi, "damped3", 13, mu, sg)
    P, _ = oracle.propagate(n, lo, hi, b, 13, mu, sg)
    for k in range(3):
        pin = inverse.input_pdf(n, lo, hi, mu[k], sg[k], None, win[k])
        Pk = np.bincount(b[b >= 0], weights=pin[b >= 0], minlength=13)
        np.testing.assert_allclose(Pk, P[k], rtol=1e-12, atol=1e-16)


def test_posterior_means_of_a_monotone_model():
    """y = x on a 1-D grid: each bin's posterior mean lies inside the x-range
    of its cells, and for a flat pdf it is the mean of those cell centres."""
    n, lo, hi = (60,), (-1.0,), (2.0,)
    f = oracle.eval_grid(n, lo, hi, "linear", (0.0, 1.0))
    e = oracle.uniform_edges(f, 7)
    b = oracle.bins(f, e)
    x = inverse.cell_centres(n, lo, hi)[0]
    for mu0, s0 in ((0.4, 1e6), (0.7, 0.3)):
        mu = np.array([[[mu0]]])
        sg = np.array([[[s0]]])
        win, _, _ = oracle.windows(n, lo, hi, mu, sg)
        P, _ = oracle.propagate(n, lo, hi, b, 7, mu, sg)
        post = inverse.posterior(n, lo, hi, b, P, mu, sg, None, win, [0])
        means = inverse.posterior_means(n, lo, hi, b, post, 7)[0, :, 0]
        for bb in range(7):
            if P[0, bb] <= 0:
                continue
            xb = x[b == bb]
            assert xb.min() - 1e-12 <= means[bb] <= xb.max() + 1e-12
            if s0 > 1e3:
                assert abs(means[bb] - xb.mean()) < 1e-12


def test_degenerate_distributions():
    n, lo, hi = (12, 10), (-1.0, -1.0), (1.0, 1.0)
    mu = np.array([[[0.1, 0.2]], [[9.0, 0.0]], [[0.0, 0.0]]])
    sg = np.array([[[0.3, 0.3]], [[0.2, 0.2]], [[0.0, 0.3]]])
    f, e, b, win = _case(n, lo, hi, "sincos2", 5, mu, sg)
    P, _ = oracle.propagate(n, lo, hi, b, 5, mu, sg)
    post = inverse.posterior(n, lo, hi, b, P, mu, sg, None, win, [0, 1, 2])
    assert np.all(np.isfinite(post[0])) and post[0].max() > 0
    assert np.all(post[1] == 0.0)          # empty window: zero column, no evidence
    assert np.all(np.isnan(post[2]))       # invalid sigma: NaN


def test_mixture_input_pdf_matches_the_c_oracle_propagation():
    n, lo, hi = (21, 18), (-2.0, -2.0), (2.0, 2.0)
    rng = np.random.default_rng(12)
    mu = rng.uniform(-1.0, 1.0, (3, 2, 2))
    sg = rng.uniform(0.2, 0.7, (3, 2, 2))
    wt = np.array([[0.2, 0.8], [0.5, 0.5], [0.9, 0.1]])
    f, e, b, win = _case(n, lo, hi, "sincos2", 9, mu, sg)
    P, _ = oracle.propagate(n, lo, hi, b, 9, mu, sg, wt)
    for k in range(3):
        pin = inverse.input_pdf(n, lo, hi, mu[k], sg[k], wt[k], win[k])
        Pk = np.bincount(b[b >= 0], weights=pin[b >= 0], minlength=9)
        np.testing.assert_allclose(Pk, P[k], rtol=1e-12, atol=1e-16)
