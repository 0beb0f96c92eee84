"""FP64 CPU oracle of the inverted model matrix (Bayes inversion) -- TEST
INFRASTRUCTURE (same rule as the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it).

Sec. 3 (Bayes theorem paragraph and its footnote): with the forward
propagation fixed, the posterior over input cells given that the output fell
in bin b is

    p(x_i | y in b, k) = [bin(i) = b] p_k(x_i) / P[k][b],

the columns of the "inverted model matrix". The footnote's identity says that
applying it after the model matrix gives back the input pdf:
    sum_b Minv[i][b] (M P_in)[b] = P_in[i]     for every cell with a bin.

Readings: a cell without a bin, or whose bin has no mass, gets posterior 0;
an invalid distribution (non-finite evidence) gives NaN. The evidence P is
the caller's propagated matrix (the posterior is relative to that forward
propagation). Per-bin posterior means E[x_d | y in b, k] are sums over the
bin's cells of posterior times cell centre.

Plain numpy: the input pdf is formed cell by cell from its definition
(Gaussian at cell centres, truncated to the per-axis window, normalised per
component, mixed with the weights), independently of the C oracle.
"""
from __future__ import annotations

import math

import numpy as np


def cell_centres(n, lo, hi):
    """x_{d,j} = lo_d + (j + 1/2) (hi_d - lo_d)/n_d (composite midpoint rule, Sec. 3)."""
    return [lo[d] + (np.arange(n[d]) + 0.5) * ((hi[d] - lo[d]) / n[d]) for d in range(len(n))]


def input_pdf(n, lo, hi, mu, sigma, weight, win):
    """p_k(x_i) for one distribution: mu, sigma [C][d], weight [C] or None,
    win [C][d][2] integer windows (empty: hi < lo). Returns FP64 [N]
    (row-major, axis 0 slowest); NaN everywhere if a component is invalid."""
    xs = cell_centres(n, lo, hi)
    D = len(n)
    C = mu.shape[0]
    p = np.zeros(int(np.prod(n)))
    grids = np.meshgrid(*[np.arange(n[d]) for d in range(D)], indexing="ij")
    idx = [g.ravel() for g in grids]
    for c in range(C):
        if any(not (sigma[c, d] > 0) or not math.isfinite(sigma[c, d]) for d in range(D)):
            return np.full(p.size, np.nan)
        keep = np.ones(p.size, dtype=bool)
        s = np.zeros(p.size)
        for d in range(D):
            j = idx[d]
            keep &= (j >= win[c, d, 0]) & (j <= win[c, d, 1])
            t = (xs[d][j] - mu[c, d]) / sigma[c, d]
            s += t * t
        w = np.where(keep, np.exp(-0.5 * s), 0.0)
        Z = w.sum()
        if Z == 0.0:
            continue
        pi = 1.0 if weight is None else float(weight[c])
        p += pi * w / Z
    return p


def posterior(n, lo, hi, bin_, P, mu, sigma, weight, win, ks):
    """Columns of the inverted model matrix for the distributions ``ks``:
    post[t][i] = p_k(x_i) / P[k][bin(i)] (0 without a bin or with P = 0)."""
    bin_ = np.asarray(bin_)
    P = np.asarray(P, dtype=np.float64)
    out = np.zeros((len(ks), bin_.size))
    for t, k in enumerate(ks):
        w = None if weight is None else weight[k]
        p = input_pdf(n, lo, hi, mu[k], sigma[k], w, win[k])
        if not np.all(np.isfinite(P[k])) or not np.all(np.isfinite(p)):
            out[t] = np.nan
            continue
        has = bin_ >= 0
        ev = np.where(has, P[k, np.where(has, bin_, 0)], 0.0)   # evidence of each cell's bin
        ok = has & (ev > 0.0)
        out[t] = np.where(ok, p / np.where(ok, ev, 1.0), 0.0)
    return out


def posterior_means(n, lo, hi, bin_, post, B):
    """E[x_d | y in b] = sum_{i: bin(i) = b} post[i] x_{d,i}: [T][B][d]."""
    xs = cell_centres(n, lo, hi)
    D = len(n)
    grids = np.meshgrid(*[np.arange(n[d]) for d in range(D)], indexing="ij")
    X = [xs[d][g.ravel()] for d, g in enumerate(grids)]
    T = post.shape[0]
    out = np.zeros((T, B, D))
    has = np.asarray(bin_) >= 0
    bsel = np.asarray(bin_)[has]
    for t in range(T):
        for d in range(D):
            np.add.at(out[t, :, d], bsel, post[t, has] * X[d][has])
    return out
