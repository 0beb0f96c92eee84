"""FP64 CPU oracle of the IPSA probability matrix and its field lines -- TEST
INFRASTRUCTURE (same rule as the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it).

Plain numpy, written from Sec. 5.2 (the IPSA probability matrix, eq. IPSA and
the translation y -> Delta y = y - y(l) of each column) and Sec. 5.3 (the
deviations are measured from y(l) = M at the input pdf's maximum). Every
function loops over columns and bins in the order the definition is stated;
nothing is blocked or fused.

Readings (the paper leaves these open):
  * A column of the output matrix is a histogram over the bins [e_b, e_{b+1}).
    Translating it by y_k and re-expressing it on a uniform Delta-y grid
    d_j = d_lo + j*h (j = 0..J) reads each bin's mass as spread evenly over the
    bin: the part of bin b that lands in [d_j, d_{j+1}) is
    P_b * |[e_b - y_k, e_{b+1} - y_k) n [d_j, d_{j+1})| / (e_{b+1} - e_b).
    Mass that lands outside [d_0, d_J) is reported as ``lost``. A column
    holding a non-finite value gives NaN throughout; a non-finite y(l) moves
    the whole column out of range (Q = 0, lost = its mass).
  * Quantiles use the same reading: the CDF is piecewise linear through
    (e_b, C_b), C_b = sum_{b' < b} P_b', and the alpha quantile is the smallest
    y with CDF(y) >= alpha * T, T = C_B (levels are fractions of the column's
    own mass).
  * The "maximum probability of y per l" is reported both as the largest bin
    probability and as the centre of the first bin that attains it.
  * The expected deviation and the binned eq. IPSAvar use bin centres
    c_b = (e_b + e_{b+1})/2 and are not divided by T (as the binned mean of the
    coarse-grained statistics is not).
  * The global marginal over l (Sec. 5.2) weights column k by rho_k as given
    (uniform 1/K when no weights are given).
"""
from __future__ import annotations

import math

import numpy as np


def target_edges(dy_lo: float, dy_width: float, n_dy: int) -> np.ndarray:
    """d_j = d_lo + j*h, j = 0..n_dy, each computed as one FP64 multiply-add."""
    return np.array([dy_lo + j * dy_width for j in range(n_dy + 1)], dtype=np.float64)


def ipsa_matrix(P, edges, y_ref, dy_lo: float, dy_width: float, n_dy: int):
    """IPSA probability matrix (Sec. 5.2, eq. IPSA followed by the per-column
    translation Delta y = y - y(l)): Q[k][j] and lost[k], FP64."""
    P = np.asarray(P, dtype=np.float64)
    e = np.asarray(edges, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    K, B = P.shape
    d = target_edges(dy_lo, dy_width, n_dy)
    Q = np.zeros((K, n_dy))
    lost = np.zeros(K)
    for k in range(K):
        y = y_ref[k]
        if not all(math.isfinite(v) for v in P[k]):
            Q[k, :] = np.nan
            lost[k] = np.nan
            continue
        if not math.isfinite(y):
            lost[k] = P[k].sum()
            continue
        for b in range(B):
            p = P[k, b]
            if p == 0.0:
                continue
            lo = e[b] - y
            hi = e[b + 1] - y
            w = e[b + 1] - e[b]
            kept = 0.0
            # every target cell the translated bin can touch (a superset: the
            # overlap test below decides)
            j0 = max(0, int(math.floor((lo - dy_lo) / dy_width)) - 1)
            j1 = min(n_dy - 1, int(math.floor((hi - dy_lo) / dy_width)) + 1)
            for j in range(j0, j1 + 1):
                a = max(lo, d[j])
                c = min(hi, d[j + 1])
                if c > a:
                    part = p * (c - a) / w
                    Q[k, j] += part
                    kept += part
            lost[k] += p - kept
    return Q, lost


def _cdf(col):
    """C_0 = 0, C_{b+1} = C_b + P_b, summed in bin order in FP64."""
    C = np.zeros(col.size + 1)
    s = 0.0
    for b in range(col.size):
        s += col[b]
        C[b + 1] = s
    return C


def ipsa_fields(P, edges, y_ref=None, levels=()):
    """Coarse-grained field lines of each column (Sec. 5.2: the most probable
    output, confidence intervals, the expected deviation from y(l) and the
    binned local expected squared deviation of eq. IPSAvar).

    Levels lie in (0, 1]. A column holding a non-finite value gives NaN
    everywhere; a column of zeros gives p_max 0, dev and delta2 0, and NaN for
    y_mode and the quantiles.

    Returns dict with y_mode[K], p_max[K], quant[K][len(levels)], and, when
    y_ref is given, dev[K] = sum_b P_b (c_b - y_k) and
    delta2[K] = 1/2 sum_b P_b (c_b - y_k)^2."""
    P = np.asarray(P, dtype=np.float64)
    e = np.asarray(edges, dtype=np.float64)
    K, B = P.shape
    levels = [float(a) for a in levels]
    nan = float("nan")
    y_mode = np.full(K, nan)
    p_max = np.full(K, nan)
    quant = np.full((K, len(levels)), nan)
    dev = np.full(K, nan) if y_ref is not None else None
    delta2 = np.full(K, nan) if y_ref is not None else None
    c = [(e[b] + e[b + 1]) / 2 for b in range(B)]
    for k in range(K):
        col = P[k]
        if not all(math.isfinite(v) for v in col):
            continue
        if y_ref is not None:
            y = float(y_ref[k])
            s1 = 0.0
            s2 = 0.0
            for b in range(B):
                t = c[b] - y
                s1 += col[b] * t
                s2 += col[b] * t * t
            dev[k] = s1
            delta2[k] = 0.5 * s2
        best = 0
        for b in range(1, B):
            if col[b] > col[best]:
                best = b
        p_max[k] = col[best]
        C = _cdf(col)
        T = C[B]
        if not T > 0.0:
            continue
        y_mode[k] = c[best]
        for q, a in enumerate(levels):
            target = a * T
            b = 0
            while C[b + 1] < target:
                b += 1
            frac = (target - C[b]) / col[b]
            frac = min(max(frac, 0.0), 1.0)
            quant[k, q] = e[b] + frac * (e[b + 1] - e[b])
    return dict(y_mode=y_mode, p_max=p_max, quant=quant, dev=dev, delta2=delta2)


def marginalize(A, rho=None):
    """Global marginal over locations (Sec. 5.2): out[j] = sum_k rho_k A[k][j]."""
    A = np.asarray(A, dtype=np.float64)
    K, n = A.shape
    r = np.full(K, 1.0 / K) if rho is None else np.asarray(rho, dtype=np.float64)
    out = np.zeros(n)
    for k in range(K):
        out += r[k] * A[k]
    return out
