"""FP64 CPU oracle for VUP / IPSA (arXiv:1908.11246) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The GPU library never uses it.

Each function is a thin ctypes wrapper over ``vup_oracle.c``; numpy arrays in,
numpy arrays out, everything FP64 (int32 for bins and windows).

Function -> paper passage it follows:
  eval_grid        Alg. VUP "generate a uniform grid", "evaluate the model"
  uniform_edges    bin partition of eq. (4) (uniform bins over [min f, max f])
  bins             indicator Theta of eq. (4), one nonzero per column (eq. MUP)
  model_matrix     sparse model matrix of eq. (5) in compressed-by-bin form
  windows          truncation of the Gaussian input pdf (eq. gaussh, Sec. 5.3)
  propagate        eq. (5) / eq. VUP with normalised input pdfs (Alg. VUP)
  moments          exact-f mean/variance of the propagated output; eq. IPSAvar
  ipsa             coarse-grained per-column variance and entropy (Sec. 5.2)
  ipsa_grad        derivative of those quantities w.r.t. the pdf parameters
  rounding_l1_bound  largest column change that rounding (reduced-precision
                   variants) can make when the value rounded is off by a
                   relative eps (a bar for comparisons at those precisions)

The IPSA probability matrix (Sec. 5.2, eq. IPSA and the per-column
translation), its field lines and the marginal over locations are plain numpy
in ``fields.py``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MODEL_IDS = {"linear": 0, "sincos2": 1, "damped3": 2, "ring4": 3, "timing2": 4, "ipsa2": 5}
PREC_IDS = {"fp64": -1, "fp32": 0, "bf16": 1, "bf16x2": 2, "fp8e4m3": 3}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_long)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    lib.orc_model_at.restype = ctypes.c_double
    lib.orc_model_at.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.orc_eval_grid.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_int, _dp, _dp]
    lib.orc_uniform_edges.argtypes = [_dp, ctypes.c_long, ctypes.c_int, _dp]
    lib.orc_bin.argtypes = [_dp, ctypes.c_long, _dp, ctypes.c_int, _ip]
    lib.orc_model_matrix.argtypes = [_ip, ctypes.c_long, ctypes.c_int, _lp, _lp]
    lib.orc_windows.restype = ctypes.c_long
    lib.orc_windows.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_long, ctypes.c_int,
                                _dp, _dp, ctypes.c_double, _ip, _ip]
    lib.orc_round_bf16.restype = ctypes.c_double
    lib.orc_round_bf16.argtypes = [ctypes.c_double]
    lib.orc_round_e4m3.restype = ctypes.c_double
    lib.orc_round_e4m3.argtypes = [ctypes.c_double]
    lib.orc_propagate.argtypes = [ctypes.c_int, _ip, _dp, _dp, _ip, ctypes.c_int, ctypes.c_long,
                                  ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                  _ip, _dp, _dp, ctypes.c_int]
    lib.orc_moments.argtypes = [ctypes.c_int, _ip, _dp, _dp, _dp, ctypes.c_long, ctypes.c_int,
                                _dp, _dp, _dp, ctypes.c_double, _dp, _dp, _dp, _dp, ctypes.c_int]
    lib.orc_ipsa.argtypes = [_dp, ctypes.c_long, ctypes.c_int, _dp, _dp, _dp, _dp]
    lib.orc_rounding_l1_bound.argtypes = [ctypes.c_int, _ip, _dp, _dp, ctypes.c_long,
                                          ctypes.c_int, _dp, _dp, _dp, ctypes.c_double,
                                          ctypes.c_int, ctypes.c_double, _dp, ctypes.c_int]
    lib.orc_ipsa_grad.argtypes = [ctypes.c_int, _ip, _dp, _dp, _ip, ctypes.c_int, _dp,
                                  ctypes.c_long, ctypes.c_int, _dp, _dp, _dp, _ip, _dp, _dp, _dp,
                                  _dp, _dp, _dp, ctypes.c_int]
    _lib = lib
    return lib


def _d(a):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _p(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _grid_args(n, lo, hi):
    d = len(n)
    n_a = np.ascontiguousarray(n, dtype=np.int32)
    lo_a = np.ascontiguousarray(lo, dtype=np.float64)
    hi_a = np.ascontiguousarray(hi, dtype=np.float64)
    return d, n_a, lo_a, hi_a


def model_at(model: str, x, theta=()) -> float:
    lib = _load()
    x = _d(np.atleast_1d(x))
    th = np.zeros(8)
    th[:len(theta)] = theta
    return lib.orc_model_at(MODEL_IDS[model], len(x), _p(th), _p(x))


def eval_grid(n, lo, hi, model: str, theta=()) -> np.ndarray:
    lib = _load()
    d, n_a, lo_a, hi_a = _grid_args(n, lo, hi)
    th = np.zeros(8)
    th[:len(theta)] = theta
    f = np.empty(int(np.prod(n)), dtype=np.float64)
    lib.orc_eval_grid(d, _p(n_a, _ip), _p(lo_a), _p(hi_a), MODEL_IDS[model], _p(th), _p(f))
    return f


def uniform_edges(f, B: int) -> np.ndarray:
    lib = _load()
    f = _d(f)
    e = np.empty(B + 1, dtype=np.float64)
    lib.orc_uniform_edges(_p(f), f.size, B, _p(e))
    return e


def bins(f, edges) -> np.ndarray:
    lib = _load()
    f = _d(f)
    e = _d(edges)
    out = np.empty(f.size, dtype=np.int32)
    lib.orc_bin(_p(f), f.size, _p(e), e.size - 1, _p(out, _ip))
    return out


def model_matrix(bin_, B: int):
    """(offsets[B+1], perm[nnz]) of the sparse one-hot model matrix, by bin."""
    lib = _load()
    b = np.ascontiguousarray(bin_, dtype=np.int32)
    off = np.empty(B + 1, dtype=np.int64)
    nnz = int((b >= 0).sum())
    perm = np.empty(max(nnz, 1), dtype=np.int64)
    lib.orc_model_matrix(_p(b, _ip), b.size, B, _p(off, _lp), _p(perm, _lp))
    return off, perm[:nnz]


def windows(n, lo, hi, mu, sigma, n_sigma: float = 4.0):
    """Integer windows [K][C][d][2] (empty: lo=0, hi=-1), bad flags [K][C], U."""
    lib = _load()
    d, n_a, lo_a, hi_a = _grid_args(n, lo, hi)
    mu = _d(mu)
    sigma = _d(sigma)
    K, C = mu.shape[0], mu.shape[1]
    win = np.empty((K, C, d, 2), dtype=np.int32)
    bad = np.empty((K, C), dtype=np.int32)
    U = lib.orc_windows(d, _p(n_a, _ip), _p(lo_a), _p(hi_a), K, C, _p(mu), _p(sigma),
                        float(n_sigma), _p(win, _ip), _p(bad, _ip))
    return win, bad, int(U)


def round_bf16(x: float) -> float:
    return _load().orc_round_bf16(float(x))


def round_e4m3(x: float) -> float:
    return _load().orc_round_e4m3(float(x))


def propagate(n, lo, hi, bin_, B, mu, sigma, weight=None, n_sigma=4.0, precision="fp64",
              win=None, nthreads=0):
    """P[K][B] (FP64) and Z[K][C]."""
    lib = _load()
    d, n_a, lo_a, hi_a = _grid_args(n, lo, hi)
    b = np.ascontiguousarray(bin_, dtype=np.int32)
    mu = _d(mu)
    sigma = _d(sigma)
    w = _d(weight)
    K, C = mu.shape[0], mu.shape[1]
    if C > 1 and w is None:
        raise ValueError("mixtures need weights")
    P = np.empty((K, B), dtype=np.float64)
    Z = np.empty((K, C), dtype=np.float64)
    wn = None if win is None else np.ascontiguousarray(win, dtype=np.int32)
    lib.orc_propagate(d, _p(n_a, _ip), _p(lo_a), _p(hi_a), _p(b, _ip), B, K, C, _p(mu),
                      _p(sigma), _p(w), float(n_sigma), PREC_IDS[precision], _p(wn, _ip),
                      _p(P), _p(Z), int(nthreads))
    return P, Z


def rounding_l1_bound(n, lo, hi, mu, sigma, weight=None, n_sigma=4.0, precision="bf16",
                      eps=2.0 ** -19, nthreads=0):
    """F[K]: bound on the column L1 distance between propagate(precision=...)
    and any propagation that rounds each density from a value within relative
    eps of the exact one (and normalises by its own rounded sum)."""
    lib = _load()
    d, n_a, lo_a, hi_a = _grid_args(n, lo, hi)
    mu = _d(mu)
    sigma = _d(sigma)
    w = _d(weight)
    K, C = mu.shape[0], mu.shape[1]
    F = np.empty(K, dtype=np.float64)
    lib.orc_rounding_l1_bound(d, _p(n_a, _ip), _p(lo_a), _p(hi_a), K, C, _p(mu), _p(sigma),
                              _p(w), float(n_sigma), PREC_IDS[precision], float(eps), _p(F),
                              int(nthreads))
    return F


def moments(n, lo, hi, f, mu, sigma, weight=None, n_sigma=4.0, fmu=None, nthreads=0):
    """(mean[K], var[K], delta2[K] or None)."""
    lib = _load()
    d, n_a, lo_a, hi_a = _grid_args(n, lo, hi)
    f = _d(f)
    mu = _d(mu)
    sigma = _d(sigma)
    w = _d(weight)
    K, C = mu.shape[0], mu.shape[1]
    mean = np.empty(K)
    var = np.empty(K)
    d2 = np.empty(K) if fmu is not None else None
    fm = _d(fmu)
    lib.orc_moments(d, _p(n_a, _ip), _p(lo_a), _p(hi_a), _p(f), K, C, _p(mu), _p(sigma), _p(w),
                    float(n_sigma), _p(fm), _p(mean), _p(var), _p(d2), int(nthreads))
    return mean, var, d2


def ipsa(P, edges):
    """(mean_hist[K], var[K], entropy[K]) of each column of P (FP64)."""
    lib = _load()
    P = _d(P)
    e = _d(edges)
    K, B = P.shape
    m = np.empty(K)
    v = np.empty(K)
    h = np.empty(K)
    lib.orc_ipsa(_p(P), K, B, _p(e), _p(m), _p(v), _p(h))
    return m, v, h


def ipsa_grad(n, lo, hi, bin_, edges, mu, sigma, weight, win, P, g_var=None, g_ent=None,
              nthreads=0):
    """Analytic gradient of g_var*Var + g_ent*H wrt mu, sigma [K][C][d] and weight [K][C]."""
    lib = _load()
    d, n_a, lo_a, hi_a = _grid_args(n, lo, hi)
    b = np.ascontiguousarray(bin_, dtype=np.int32)
    e = _d(edges)
    mu = _d(mu)
    sigma = _d(sigma)
    w = _d(weight)
    K, C = mu.shape[0], mu.shape[1]
    P = _d(P)
    gv = _d(g_var)
    ge = _d(g_ent)
    wn = np.ascontiguousarray(win, dtype=np.int32)
    gm = np.empty((K, C, d))
    gs = np.empty((K, C, d))
    gw = np.empty((K, C))
    lib.orc_ipsa_grad(d, _p(n_a, _ip), _p(lo_a), _p(hi_a), _p(b, _ip), e.size - 1, _p(e), K, C,
                      _p(mu), _p(sigma), _p(w), _p(wn, _ip), _p(P), _p(gv), _p(ge), _p(gm),
                      _p(gs), _p(gw), int(nthreads))
    return gm, gs, gw


def objective(n, lo, hi, bin_, edges, mu, sigma, weight, win, g_var, g_ent):
    """Q_k = g_var Var_k + g_ent H_k of the FP64 forward on frozen windows."""
    B = len(edges) - 1
    P, _ = propagate(n, lo, hi, bin_, B, mu, sigma, weight, precision="fp64", win=win)
    _, v, h = ipsa(P, edges)
    return np.asarray(g_var) * v + np.asarray(g_ent) * h


# ---------------------------------------------------------------------------
# convenience: the whole oracle pipeline for a workloads.Workload
# ---------------------------------------------------------------------------
def run_workload(wl, precision="fp64", with_moments=True, nthreads=0):
    f = eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
    edges = uniform_edges(f, wl.B)
    b = bins(f, edges)
    P, Z = propagate(wl.n, wl.lo, wl.hi, b, wl.B, wl.mu, wl.sigma, wl.weight, wl.n_sigma,
                     precision, nthreads=nthreads)
    out = dict(f=f, edges=edges, bin=b, P=P, Z=Z)
    if with_moments:
        out["mean"], out["var"], _ = moments(wl.n, wl.lo, wl.hi, f, wl.mu, wl.sigma, wl.weight,
                                             wl.n_sigma, nthreads=nthreads)
    out["mean_hist"], out["var_hist"], out["entropy"] = ipsa(P, edges)
    return out
