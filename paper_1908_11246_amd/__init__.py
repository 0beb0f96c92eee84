"""Python binding of libvup.so: Vectorized Uncertainty Propagation (VUP) and
Input Probability Sensitivity Analysis (IPSA), arXiv:1908.11246, on MI355X.

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and the current HIP stream. The
binding fails loudly when the library or a GPU is missing; there is no CPU
fallback.

    mm = build_model_matrix(grid, f, edges)        # eq. (5): model matrix, once
    P, Z = propagate(mm, mu, sigma)                # eq. VUP for all K pdfs at once
    mean, var, _ = moments(mm, mu, sigma)          # exact-f output moments
    mean_h, var_h, ent = ipsa(mm, P)               # IPSA coarse-grained quantities
    var_h, ent = IPSA.apply(mu, sigma, None, mm)   # differentiable wrt mu, sigma
    y_l = eval_points("ipsa2", mu[:, 0, :])        # y(l): the model at each pdf's maximum
    Q, lost = ipsa_matrix(mm, P, y_l, -3.0, 0.01, 600)   # IPSA probability matrix
    fl = ipsa_fields(mm, P, y_l, (0.025, 0.975))   # mode, intervals, deviation per l
    g = marginalize(Q)                             # global marginal over locations
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libvup.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "vup.h")

VUP_OK = 0
STATUS = {-1: "VUP_EINVAL", -2: "VUP_ENODEV", -3: "VUP_EDEVICE", -4: "VUP_EUNSUPPORTED",
          -5: "VUP_EWORKSPACE"}
PRECISIONS = {"fp32": 0, "bf16": 1, "bf16x2": 2, "fp8e4m3": 3}
MODELS = {"linear": 0, "sincos2": 1, "damped3": 2, "ring4": 3, "timing2": 4, "ipsa2": 5}


class VupError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class VupGrid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 4),
                ("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4)]


class VupModel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("theta", ctypes.c_double * 8)]


class VupDists(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int64), ("ncomp", ctypes.c_int32), ("ndim", ctypes.c_int32),
                ("n_sigma", ctypes.c_double), ("mu", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("weight", ctypes.c_void_p)]


class VupSepDists(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32 * 2), ("n_sigma", ctypes.c_double),
                ("mu", ctypes.c_void_p * 2), ("sigma", ctypes.c_void_p * 2),
                ("precision", ctypes.c_int32)]


class VupMM(ctypes.Structure):
    _fields_ = [("grid", VupGrid), ("B", ctypes.c_int32), ("pitch", ctypes.c_int32),
                ("N", ctypes.c_int64), ("rows", ctypes.c_int64), ("ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t), ("off_edges", ctypes.c_size_t),
                ("off_binmap", ctypes.c_size_t), ("off_f32", ctypes.c_size_t),
                ("off_counts", ctypes.c_size_t), ("off_offsets", ctypes.c_size_t),
                ("off_perm", ctypes.c_size_t), ("off_scratch", ctypes.c_size_t),
                ("off_counters", ctypes.c_size_t), ("off_runs", ctypes.c_size_t),
                ("off_rowptr", ctypes.c_size_t), ("off_runidx", ctypes.c_size_t),
                ("sweep", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("magic", ctypes.c_uint64)]


_lib = None
_vp = ctypes.c_void_p
_P = ctypes.POINTER


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIBPATH)
    lib.vup_last_error.restype = ctypes.c_char_p
    lib.vup_version.restype = ctypes.c_char_p
    lib.vup_eval_grid.argtypes = [_P(VupGrid), _P(VupModel), _vp, _vp]
    lib.vup_uniform_edges.argtypes = [_vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp]
    lib.vup_bin_workspace_bytes.restype = ctypes.c_size_t
    lib.vup_bin_workspace_bytes.argtypes = [_P(VupGrid), ctypes.c_int32]
    lib.vup_bin.argtypes = [_P(VupGrid), _vp, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_size_t,
                            _P(VupMM), _vp]
    lib.vup_windows.argtypes = [_P(VupGrid), _P(VupDists), _vp, _vp]
    lib.vup_propagate.argtypes = [_P(VupMM), _P(VupDists), ctypes.c_int32, _vp, _vp, _vp]
    lib.vup_moments.argtypes = [_P(VupMM), _P(VupDists), _P(VupModel), _vp, _vp, _vp, _vp]
    lib.vup_moments_tiled_workspace_bytes.restype = ctypes.c_size_t
    lib.vup_moments_tiled_workspace_bytes.argtypes = [_P(VupMM), _P(VupDists)]
    lib.vup_moments_tiled.argtypes = [_P(VupMM), _P(VupDists), _P(VupModel), _vp, ctypes.c_size_t,
                                      _vp, _vp, _vp, _vp]
    lib.vup_ipsa.argtypes = [_P(VupMM), ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]
    lib.vup_ipsa_backward.argtypes = [_P(VupMM), _P(VupDists), _vp, _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp]
    lib.vup_counters.argtypes = [_P(VupMM), _vp, _P(ctypes.c_int64)]
    lib.vup_set_sweep_mode.argtypes = [_P(VupMM), ctypes.c_int32, _vp]
    lib.vup_separable_workspace_bytes.restype = ctypes.c_size_t
    lib.vup_separable_workspace_bytes.argtypes = [_P(VupMM), ctypes.c_int32, ctypes.c_int32]
    lib.vup_propagate_separable.argtypes = [_P(VupMM), _P(VupSepDists), _vp, ctypes.c_size_t, _vp,
                                            _vp, _vp]
    lib.vup_eval_points.argtypes = [_P(VupModel), ctypes.c_int32, ctypes.c_int64, _vp,
                                    ctypes.c_int64, _vp, _vp]
    lib.vup_ipsa_matrix.argtypes = [_P(VupMM), ctypes.c_int64, _vp, _vp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp]
    lib.vup_ipsa_fields.argtypes = [_P(VupMM), ctypes.c_int64, _vp, _vp, ctypes.c_int32,
                                    _P(ctypes.c_double), _vp, _vp, _vp, _vp, _vp, _vp]
    lib.vup_posterior.argtypes = [_P(VupMM), _P(VupDists), ctypes.c_int64, _vp, _vp, _vp, _vp, _vp,
                                  _vp]
    lib.vup_marginal_workspace_bytes.restype = ctypes.c_size_t
    lib.vup_marginal_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
    lib.vup_marginalize.argtypes = [ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_size_t,
                                    _vp, _vp]
    lib.vup_marginalize_noalloc.argtypes = [ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp]
    _lib = lib
    return lib


def lib():
    return _load()


def header_functions() -> list:
    """Names of the functions declared in include/vup.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(vup_\w+)\s*\(", txt, re.M)))


def _check(code: int):
    if code != VUP_OK:
        raise VupError(code, _load().vup_last_error().decode())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f64(t, device) -> torch.Tensor:
    t = torch.as_tensor(t)
    return t.to(device=device, dtype=torch.float64).contiguous()


def make_grid(n: Sequence[int], lo: Sequence[float], hi: Sequence[float]) -> VupGrid:
    g = VupGrid()
    g.ndim = len(n)
    for d in range(len(n)):
        g.n[d] = int(n[d])
        g.lo[d] = float(lo[d])
        g.hi[d] = float(hi[d])
    return g


def make_model(name: str, theta: Sequence[float] = ()) -> VupModel:
    m = VupModel()
    m.kind = MODELS[name]
    for i, v in enumerate(theta):
        m.theta[i] = float(v)
    return m


def _dists(mu: torch.Tensor, sigma: torch.Tensor, weight: Optional[torch.Tensor],
           n_sigma: float) -> VupDists:
    d = VupDists()
    d.K = mu.shape[0]
    d.ncomp = mu.shape[1]
    d.ndim = mu.shape[2]
    d.n_sigma = float(n_sigma)
    d.mu = mu.data_ptr() if mu.numel() else None
    d.sigma = sigma.data_ptr() if sigma.numel() else None
    d.weight = None if weight is None else weight.data_ptr()
    return d


def _norm_params(mu, sigma, weight, device):
    mu = _dev_f64(mu, device)
    sigma = _dev_f64(sigma, device)
    if mu.dim() == 2:
        mu = mu.unsqueeze(1)
        sigma = sigma.unsqueeze(1)
    if mu.shape != sigma.shape:
        raise ValueError("mu and sigma must have the same shape [K][C][d]")
    w = None if weight is None else _dev_f64(weight, device)
    return mu, sigma, w


def eval_grid(grid: VupGrid, model: str, theta: Sequence[float] = (), device="cuda") -> torch.Tensor:
    """Alg. VUP: f_i = M(x_i) at every cell centre (FP64, row major)."""
    N = 1
    for d in range(grid.ndim):
        N *= grid.n[d]
    f = torch.empty(N, dtype=torch.float64, device=device)
    m = make_model(model, theta)
    _check(_load().vup_eval_grid(ctypes.byref(grid), ctypes.byref(m), _ptr(f), _vp(_stream())))
    return f


def uniform_edges(f: torch.Tensor, B: int) -> torch.Tensor:
    e = torch.empty(B + 1, dtype=torch.float64, device=f.device)
    _check(_load().vup_uniform_edges(_ptr(f), f.numel(), int(B), _ptr(e), _vp(_stream())))
    return e


class ModelMatrix:
    """The sparse one-hot model matrix of eq. (5), built once by vup_bin and
    reused for every propagated distribution. Owns its device workspace."""

    def __init__(self, grid: VupGrid, f: torch.Tensor, edges: torch.Tensor,
                 want_bin: bool = True, resolve_sweep: bool = True):
        lib_ = _load()
        self.grid = grid
        self.B = edges.numel() - 1
        nbytes = lib_.vup_bin_workspace_bytes(ctypes.byref(grid), self.B)
        if nbytes == 0:
            raise VupError(-1, "invalid grid or bin count")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=f.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.mm = VupMM()
        self.bin = torch.empty(f.numel(), dtype=torch.int32, device=f.device) if want_bin else None
        _check(lib_.vup_bin(ctypes.byref(grid), _ptr(f), _ptr(edges), self.B, _ptr(self.bin),
                            _vp(self._ws_ptr), nbytes, ctypes.byref(self.mm), _vp(_stream())))
        self.device = f.device
        if resolve_sweep:
            # fix the FP32 sweep form now (one stream sync at set-up), so that
            # each propagation launches only that form
            self.set_sweep_mode("auto")

    def _view(self, off, dtype, count):
        start = self._ws_ptr - self.ws.data_ptr() + off
        esz = torch.empty((), dtype=dtype).element_size()
        return self.ws[start:start + count * esz].view(dtype)

    @property
    def edges(self) -> torch.Tensor:
        return self._view(self.mm.off_edges, torch.float64, self.B + 1)

    @property
    def counts(self) -> torch.Tensor:
        """cells per bin; index B counts cells with no bin."""
        return self._view(self.mm.off_counts, torch.int64, self.B + 1)

    @property
    def offsets(self) -> torch.Tensor:
        """CSR row starts of the model matrix (by bin); offsets[B] = binned cells."""
        return self._view(self.mm.off_offsets, torch.int64, self.B + 1)

    @property
    def runs(self) -> torch.Tensor:
        """run records (first cell | 4*bin << 16) of every row, one terminator per row."""
        n = int(self.mm.N + self.mm.rows)
        return self._view(self.mm.off_runs, torch.int32, n)

    @property
    def rowptr(self) -> torch.Tensor:
        return self._view(self.mm.off_rowptr, torch.int32, int(self.mm.rows) + 1)

    @property
    def runidx(self) -> torch.Tensor:
        """run of each cell (padded rows), relative to its row's first run."""
        return self._view(self.mm.off_runidx, torch.int16, int(self.mm.rows * self.mm.pitch))

    @property
    def perm(self) -> torch.Tensor:
        """binned cell indices sorted by bin, increasing within a bin."""
        return self._view(self.mm.off_perm, torch.int32, int(self.mm.N))

    @property
    def sweep(self) -> str:
        """FP32 propagation form in use: "auto" (unresolved), "cells" or "runs"."""
        return {0: "auto", 1: "cells", 2: "runs"}[self.mm.sweep]

    def set_sweep_mode(self, mode: str = "auto"):
        """FP32 propagation form: "auto" (resolve from the run statistics; syncs),
        "cells" (per-cell) or "runs" (run form)."""
        m = {"auto": 0, "cells": 1, "runs": 2}[mode]
        _check(_load().vup_set_sweep_mode(ctypes.byref(self.mm), m, _vp(_stream())))

    def counters(self) -> dict:
        out = (ctypes.c_int64 * 4)()
        _check(_load().vup_counters(ctypes.byref(self.mm), _vp(_stream()), out))
        return dict(outside=out[0], bad_edges=out[1], bad_param=out[2], empty=out[3])


def build_model_matrix(grid: VupGrid, f: torch.Tensor, edges: torch.Tensor,
                       want_bin: bool = True, resolve_sweep: bool = True) -> ModelMatrix:
    return ModelMatrix(grid, f, edges, want_bin, resolve_sweep)


def windows(grid: VupGrid, mu, sigma, n_sigma: float = 4.0, device="cuda",
            weight=None) -> torch.Tensor:
    """Integer truncation windows [K][C][d][2] (inclusive; empty = (0, -1))."""
    mu, sigma, w = _norm_params(mu, sigma, weight, device)
    K, C, D = mu.shape
    if C > 1 and w is None:
        w = torch.full((K, C), 1.0 / C, dtype=torch.float64, device=device)
    win = torch.empty((K, C, D, 2), dtype=torch.int32, device=device)
    d = _dists(mu, sigma, w, n_sigma)
    _check(_load().vup_windows(ctypes.byref(grid), ctypes.byref(d), _ptr(win), _vp(_stream())))
    return win


def propagate(mm: ModelMatrix, mu, sigma, weight=None, precision: str = "fp32",
              n_sigma: float = 4.0, out: Optional[torch.Tensor] = None, want_Z: bool = True):
    """eq. VUP: P[K][B] (FP32) and Z[K][C] (FP64) for all distributions at once."""
    mu, sigma, w = _norm_params(mu, sigma, weight, mm.device)
    K, C, _ = mu.shape
    P = out if out is not None else torch.empty((K, mm.B), dtype=torch.float32, device=mm.device)
    Z = torch.empty((K, C), dtype=torch.float64, device=mm.device) if want_Z else None
    d = _dists(mu, sigma, w, n_sigma)
    _check(_load().vup_propagate(ctypes.byref(mm.mm), ctypes.byref(d), PRECISIONS[precision],
                                 _ptr(P), _ptr(Z), _vp(_stream())))
    return P, Z


class SeparableWorkspace:
    """Device workspace of the separable (banded MFMA) propagation."""

    def __init__(self, mm: ModelMatrix, Mx: int, My: int):
        n = _load().vup_separable_workspace_bytes(ctypes.byref(mm.mm), int(Mx), int(My))
        if n == 0:
            raise VupError(-1, "separable form needs a 2-D model matrix")
        self.buf = torch.empty(n + 256, dtype=torch.uint8, device=mm.device)
        self.ptr = (self.buf.data_ptr() + 255) // 256 * 256
        self.nbytes = n
        self.M = (int(Mx), int(My))


def propagate_separable(mm: ModelMatrix, mu_x, mu_y, sigma_x, sigma_y, n_sigma: float = 4.0,
                        ws: Optional[SeparableWorkspace] = None, want_Z: bool = True,
                        precision: str = "fp32"):
    """eq. VUP for the tensor-product family k = mx*My + my (banded MFMA form);
    precision "fp32", "bf16" or "bf16x2" picks the contraction's operands."""
    mx = _dev_f64(mu_x, mm.device)
    my = _dev_f64(mu_y, mm.device)
    sx = _dev_f64(sigma_x, mm.device)
    sy = _dev_f64(sigma_y, mm.device)
    Mx, My = mx.numel(), my.numel()
    if ws is None or ws.M != (Mx, My):
        ws = SeparableWorkspace(mm, Mx, My)
    P = torch.empty((Mx * My, mm.B), dtype=torch.float32, device=mm.device)
    Z = torch.empty(Mx * My, dtype=torch.float64, device=mm.device) if want_Z else None
    s = VupSepDists()
    s.M[0], s.M[1] = Mx, My
    s.n_sigma = float(n_sigma)
    s.mu[0], s.mu[1] = mx.data_ptr(), my.data_ptr()
    s.sigma[0], s.sigma[1] = sx.data_ptr(), sy.data_ptr()
    s.precision = PRECISIONS[precision]
    _check(_load().vup_propagate_separable(ctypes.byref(mm.mm), ctypes.byref(s), _vp(ws.ptr),
                                           ws.nbytes, _ptr(P), _ptr(Z), _vp(_stream())))
    return P, Z, ws


def moments(mm: ModelMatrix, mu, sigma, weight=None, model: Optional[str] = None,
            theta: Sequence[float] = (), n_sigma: float = 4.0, tiled: bool = True,
            workspace: Optional[torch.Tensor] = None):
    """(mean[K], var[K], delta2[K] or None) from the exact model values.

    ``tiled`` selects vup_moments_tiled (matrix-core tiles; 2-D grids with
    single-component pdfs, other cases run the per-pdf kernel) over
    vup_moments. ``workspace`` (uint8, on the device) is used when large
    enough, else one is allocated."""
    mu, sigma, w = _norm_params(mu, sigma, weight, mm.device)
    K = mu.shape[0]
    mean = torch.empty(K, dtype=torch.float64, device=mm.device)
    var = torch.empty(K, dtype=torch.float64, device=mm.device)
    d2 = torch.empty(K, dtype=torch.float64, device=mm.device) if model else None
    m = make_model(model, theta) if model else None
    d = _dists(mu, sigma, w, n_sigma)
    lib = _load()
    mref = ctypes.byref(m) if m is not None else None
    if tiled:
        ws, nb = _moments_ws(mm, d, workspace)
        _check(lib.vup_moments_tiled(ctypes.byref(mm.mm), ctypes.byref(d), mref,
                                     _ptr(ws) if ws is not None else None, nb, _ptr(mean),
                                     _ptr(var), _ptr(d2), _vp(_stream())))
    else:
        _check(lib.vup_moments(ctypes.byref(mm.mm), ctypes.byref(d), mref, _ptr(mean), _ptr(var),
                               _ptr(d2), _vp(_stream())))
    return mean, var, d2


def moments_workspace(mm: ModelMatrix, mu, sigma, weight=None, n_sigma: float = 4.0):
    """A device workspace for ``moments(..., tiled=True)`` with these pdfs
    (None when the tiled form does not apply)."""
    mu, sigma, w = _norm_params(mu, sigma, weight, mm.device)
    ws, _ = _moments_ws(mm, _dists(mu, sigma, w, n_sigma), None)
    return ws


def _moments_ws(mm, d, workspace):
    nb = int(_load().vup_moments_tiled_workspace_bytes(ctypes.byref(mm.mm), ctypes.byref(d)))
    if nb == 0:
        return None, 0
    if workspace is not None and workspace.numel() >= nb and workspace.data_ptr() % 256 == 0:
        return workspace, workspace.numel()
    return torch.empty(nb, dtype=torch.uint8, device=mm.device), nb


def ipsa(mm: ModelMatrix, P: torch.Tensor):
    """(mean_hist[K], var[K], entropy[K]) of each propagated column (FP64)."""
    K = P.shape[0]
    m = torch.empty(K, dtype=torch.float64, device=P.device)
    v = torch.empty(K, dtype=torch.float64, device=P.device)
    h = torch.empty(K, dtype=torch.float64, device=P.device)
    _check(_load().vup_ipsa(ctypes.byref(mm.mm), K, _ptr(P), _ptr(m), _ptr(v), _ptr(h),
                            _vp(_stream())))
    return m, v, h


def eval_points(model: str, x, theta: Sequence[float] = (), ndim: Optional[int] = None,
                device="cuda") -> torch.Tensor:
    """y_i = M(x_i) at the rows of x ([n][ldx]; the first ``ndim`` entries of
    each row are the point, default all of them). ``x`` may be a strided view
    such as mu[:, 0, :] of a [K][C][d] parameter tensor."""
    x = torch.as_tensor(x)
    if x.device.type != "cuda" or x.dtype != torch.float64:
        x = x.to(device=device, dtype=torch.float64)
    if x.dim() != 2 or x.stride(1) != 1:
        x = x.contiguous()
    n = x.shape[0]
    nd = x.shape[1] if ndim is None else int(ndim)
    ldx = x.stride(0) if n > 1 else x.shape[1]
    y = torch.empty(n, dtype=torch.float64, device=x.device)
    m = make_model(model, theta)
    _check(_load().vup_eval_points(ctypes.byref(m), nd, n, _ptr(x) if n else None, max(ldx, nd),
                                   _ptr(y), _vp(_stream())))
    return y


def ipsa_matrix(mm: ModelMatrix, P: torch.Tensor, y_ref: torch.Tensor, dy_lo: float,
                dy_width: float, n_dy: int):
    """IPSA probability matrix Q[K][n_dy] (FP32) and lost mass[K] (FP64):
    each column of P translated by y_ref and re-binned on d_j = dy_lo + j*dy_width."""
    K = P.shape[0]
    y = _dev_f64(y_ref, P.device)
    Q = torch.empty((K, int(n_dy)), dtype=torch.float32, device=P.device)
    lost = torch.empty(K, dtype=torch.float64, device=P.device)
    _check(_load().vup_ipsa_matrix(ctypes.byref(mm.mm), K, _ptr(P), _ptr(y), float(dy_lo),
                                   float(dy_width), int(n_dy), _ptr(Q), _ptr(lost),
                                   _vp(_stream())))
    return Q, lost


def ipsa_fields(mm: ModelMatrix, P: torch.Tensor, y_ref: Optional[torch.Tensor] = None,
                levels: Sequence[float] = ()):
    """Field lines of each column: y_mode, p_max, quant[K][len(levels)] and,
    with y_ref, dev and delta2 (all FP64)."""
    K = P.shape[0]
    dev_ = P.device
    f64 = dict(dtype=torch.float64, device=dev_)
    y = None if y_ref is None else _dev_f64(y_ref, dev_)
    out = dict(y_mode=torch.empty(K, **f64), p_max=torch.empty(K, **f64),
               quant=torch.empty((K, len(levels)), **f64) if len(levels) else None,
               dev=torch.empty(K, **f64) if y is not None else None,
               delta2=torch.empty(K, **f64) if y is not None else None)
    lv = (ctypes.c_double * max(len(levels), 1))(*[float(a) for a in levels])
    _check(_load().vup_ipsa_fields(ctypes.byref(mm.mm), K, _ptr(P), _ptr(y), len(levels), lv,
                                   _ptr(out["y_mode"]), _ptr(out["p_max"]), _ptr(out["quant"]),
                                   _ptr(out["dev"]), _ptr(out["delta2"]), _vp(_stream())))
    return out


def marginal_workspace_bytes(K: int, n: int) -> int:
    return int(_load().vup_marginal_workspace_bytes(int(K), int(n)))


def marginalize(A: torch.Tensor, rho: Optional[torch.Tensor] = None,
                ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out[j] = sum_k rho_k A[k][j] (FP64; rho None: 1/K). ``ws`` may be a
    reusable uint8 device tensor of at least marginal_workspace_bytes(K, n)."""
    K, n = A.shape
    r = None if rho is None else _dev_f64(rho, A.device)
    need = marginal_workspace_bytes(K, n)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=A.device)
    out = torch.empty(n, dtype=torch.float64, device=A.device)
    _check(_load().vup_marginalize(K, n, _ptr(A), _ptr(r), _ptr(ws), ws.numel(), _ptr(out),
                                   _vp(_stream())))
    return out


def marginalize_noalloc(A: torch.Tensor, rho: Optional[torch.Tensor] = None,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """marginalize() with the partial sums in the library's own device array
    (no workspace); ``out`` may be a preallocated FP64 tensor of n elements."""
    K, n = A.shape
    r = None if rho is None else _dev_f64(rho, A.device)
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=A.device)
    _check(_load().vup_marginalize_noalloc(K, n, _ptr(A), _ptr(r), _ptr(out), _vp(_stream())))
    return out


def posterior(mm: ModelMatrix, mu, sigma, weight, sel, P: torch.Tensor, Z: torch.Tensor,
              n_sigma: float = 4.0, want_mean: bool = True):
    """Bayes inversion (Sec. 3): post[t][i] = p_k(x_i) / P[k][bin(i)] for k = sel[t]
    (FP32 [n_sel][N]) and, optionally, per-bin posterior means [n_sel][B][ndim]."""
    mu, sigma, w = _norm_params(mu, sigma, weight, mm.device)
    s = torch.as_tensor(sel).to(device=mm.device, dtype=torch.int64).contiguous()
    n_sel = s.numel()
    post = torch.empty((n_sel, int(mm.mm.N)), dtype=torch.float32, device=mm.device)
    mean = (torch.empty((n_sel, mm.B, mm.grid.ndim), dtype=torch.float64, device=mm.device)
            if want_mean else None)
    d = _dists(mu, sigma, w, n_sigma)
    _check(_load().vup_posterior(ctypes.byref(mm.mm), ctypes.byref(d), n_sel, _ptr(s), _ptr(P),
                                 _ptr(Z.contiguous()), _ptr(post), _ptr(mean), _vp(_stream())))
    return post, mean


def ipsa_backward(mm: ModelMatrix, mu, sigma, weight, P, mean_hist, g_var=None, g_ent=None,
                  n_sigma: float = 4.0):
    """Gradients of g_var*var + g_ent*entropy wrt mu, sigma [K][C][d], weight [K][C]."""
    mu, sigma, w = _norm_params(mu, sigma, weight, mm.device)
    K, C, D = mu.shape
    gm = torch.empty((K, C, D), dtype=torch.float64, device=mm.device)
    gs = torch.empty((K, C, D), dtype=torch.float64, device=mm.device)
    gw = torch.empty((K, C), dtype=torch.float64, device=mm.device)
    gv = None if g_var is None else _dev_f64(g_var, mm.device)
    ge = None if g_ent is None else _dev_f64(g_ent, mm.device)
    d = _dists(mu, sigma, w, n_sigma)
    _check(_load().vup_ipsa_backward(ctypes.byref(mm.mm), ctypes.byref(d), _ptr(P),
                                     _ptr(mean_hist), _ptr(gv), _ptr(ge), _ptr(gm), _ptr(gs),
                                     _ptr(gw), _vp(_stream())))
    return gm, gs, gw


class IPSA(torch.autograd.Function):
    """IPSA map (per-location output variance and entropy) as a differentiable
    function of the input pdf parameters; the backward is the library's
    adjoint sweep (windows held fixed)."""

    @staticmethod
    def forward(ctx, mu, sigma, weight, mm: ModelMatrix, n_sigma: float = 4.0):
        P, _ = propagate(mm, mu.detach(), sigma.detach(),
                         None if weight is None else weight.detach(), "fp32", n_sigma)
        mean_h, var, ent = ipsa(mm, P)
        ctx.mm = mm
        ctx.n_sigma = n_sigma
        ctx.has_weight = weight is not None
        ctx.save_for_backward(mu.detach(), sigma.detach(),
                              weight.detach() if weight is not None else mu.new_empty(0), P,
                              mean_h)
        return var, ent

    @staticmethod
    def backward(ctx, g_var, g_ent):
        mu, sigma, weight, P, mean_h = ctx.saved_tensors
        w = weight if ctx.has_weight else None
        gv = g_var if g_var is not None else torch.zeros_like(mean_h)
        ge = g_ent if g_ent is not None else torch.zeros_like(mean_h)
        gm, gs, gw = ipsa_backward(ctx.mm, mu, sigma, w, P, mean_h, gv.contiguous(),
                                   ge.contiguous(), ctx.n_sigma)
        gm = gm.reshape(mu.shape).to(mu.dtype)
        gs = gs.reshape(sigma.shape).to(sigma.dtype)
        gwo = gw.reshape(weight.shape).to(weight.dtype) if ctx.has_weight else None
        return gm, gs, gwo, None, None
