"""Host-side checks of the C ABI: the library loads, exports every entry point
include/vup.h declares, and rejects invalid arguments before touching a GPU.
No compute call is made here (this runs on machines without a GPU)."""
import ctypes
import subprocess

import pytest
import torch

import paper_1908_11246_amd as vup

EINVAL, ENODEV, EWORKSPACE, EUNSUPPORTED = -1, -2, -5, -4


@pytest.fixture(scope="module")
def lib():
    return vup.lib()


def test_exports_every_declared_symbol(lib):
    names = vup.header_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", vup.LIBPATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for n in names:
        assert n in exported, n
        assert getattr(lib, n) is not None


def test_version_and_empty_error(lib):
    assert b"gfx950" in lib.vup_version()
    assert isinstance(lib.vup_last_error(), bytes)


def _grid(n=(8, 8), lo=(0.0, 0.0), hi=(1.0, 1.0)):
    return vup.make_grid(n, lo, hi)


def test_invalid_grids_rejected(lib):
    m = vup.make_model("sincos2")
    dummy = ctypes.c_void_p(0x1000)
    g = _grid()
    g.ndim = 0
    assert lib.vup_eval_grid(ctypes.byref(g), ctypes.byref(m), dummy, None) == EINVAL
    g = _grid()
    g.n[1] = 0
    assert lib.vup_eval_grid(ctypes.byref(g), ctypes.byref(m), dummy, None) == EINVAL
    assert b"n[1]" in lib.vup_last_error()
    g = _grid(hi=(1.0, 0.0))
    assert lib.vup_eval_grid(ctypes.byref(g), ctypes.byref(m), dummy, None) == EINVAL
    g = _grid(lo=(0.0, float("nan")))
    assert lib.vup_eval_grid(ctypes.byref(g), ctypes.byref(m), dummy, None) == EINVAL
    # model / ndim mismatch and unknown model
    g3 = _grid((4, 4, 4), (0, 0, 0), (1, 1, 1))
    assert lib.vup_eval_grid(ctypes.byref(g3), ctypes.byref(m), dummy, None) == EINVAL
    m.kind = 99
    assert lib.vup_eval_grid(ctypes.byref(_grid()), ctypes.byref(m), dummy, None) == EINVAL
    # NULL output
    assert lib.vup_eval_grid(ctypes.byref(_grid()), ctypes.byref(vup.make_model("sincos2")),
                             None, None) == EINVAL
    # too many cells for 32-bit offsets
    big = _grid((65536, 65536), (0, 0), (1, 1))
    assert lib.vup_eval_grid(ctypes.byref(big), ctypes.byref(vup.make_model("sincos2")),
                             dummy, None) == EUNSUPPORTED


def test_edges_and_bin_arguments(lib):
    dummy = ctypes.c_void_p(0x1000)
    assert lib.vup_uniform_edges(dummy, 10, 0, dummy, None) == EINVAL
    assert lib.vup_uniform_edges(dummy, 10, 5000, dummy, None) == EINVAL
    assert lib.vup_uniform_edges(dummy, 0, 4, dummy, None) == EINVAL
    assert lib.vup_uniform_edges(None, 10, 4, dummy, None) == EINVAL
    g = _grid()
    assert lib.vup_bin_workspace_bytes(ctypes.byref(g), 16) > 0
    assert lib.vup_bin_workspace_bytes(ctypes.byref(g), 0) == 0
    mm = vup.VupMM()
    need = lib.vup_bin_workspace_bytes(ctypes.byref(g), 16)
    assert lib.vup_bin(ctypes.byref(g), dummy, dummy, 16, None, None, need,
                       ctypes.byref(mm), None) == EWORKSPACE
    assert lib.vup_bin(ctypes.byref(g), dummy, dummy, 16, None, ctypes.c_void_p(0x1001), need,
                       ctypes.byref(mm), None) == EWORKSPACE
    assert lib.vup_bin(ctypes.byref(g), dummy, dummy, 16, None, ctypes.c_void_p(0x100000),
                       need - 1, ctypes.byref(mm), None) == EWORKSPACE
    assert lib.vup_bin(ctypes.byref(g), dummy, dummy, 0, None, ctypes.c_void_p(0x100000), need,
                       ctypes.byref(mm), None) == EINVAL


def test_workspace_grows_with_grid_and_bins(lib):
    a = lib.vup_bin_workspace_bytes(ctypes.byref(_grid((64, 64))), 64)
    b = lib.vup_bin_workspace_bytes(ctypes.byref(_grid((128, 64))), 64)
    c = lib.vup_bin_workspace_bytes(ctypes.byref(_grid((64, 64))), 1024)
    assert 0 < a < b and a < c
    # 1024 x 1024 cells: FP32 map, bin map, sorted cells, run records and the
    # cell-to-run index (16 bytes per cell), plus the (bin, chunk) count table
    # of the sort (1 MiB at B = 256)
    d = lib.vup_bin_workspace_bytes(ctypes.byref(_grid((1024, 1024))), 256)
    assert 16 * 2 ** 20 <= d <= 18 * 2 ** 20


def test_descriptor_must_come_from_vup_bin(lib):
    mm = vup.VupMM()
    d = vup.VupDists()
    d.K = 1
    d.ncomp = 1
    d.ndim = 2
    d.n_sigma = 4.0
    dummy = ctypes.c_void_p(0x1000)
    assert lib.vup_propagate(ctypes.byref(mm), ctypes.byref(d), 0, dummy, None, None) == EWORKSPACE
    assert lib.vup_moments(ctypes.byref(mm), ctypes.byref(d), None, dummy, dummy, None,
                           None) == EWORKSPACE
    assert lib.vup_ipsa(ctypes.byref(mm), 1, dummy, None, None, None, None) == EWORKSPACE
    assert lib.vup_counters(ctypes.byref(mm), None, (ctypes.c_int64 * 4)()) == EWORKSPACE


def _fake_mm(lib, B=16, n=(8, 8)):
    """A descriptor that passes the host checks (its workspace is never touched,
    because every call below fails validation before any launch)."""
    mm = vup.VupMM()
    mm.grid = _grid(n)
    mm.B = B
    mm.ws = 0x100000
    mm.magic = 0x5655504d4d763031
    return mm


def test_dists_validation(lib):
    mm = _fake_mm(lib)
    dummy = ctypes.c_void_p(0x1000)

    def dists(**kw):
        d = vup.VupDists()
        d.K, d.ncomp, d.ndim, d.n_sigma = 4, 1, 2, 4.0
        d.mu, d.sigma, d.weight = 0x1000, 0x2000, None
        for k, v in kw.items():
            setattr(d, k, v)
        return d

    cases = [dict(K=-1), dict(ncomp=3), dict(ndim=3), dict(n_sigma=0.0),
             dict(n_sigma=float("inf")), dict(mu=None), dict(ncomp=2), dict(weight=0x3000)]
    for kw in cases:
        d = dists(**kw)
        assert lib.vup_propagate(ctypes.byref(mm), ctypes.byref(d), 0, dummy, None, None) == EINVAL, kw
    d = dists()
    assert lib.vup_propagate(ctypes.byref(mm), ctypes.byref(d), 7, dummy, None, None) == EINVAL
    assert lib.vup_propagate(ctypes.byref(mm), ctypes.byref(d), 0, None, None, None) == EINVAL
    # delta2 needs one component and the model
    d2 = dists(ncomp=2, weight=0x3000)
    assert lib.vup_moments(ctypes.byref(mm), ctypes.byref(d2), None, dummy, dummy, dummy,
                           None) == EUNSUPPORTED
    assert lib.vup_moments(ctypes.byref(mm), ctypes.byref(d), None, dummy, dummy, dummy,
                           None) == EINVAL
    # ... a model of the grid's ndim (a 4-D model on a 2-D grid would read
    # coordinates the distributions do not have)
    m4 = vup.make_model("ring4")
    assert lib.vup_moments(ctypes.byref(mm), ctypes.byref(d), ctypes.byref(m4), dummy, dummy,
                           dummy, None) == EINVAL
    assert b"ndim" in lib.vup_last_error()
    m_bad = vup.make_model("sincos2")
    m_bad.kind = 42
    assert lib.vup_moments(ctypes.byref(mm), ctypes.byref(d), ctypes.byref(m_bad), dummy, dummy,
                           dummy, None) == EINVAL
    assert lib.vup_ipsa_backward(ctypes.byref(mm), ctypes.byref(d), None, dummy, None, None,
                                 dummy, dummy, None, None) == EINVAL


def test_moments_tiled_arguments(lib):
    """vup_moments_tiled: workspace size (80 + 8 + 16 bytes per pdf and 32 per
    64 x 64 tile, each part rounded up to 256), workspace checks, and the
    per-pdf kernel's rules where the tiled form does not apply."""
    mm = _fake_mm(lib)
    dummy = ctypes.c_void_p(0x1000)

    def dists(**kw):
        d = vup.VupDists()
        d.K, d.ncomp, d.ndim, d.n_sigma = 4, 1, 2, 4.0
        d.mu, d.sigma, d.weight = 0x1000, 0x2000, None
        for k, v in kw.items():
            setattr(d, k, v)
        return d

    d = dists()
    ws_bytes = lib.vup_moments_tiled_workspace_bytes(ctypes.byref(mm), ctypes.byref(d))
    assert ws_bytes == 512 + 256 + 256 + 256
    big = vup.VupDists()
    big.K, big.ncomp, big.ndim, big.n_sigma, big.mu, big.sigma = 1000, 1, 2, 4.0, 0x1000, 0x2000
    assert lib.vup_moments_tiled_workspace_bytes(ctypes.byref(mm), ctypes.byref(big)) == (
        80128 + 8192 + 16128 + 256)
    ws = ctypes.c_void_p(0x200000)

    def call(dd, ws_, nb, mean=dummy, var=dummy, d2=None, model=None):
        return lib.vup_moments_tiled(ctypes.byref(mm), ctypes.byref(dd), model, ws_, nb, mean, var,
                                     d2, None)

    assert call(d, None, ws_bytes) == EWORKSPACE
    assert call(d, ctypes.c_void_p(0x200010), ws_bytes) == EWORKSPACE
    assert b"aligned" in lib.vup_last_error()
    assert call(d, ws, ws_bytes - 1) == EWORKSPACE
    assert call(d, ws, ws_bytes, mean=None) == EINVAL
    assert call(d, ws, ws_bytes, d2=dummy) == EINVAL
    m4 = vup.make_model("ring4")
    assert call(d, ws, ws_bytes, d2=dummy, model=ctypes.byref(m4)) == EINVAL
    # tiles per axis up to 65 535, at most 2^20 in all; 3-D grids are not tiled
    long_mm = _fake_mm(lib, n=(16448, 8))
    assert lib.vup_moments_tiled_workspace_bytes(ctypes.byref(long_mm), ctypes.byref(d)) > 0
    big_mm = _fake_mm(lib, n=(65600, 1100))
    assert lib.vup_moments_tiled_workspace_bytes(ctypes.byref(big_mm), ctypes.byref(d)) == 0
    mm3 = _fake_mm(lib)
    mm3.grid = _grid((8, 8, 8), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    d3 = dists(ndim=3)
    assert lib.vup_moments_tiled_workspace_bytes(ctypes.byref(mm3), ctypes.byref(d3)) == 0
    # mixtures: not tiled (no workspace), vup_moments' rules apply
    d2c = dists(ncomp=2, weight=0x3000)
    assert lib.vup_moments_tiled_workspace_bytes(ctypes.byref(mm), ctypes.byref(d2c)) == 0
    assert call(d2c, None, 0, d2=dummy) == EUNSUPPORTED
    assert call(dists(K=-1), ws, ws_bytes) == EINVAL


def test_grid_too_long_for_lds_is_unsupported(lib):
    # factor tables of every axis live in LDS; four 16384-cell axes do not fit
    mm = _fake_mm(lib, B=16, n=(60000, 30000))
    d = vup.VupDists()
    d.K, d.ncomp, d.ndim, d.n_sigma = 1, 1, 2, 4.0
    d.mu, d.sigma = 0x1000, 0x2000
    mm.grid = _grid((16, 65536))
    assert lib.vup_propagate(ctypes.byref(mm), ctypes.byref(d), 0, ctypes.c_void_p(0x1000),
                             None, None) in (EUNSUPPORTED, EINVAL)


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-GPU path")
def test_no_device_is_reported(lib):
    g = _grid()
    m = vup.make_model("sincos2")
    assert lib.vup_eval_grid(ctypes.byref(g), ctypes.byref(m), ctypes.c_void_p(0x1000),
                             None) == ENODEV
    assert b"device" in lib.vup_last_error()


def test_field_line_arguments(lib):
    """Argument checks of the IPSA matrix / field lines / marginal / point
    evaluation entry points (all fail before any launch)."""
    mm = _fake_mm(lib)
    dummy = ctypes.c_void_p(0x1000)
    m = vup.make_model("ipsa2")
    # eval_points: ndim mismatch, ldx < ndim, negative n, NULL arrays
    assert lib.vup_eval_points(ctypes.byref(m), 3, 4, dummy, 3, dummy, None) == EINVAL
    assert lib.vup_eval_points(ctypes.byref(m), 2, 4, dummy, 1, dummy, None) == EINVAL
    assert lib.vup_eval_points(ctypes.byref(m), 2, -1, dummy, 2, dummy, None) == EINVAL
    assert lib.vup_eval_points(ctypes.byref(m), 2, 4, None, 2, dummy, None) == EINVAL
    assert lib.vup_eval_points(None, 2, 4, dummy, 2, dummy, None) == EINVAL
    # ipsa_matrix: bad target grid, NULL arrays, K < 0, bad descriptor
    mat = lib.vup_ipsa_matrix
    assert mat(ctypes.byref(mm), 4, dummy, dummy, 0.0, 0.1, 0, dummy, None, None) == EINVAL
    assert mat(ctypes.byref(mm), 4, dummy, dummy, 0.0, 0.0, 8, dummy, None, None) == EINVAL
    assert mat(ctypes.byref(mm), 4, dummy, dummy, float("nan"), 0.1, 8, dummy, None,
               None) == EINVAL
    assert mat(ctypes.byref(mm), 4, dummy, dummy, 0.0, float("inf"), 8, dummy, None,
               None) == EINVAL
    assert mat(ctypes.byref(mm), 4, dummy, None, 0.0, 0.1, 8, dummy, None, None) == EINVAL
    assert mat(ctypes.byref(mm), -1, dummy, dummy, 0.0, 0.1, 8, dummy, None, None) == EINVAL
    assert mat(ctypes.byref(vup.VupMM()), 4, dummy, dummy, 0.0, 0.1, 8, dummy, None,
               None) == EWORKSPACE
    # ipsa_fields: levels outside (0, 1], too many, dev without y_ref, quant without levels
    fl = lib.vup_ipsa_fields
    lv = (ctypes.c_double * 17)(*([0.5] * 17))
    bad = (ctypes.c_double * 2)(0.5, 0.0)
    over = (ctypes.c_double * 1)(1.5)
    assert fl(ctypes.byref(mm), 4, dummy, dummy, 2, bad, None, None, dummy, None, None,
              None) == EINVAL
    assert fl(ctypes.byref(mm), 4, dummy, dummy, 1, over, None, None, dummy, None, None,
              None) == EINVAL
    assert fl(ctypes.byref(mm), 4, dummy, dummy, 17, lv, None, None, dummy, None, None,
              None) == EINVAL
    assert fl(ctypes.byref(mm), 4, dummy, None, 1, lv, None, None, None, dummy, None,
              None) == EINVAL
    assert fl(ctypes.byref(mm), 4, dummy, dummy, 0, None, None, None, dummy, None, None,
              None) == EINVAL
    assert fl(ctypes.byref(mm), 4, None, dummy, 1, lv, dummy, None, None, None, None,
              None) == EINVAL
    # marginal: workspace size rule and checks
    assert lib.vup_marginal_workspace_bytes(65536, 256) == 2048 * 256 * 8
    assert lib.vup_marginal_workspace_bytes(0, 256) == 0
    assert lib.vup_marginal_workspace_bytes(10, 0) == 0
    assert lib.vup_marginalize(10, 0, dummy, None, dummy, 1 << 20, dummy, None) == EINVAL
    assert lib.vup_marginalize(-1, 4, dummy, None, dummy, 1 << 20, dummy, None) == EINVAL
    assert lib.vup_marginalize(10, 4, None, None, dummy, 1 << 20, dummy, None) == EINVAL
    need = lib.vup_marginal_workspace_bytes(100, 9)
    assert lib.vup_marginalize(100, 9, dummy, None, dummy, need - 1, dummy, None) == EWORKSPACE
    assert lib.vup_marginalize(100, 9, dummy, None, None, need, dummy, None) == EWORKSPACE
    # the allocation-free marginal: same argument checks, and sizes whose
    # partial sums exceed its 8 MiB array are refused before any launch
    noalloc = lib.vup_marginalize_noalloc
    assert noalloc(-1, 4, dummy, None, dummy, None) == EINVAL
    assert noalloc(10, 0, dummy, None, dummy, None) == EINVAL
    assert noalloc(10, 4, None, None, dummy, None) == EINVAL
    assert noalloc(10, 4, dummy, None, None, None) == EINVAL
    assert noalloc(10, (1 << 20) + 1, dummy, None, dummy, None) == EUNSUPPORTED
    assert b"scratch" in lib.vup_last_error()
    assert lib.vup_marginal_workspace_bytes(1 << 30, 1 << 20) <= 8 << 20


def test_posterior_arguments(lib):
    mm = _fake_mm(lib)
    dummy = ctypes.c_void_p(0x1000)
    d = vup.VupDists()
    d.K, d.ncomp, d.ndim, d.n_sigma = 4, 1, 2, 4.0
    d.mu, d.sigma = 0x1000, 0x2000
    post = lib.vup_posterior
    assert post(ctypes.byref(mm), ctypes.byref(d), -1, dummy, dummy, dummy, dummy, None,
                None) == EINVAL
    assert post(ctypes.byref(mm), ctypes.byref(d), 70000, dummy, dummy, dummy, dummy, None,
                None) == EUNSUPPORTED
    for i in range(4):
        args = [dummy, dummy, dummy, dummy]
        args[i] = None
        assert post(ctypes.byref(mm), ctypes.byref(d), 3, *args, None, None) == EINVAL
    d.ndim = 3
    assert post(ctypes.byref(mm), ctypes.byref(d), 3, dummy, dummy, dummy, dummy, None,
                None) == EINVAL
    assert post(ctypes.byref(vup.VupMM()), ctypes.byref(d), 3, dummy, dummy, dummy, dummy, None,
                None) == EWORKSPACE


def test_separable_arguments(lib):
    mm = _fake_mm(lib)
    dummy = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x100000)
    need = lib.vup_separable_workspace_bytes(ctypes.byref(mm), 20, 20)
    assert need > 0
    s = vup.VupSepDists()
    s.M[0], s.M[1] = 20, 20
    s.n_sigma = 4.0
    s.mu[0], s.mu[1], s.sigma[0], s.sigma[1] = 0x1000, 0x2000, 0x3000, 0x4000
    sep = lib.vup_propagate_separable
    # the contraction's operand format: FP32, BF16 or split BF16 only
    for bad in (3, -1, 7):
        s.precision = bad
        assert sep(ctypes.byref(mm), ctypes.byref(s), ws, need, dummy, None, None) == EINVAL
        assert b"precision" in lib.vup_last_error()
    s.precision = 1
    assert sep(ctypes.byref(mm), ctypes.byref(s), ws, need - 1, dummy, None, None) == EWORKSPACE
    assert sep(ctypes.byref(mm), ctypes.byref(s), ctypes.c_void_p(0x100001), need, dummy, None,
               None) == EWORKSPACE
    s.M[1] = 0
    assert sep(ctypes.byref(mm), ctypes.byref(s), ws, need, dummy, None, None) == EINVAL
    s.M[1] = 20
    s.n_sigma = 0.0
    assert sep(ctypes.byref(mm), ctypes.byref(s), ws, need, dummy, None, None) == EINVAL
    s.n_sigma = 4.0
    assert sep(ctypes.byref(mm), ctypes.byref(s), ws, need, None, None, None) == EINVAL
    mm3 = _fake_mm(lib, n=(4, 4))
    mm3.grid = _grid((4, 4, 4), (0, 0, 0), (1, 1, 1))
    assert sep(ctypes.byref(mm3), ctypes.byref(s), ws, need, dummy, None, None) == EUNSUPPORTED
