"""vup_marginalize_noalloc (the marginal over locations for callers that
cannot allocate) against the workspace form vup_marginalize, both through the
C ABI: two calls in a row, the second with a smaller input, then the call
whose partial sums need the whole scratch array, and the host-side rejection
of a size beyond it. The two entry points run the same kernels with the same
chunking, so their results are compared bit for bit; both are also checked
against a plain FP64 sum."""
import ctypes
import sys

import numpy as np
import pytest
import torch

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


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _workspace_form(vup, A, rho):
    lib = vup.lib()
    K, n = A.shape
    need = lib.vup_marginal_workspace_bytes(K, n)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=DEV)
    out = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.vup_marginalize(K, n, _p(A), _p(rho), _p(ws), ws.numel(), _p(out), s) == 0
    return out


def _noalloc_form(vup, A, rho):
    lib = vup.lib()
    K, n = A.shape
    out = torch.full((n,), float("nan"), dtype=torch.float64, device=DEV)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.vup_marginalize_noalloc(K, n, _p(A), _p(rho), _p(out), s)
    assert rc == 0, lib.vup_last_error()
    return out


@pytest.mark.parametrize("K, n, with_rho", [(5000, 300, True), (700, 64, False),
                                            (65536, 768, True), (0, 5, False)])
def test_noalloc_marginal_matches_workspace_form(vup, K, n, with_rho):
    _say(f"[noalloc marginal] K={K} n={n} rho={with_rho} "
         f"partial sums {vup.lib().vup_marginal_workspace_bytes(K, n)} bytes")
    rng = np.random.default_rng(7000 + K + n)
    A = torch.from_numpy(rng.random((K, n), dtype=np.float32)).to(DEV)
    rho = (torch.from_numpy(rng.dirichlet(np.ones(K)) if K else np.zeros(0)).to(DEV)
           if with_rho else None)
    want = _workspace_form(vup, A, rho)
    got = _noalloc_form(vup, A, rho)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    w = rho.cpu().numpy() if with_rho else np.full(K, 1.0 / max(K, 1))
    ref = (w[:, None] * A.cpu().numpy().astype(np.float64)).sum(axis=0)
    assert np.allclose(got.cpu().numpy(), ref, rtol=1e-12, atol=1e-15)


def test_noalloc_marginal_rejects_beyond_scratch(vup):
    lib = vup.lib()
    A = torch.zeros((2, 8), dtype=torch.float32, device=DEV)
    out = torch.full((8,), 7.0, dtype=torch.float64, device=DEV)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # n = 2^20 + 1 needs more than the 8 MiB array (the pointer is never read:
    # the call fails on the host before anything is enqueued)
    assert lib.vup_marginalize_noalloc(2, (1 << 20) + 1, _p(A), None, _p(out), s) == -4
    assert b"scratch" in lib.vup_last_error()
    torch.cuda.synchronize()
    assert (out == 7.0).all()
