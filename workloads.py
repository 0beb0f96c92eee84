"""Seeded synthetic inputs for vectorized uncertainty propagation (VUP) runs.

This module only *describes* problems: a grid (domain and cell counts), a model
by name, a bin count, and the parameters (means, standard deviations, mixture
weights) of the K input distributions. It contains none of the method's
arithmetic: no densities, windows, bins or moments are computed here. Both the
HIP path and the CPU oracle receive exactly these arrays.

Workloads (all analytic and synthetic; the paper's Sec. 4.1 and Sec. 5.3 runs
also use analytic models on uniform grids, so no dataset is involved):

* ``grid64``   2-D 64x64 on [-3,3]^2, f = sin x + 0.5 cos 2y + xy/4, B = 64,
               K = 256 isotropic Gaussians, means on the 16x16 midpoint
               subgrid, sigma = 0.25.
* ``grid1024`` 2-D 1024x1024 on [-3,3]^2, same f, B = 256, K = 65536 means on
               the 256x256 midpoint subgrid, sigma_k ~ U[0.05, 0.5]
               (isotropic, seed 11246002).
* ``grid128_3d`` 3-D 128^3 on [-2,2]^3, f = exp(-0.1 z) sin x cos y + 0.1 xyz,
               B = 512, K = 32768 diagonal Gaussians, mu ~ U[-1.5,1.5]^3,
               per-axis sigma ~ U[0.05, 0.3] (seed 11246003).
* ``grid48_4d`` 4-D 48^4 on [-2,2]^4, f = sum_j sin(x_j) x_{j+1 mod 4}
               + 0.05 (sum_j x_j)^2, B = 1024, K = 16384 two-component
               mixtures, weights Dirichlet(1,1), mu ~ U[-1.5,1.5]^4,
               isotropic sigma per component ~ U[0.05, 0.25] (seed 11246005).

* ``ipsa_example(sigma_l)`` the IPSA example of Sec. 5.3: 2-D 1000 x 1000
               grid over (x, alpha) in [-5,5] x [-1,1] (N = 10^6), model
               x^2 + 5 sin 3x + alpha, B = 1000, K = 1000 measurement
               locations l on the 1000-cell midpoints of [-5,5], pdf centred
               at (l, 0) with sigma = (sigma_l, 0.25), truncated at the domain
               boundary (8-sigma windows, so the boundary is the only cut that
               matters). The paper runs sigma_l in {0.05, 0.25, 0.5, 1, 3}; it
               does not state the domain, which is a reading (x spans the
               locations, alpha spans 4 sigma_alpha).

* ``timing_study(L)`` the timing experiment of Sec. 4.1: 2-D 1000 x 1000 grid
               over (x, alpha) in [-3,3]^2 (N = 10^6), model
               1.1 sin x + 7 sin^2 alpha, L Gaussians with sigma = (1, 1)
               differing only in mu_x (L points on the midpoint subgrid of
               [-2,2], mu_alpha = 0), untruncated (windows span the grid),
               B = 1000. The paper does not state the domain, sigma or the
               bin count; these are readings.

Means "on an M x M subgrid" are the subgrid cell midpoints
lo + (m + 1/2)(hi - lo)/M on each axis, with k = m0 * M + m1.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

SEED_GRID1024 = 11246002
SEED_GRID128_3D = 11246003
SEED_FD_SUBSET = 11246004
SEED_GRID48_4D = 11246005

# model names understood by both the library binding and the oracle wrapper
MODELS = ("linear", "sincos2", "damped3", "ring4", "timing2", "ipsa2")


@dataclasses.dataclass
class Workload:
    name: str
    ndim: int
    n: tuple            # cells per axis, axis 0 slowest in memory
    lo: tuple           # domain lower edge per axis
    hi: tuple           # domain upper edge per axis
    model: str          # one of MODELS
    theta: tuple        # model parameters (only "linear" uses them)
    B: int              # number of output bins
    mu: np.ndarray      # [K][C][d] float64
    sigma: np.ndarray   # [K][C][d] float64
    weight: Optional[np.ndarray]  # [K][C] float64, None when C == 1
    n_sigma: float = 4.0

    @property
    def K(self) -> int:
        return int(self.mu.shape[0])

    @property
    def C(self) -> int:
        return int(self.mu.shape[1])

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    def subset(self, ks) -> "Workload":
        """Same grid/model/bins, only the distributions with indices ``ks``."""
        ks = np.asarray(ks, dtype=np.int64)
        return dataclasses.replace(
            self, name=f"{self.name}[subset {len(ks)}]",
            mu=np.ascontiguousarray(self.mu[ks]),
            sigma=np.ascontiguousarray(self.sigma[ks]),
            weight=None if self.weight is None else np.ascontiguousarray(self.weight[ks]))


def subgrid_midpoints(lo: float, hi: float, M: int) -> np.ndarray:
    """Midpoints of an M-cell subdivision of [lo, hi]."""
    return lo + (np.arange(M, dtype=np.float64) + 0.5) * ((hi - lo) / M)


def _subgrid_means_2d(lo, hi, M):
    m = subgrid_midpoints(lo, hi, M)
    mu = np.empty((M * M, 1, 2), dtype=np.float64)
    mu[:, 0, 0] = np.repeat(m, M)
    mu[:, 0, 1] = np.tile(m, M)
    return mu


def grid64() -> Workload:
    mu = _subgrid_means_2d(-3.0, 3.0, 16)
    sigma = np.full_like(mu, 0.25)
    return Workload("grid64", 2, (64, 64), (-3.0, -3.0), (3.0, 3.0), "sincos2", (),
                    64, mu, sigma, None)


def grid1024(seed: int = SEED_GRID1024) -> Workload:
    mu = _subgrid_means_2d(-3.0, 3.0, 256)
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.uniform(0.05, 0.5, size=mu.shape[0])
    sigma = np.repeat(s[:, None, None], 2, axis=2)
    return Workload("grid1024", 2, (1024, 1024), (-3.0, -3.0), (3.0, 3.0), "sincos2", (),
                    256, mu, np.ascontiguousarray(sigma), None)


def grid128_3d(seed: int = SEED_GRID128_3D) -> Workload:
    K = 32768
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = rng.uniform(-1.5, 1.5, size=(K, 1, 3))
    sigma = rng.uniform(0.05, 0.3, size=(K, 1, 3))
    return Workload("grid128_3d", 3, (128, 128, 128), (-2.0,) * 3, (2.0,) * 3, "damped3", (),
                    512, mu, sigma, None)


def grid48_4d(seed: int = SEED_GRID48_4D) -> Workload:
    K = 16384
    rng = np.random.Generator(np.random.PCG64(seed))
    weight = rng.dirichlet([1.0, 1.0], size=K)
    mu = rng.uniform(-1.5, 1.5, size=(K, 2, 4))
    s = rng.uniform(0.05, 0.25, size=(K, 2))
    sigma = np.repeat(s[:, :, None], 4, axis=2)
    return Workload("grid48_4d", 4, (48,) * 4, (-2.0,) * 4, (2.0,) * 4, "ring4", (),
                    1024, mu, np.ascontiguousarray(sigma), np.ascontiguousarray(weight))


def fd_subset(K: int, count: int = 64, seed: int = SEED_FD_SUBSET) -> np.ndarray:
    """Seeded subset of distribution indices used for finite-difference checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(K, size=min(count, K), replace=False))


def sample_indices(K: int, count: int, seed: int) -> np.ndarray:
    """Seeded sorted sample of distribution indices (parity sampling, CPU baseline)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(K, size=min(count, K), replace=False))


def random_workload(name: str, n, lo, hi, model: str, B: int, K: int, C: int,
                    sigma_range, seed: int, theta=(), mu_margin: float = 0.0,
                    isotropic: bool = False) -> Workload:
    """Generic seeded workload: means uniform in the domain shrunk by ``mu_margin``
    per side, sigma uniform in ``sigma_range``; mixture weights Dirichlet(1,..,1)."""
    d = len(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    lo_a = np.asarray(lo, dtype=np.float64)
    hi_a = np.asarray(hi, dtype=np.float64)
    mu = rng.uniform(lo_a + mu_margin, hi_a - mu_margin, size=(K, C, d))
    if isotropic:
        s = rng.uniform(sigma_range[0], sigma_range[1], size=(K, C))
        sigma = np.repeat(s[:, :, None], d, axis=2)
    else:
        sigma = rng.uniform(sigma_range[0], sigma_range[1], size=(K, C, d))
    weight = rng.dirichlet(np.ones(C), size=K) if C > 1 else None
    return Workload(name, d, tuple(int(x) for x in n), tuple(float(x) for x in lo),
                    tuple(float(x) for x in hi), model, tuple(theta), B,
                    np.ascontiguousarray(mu), np.ascontiguousarray(sigma),
                    None if weight is None else np.ascontiguousarray(weight))


def narrow_workload(name: str, n, lo, hi, model: str, B: int, K: int, seed: int,
                    narrow_sets) -> Workload:
    """Pdfs far narrower than a cell along some axes. Distribution k is narrow
    along the axes of ``narrow_sets[k % len(narrow_sets)]``: there sigma is
    1/200 to 1/80 of a cell and the mean sits 0.1 to 0.45 cells from the
    centre of a cell, so its truncation window is the one cell holding the
    mean, whose centre is t* = 14 .. tmax sigma away (tmax 36, 25, 20 for one,
    two, three narrow axes: each such factor, e^(-t*^2/2), lies below FP32's
    range and the product of all of them inside FP64's). The other axes take
    sigma ~ U[0.05, 0.5] and a mean at least 0.5 inside the domain."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = len(n)
    h = [(hi[i] - lo[i]) / n[i] for i in range(d)]
    mu = np.empty((K, 1, d))
    sigma = np.empty((K, 1, d))
    for k in range(K):
        narrow = narrow_sets[k % len(narrow_sets)]
        tmax = {1: 36.0, 2: 25.0}.get(len(narrow), 20.0)
        for ax in range(d):
            if ax in narrow:
                while True:
                    c = int(rng.integers(1, n[ax] - 1))
                    u = rng.uniform(0.1, 0.45) * (1.0 if rng.uniform() < 0.5 else -1.0)
                    v = rng.uniform(1.0 / 200.0, 1.0 / 80.0)
                    if 14.0 <= abs(u) / v <= tmax:
                        break
                mu[k, 0, ax] = lo[ax] + (c + 0.5 + u) * h[ax]
                sigma[k, 0, ax] = v * h[ax]
            else:
                mu[k, 0, ax] = rng.uniform(lo[ax] + 0.5, hi[ax] - 0.5)
                sigma[k, 0, ax] = rng.uniform(0.05, 0.5)
    return Workload(name, d, tuple(int(x) for x in n), tuple(float(x) for x in lo),
                    tuple(float(x) for x in hi), model, (), B, mu, sigma, None)


IPSA_EXAMPLE_SIGMAS = (0.05, 0.25, 0.5, 1.0, 3.0)


def ipsa_example(sigma_l: float = 0.25) -> Workload:
    K = 1000
    l = subgrid_midpoints(-5.0, 5.0, K)
    mu = np.zeros((K, 1, 2), dtype=np.float64)
    mu[:, 0, 0] = l
    sigma = np.empty((K, 1, 2), dtype=np.float64)
    sigma[:, 0, 0] = sigma_l
    sigma[:, 0, 1] = 0.25
    return Workload(f"ipsa_example[sigma_l={sigma_l}]", 2, (1000, 1000), (-5.0, -1.0),
                    (5.0, 1.0), "ipsa2", (), 1000, mu, sigma, None, n_sigma=8.0)


def timing_study(L: int) -> Workload:
    mu = np.zeros((L, 1, 2), dtype=np.float64)
    mu[:, 0, 0] = subgrid_midpoints(-2.0, 2.0, L)
    sigma = np.ones((L, 1, 2), dtype=np.float64)
    return Workload(f"timing_study[L={L}]", 2, (1000, 1000), (-3.0, -3.0), (3.0, 3.0), "timing2",
                    (), 1000, mu, sigma, None, n_sigma=1.0e6)


CONFIGS = {
    "grid64": grid64,
    "grid1024": grid1024,
    "grid128_3d": grid128_3d,
    "grid48_4d": grid48_4d,
}
