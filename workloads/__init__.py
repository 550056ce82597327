"""Seeded synthetic inputs for the binned KDE path.

This module is shared by the CPU oracle, the GPU tests and the benchmark. It
only draws samples and picks the problem description (H, grid box); it holds
none of the estimator's arithmetic (no binning, no kernel weights, no
convolution). Everything is NumPy FP64 on the host; the GPU path receives the
arrays produced here and never generates data itself.

Workloads (named by what they are):

* ``mix2d_small``   d=2, n=1,000, equal-weight 3-component normal mixture with
  means (-1,0), (1,0.5), (0,-1.5), unit marginal variances and correlations
  -0.6, 0.7, 0; H = [[0.09, 0.06], [0.06, 0.08]]; 64x64 grid.
* ``mix2d_512``     d=2, n=1,000,000, 5-component mixture with means in
  [-4,4]^2 and random SPD covariances (random rotation, smallest eigenvalue in
  [0.1,0.5], eigenvalue ratio in [1,10]); H is the normal-scale rule with the
  correlation fixed at 0.8; 512x512 grid.
* ``mix3d_128``     d=3, n=1,000,000, 4-component mixture with means in
  [-4,4]^3, random rotations, eigenvalue ratio up to 20; H is the full
  normal-scale matrix; 128x128x128 grid.
* ``batch2d``       many independent 2-D problems (256 by default): each with
  n log-uniform in [1e3, 1e6] drawn from a 2-5 component mixture, grid side
  drawn from {64, 128, 256, 512}, and H a random SPD matrix (random rotation,
  eigenvalue ratio up to 20) whose determinant matches the normal-scale
  matrix of its sample.

The grid box of every workload is the data range widened by three marginal
bandwidth standard deviations sqrt(H_kk) on each side.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_BASE = 150802766


@dataclass
class Workload:
    name: str
    X: np.ndarray          # (n, d) float64, row-major
    H: np.ndarray          # (d, d) float64, symmetric positive definite
    lo: np.ndarray         # (d,) float64, first grid node per axis
    hi: np.ndarray         # (d,) float64, last grid node per axis
    M: tuple               # grid nodes per axis

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])


def random_rotation(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix (QR of a Gaussian matrix, sign-fixed)."""
    A = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(A)
    return Q * np.sign(np.diag(R))


def random_spd(rng: np.random.Generator, d: int, lam_min=(0.1, 0.5), ratio=(1.0, 10.0)) -> np.ndarray:
    """Random SPD matrix: random rotation, smallest eigenvalue and eigenvalue ratio drawn uniformly."""
    lmin = rng.uniform(*lam_min)
    r = rng.uniform(*ratio)
    if d == 1:
        lams = np.array([lmin])
    else:
        inner = rng.uniform(1.0, r, size=d - 2)
        lams = lmin * np.concatenate(([1.0], inner, [r]))
    Q = random_rotation(rng, d)
    S = (Q * lams) @ Q.T
    return 0.5 * (S + S.T)


def sample_mixture(rng: np.random.Generator, n: int, means, covs) -> np.ndarray:
    """n draws from an equal-weight normal mixture, returned as (n, d) float64."""
    means = np.asarray(means, dtype=np.float64)
    k, d = means.shape
    comp = rng.integers(0, k, size=n)
    Z = rng.standard_normal((n, d))
    X = np.empty((n, d), dtype=np.float64)
    for c in range(k):
        idx = np.nonzero(comp == c)[0]
        Lc = np.linalg.cholesky(np.asarray(covs[c], dtype=np.float64))
        X[idx] = means[c] + Z[idx] @ Lc.T
    return X


def grid_box(X: np.ndarray, H: np.ndarray, nsd: float = 3.0):
    """Data range widened by ``nsd`` marginal bandwidth SDs sqrt(H_kk) per side."""
    s = np.sqrt(np.diag(H))
    return X.min(axis=0) - nsd * s, X.max(axis=0) + nsd * s


def normal_scale_H(X: np.ndarray, corr: float | None = None) -> np.ndarray:
    """Normal-scale bandwidth (4/(d+2))^(2/(d+4)) n^(-2/(d+4)) S.

    With ``corr`` given, S is rebuilt from the sample standard deviations and
    that fixed correlation (used for the 2-D workload whose H has a prescribed
    correlation); otherwise S is the full sample covariance.
    """
    n, d = X.shape
    S = np.atleast_2d(np.cov(X, rowvar=False))
    if corr is not None:
        sd = np.sqrt(np.diag(S))
        Rm = np.full((d, d), corr)
        np.fill_diagonal(Rm, 1.0)
        S = Rm * np.outer(sd, sd)
    c = (4.0 / (d + 2.0)) ** (2.0 / (d + 4.0)) * n ** (-2.0 / (d + 4.0))
    H = c * S
    return 0.5 * (H + H.T)


def mix2d_small(seed_offset: int = 0) -> Workload:
    rng = np.random.default_rng(SEED_BASE + 1 + seed_offset)
    means = [(-1.0, 0.0), (1.0, 0.5), (0.0, -1.5)]
    covs = [np.array([[1.0, r], [r, 1.0]]) for r in (-0.6, 0.7, 0.0)]
    X = sample_mixture(rng, 1000, means, covs)
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    lo, hi = grid_box(X, H)
    return Workload("mix2d_small", X, H, lo, hi, (64, 64))


def mix2d_512(n: int = 1_000_000, M: int = 512, seed_offset: int = 0) -> Workload:
    rng = np.random.default_rng(SEED_BASE + 2 + seed_offset)
    k = 5
    means = rng.uniform(-4.0, 4.0, size=(k, 2))
    covs = [random_spd(rng, 2, ratio=(1.0, 10.0)) for _ in range(k)]
    X = sample_mixture(rng, n, means, covs)
    H = normal_scale_H(X, corr=0.8)
    lo, hi = grid_box(X, H)
    return Workload("mix2d_512", X, H, lo, hi, (M, M))


def mix3d_128(n: int = 1_000_000, M: int = 128, seed_offset: int = 0) -> Workload:
    rng = np.random.default_rng(SEED_BASE + 3 + seed_offset)
    k = 4
    means = rng.uniform(-4.0, 4.0, size=(k, 3))
    covs = [random_spd(rng, 3, ratio=(1.0, 20.0)) for _ in range(k)]
    X = sample_mixture(rng, n, means, covs)
    H = normal_scale_H(X)
    lo, hi = grid_box(X, H)
    return Workload("mix3d_128", X, H, lo, hi, (M, M, M))


def mix4d_48(n: int = 1_000_000, M: int = 48, seed_offset: int = 0) -> Workload:
    rng = np.random.default_rng(SEED_BASE + 5 + seed_offset)
    k = 4
    means = rng.uniform(-4.0, 4.0, size=(k, 4))
    covs = [random_spd(rng, 4, ratio=(1.0, 20.0)) for _ in range(k)]
    X = sample_mixture(rng, n, means, covs)
    H = normal_scale_H(X)
    lo, hi = grid_box(X, H)
    return Workload("mix4d_48", X, H, lo, hi, (M, M, M, M))


def batch2d(count: int = 256, seed_offset: int = 0, n_range=(1e3, 1e6), sides=(64, 128, 256, 512),
            ratio_max: float = 20.0) -> list:
    rng = np.random.default_rng(SEED_BASE + 4 + seed_offset)
    out = []
    for i in range(count):
        k = int(rng.integers(2, 6))
        means = rng.uniform(-4.0, 4.0, size=(k, 2))
        covs = [random_spd(rng, 2, ratio=(1.0, 10.0)) for _ in range(k)]
        n = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        M = int(rng.choice(np.asarray(sides)))
        X = sample_mixture(rng, n, means, covs)
        g = np.sqrt(np.linalg.det(normal_scale_H(X)))       # geometric mean of its eigenvalues
        r = rng.uniform(1.0, ratio_max)
        Q = random_rotation(rng, 2)
        lams = g * np.array([1.0 / np.sqrt(r), np.sqrt(r)])
        H = (Q * lams) @ Q.T
        H = 0.5 * (H + H.T)
        lo, hi = grid_box(X, H)
        out.append(Workload(f"batch2d_{i}", X, H, lo, hi, (M, M)))
    return out


WORKLOADS = {
    "mix2d_small": mix2d_small,
    "mix2d_512": mix2d_512,
    "mix3d_128": mix3d_128,
    "mix4d_48": mix4d_48,
}


def small_mixture(seed: int, d: int, n: int, M, k: int = 3, ratio=(1.0, 10.0),
                  H_scale: float = 1.0, diagonal_H: bool = False) -> Workload:
    """Reduced-size mixture of the same structure, for parity cases of any shape.

    ``M`` may be an int (same on every axis) or a per-axis tuple; H is the
    normal-scale matrix times ``H_scale`` (its diagonal only when requested).
    """
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    means = rng.uniform(-3.0, 3.0, size=(k, d))
    covs = [random_spd(rng, d, ratio=ratio) for _ in range(k)]
    X = sample_mixture(rng, n, means, covs)
    H = H_scale * normal_scale_H(X) if n > d else H_scale * np.eye(d) * 0.1
    if diagonal_H:
        H = np.diag(np.diag(H))
    lo, hi = grid_box(X, H)
    if np.isscalar(M):
        M = (int(M),) * d
    return Workload(f"mix{d}d_seed{seed}", X, H, lo, hi, tuple(int(m) for m in M))
