"""Learned bandwidth proposal for 2-D samples.

A small network maps 24 summary features of a sample to the Cholesky
coordinates of a bandwidth matrix; it is trained on the GPU (kde_mlp_*
kernels) against LSCV-optimal bandwidths found by the plain search of
``lscv`` on the binned objective, and the plain search stays available as
fallback and as reference (``evaluate``).

Frame: with sample mean m, covariance S = L L' and the normal-scale factor
c_n = n^(-1/3) (d = 2), a bandwidth is written H = c_n L A L' and the network
predicts the Cholesky coordinates of A (log R_11, R_21, log R_22 with
A = R R'). The normal-scale rule is A = I, i.e. all-zero outputs.

Features (24, of the whitened sample Z = (X - m) L^-T): skewness and excess
kurtosis per axis (4), E[z1^2 z2], E[z1 z2^2], E[z1^2 z2^2] - 1 (3), the 7
interior octiles per axis (14), the correlation of X, log(lambda_max /
lambda_min) of S and log10 n (3).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import kde as K
from . import lscv as S

N_FEATURES = 24


def frame(X: np.ndarray):
    """(c_n, L) of H = c_n L A L'."""
    n = X.shape[0]
    Sx = np.cov(X, rowvar=False)
    return n ** (-1.0 / 3.0), np.linalg.cholesky(Sx)


def features(X: np.ndarray) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    m = X.mean(axis=0)
    Sx = np.cov(X, rowvar=False)
    L = np.linalg.cholesky(Sx)
    Z = np.linalg.solve(L, (X - m).T).T
    z1, z2 = Z[:, 0], Z[:, 1]
    f = [np.mean(z1 ** 3), np.mean(z2 ** 3), np.mean(z1 ** 4) - 3.0, np.mean(z2 ** 4) - 3.0,
         np.mean(z1 ** 2 * z2), np.mean(z1 * z2 ** 2), np.mean(z1 ** 2 * z2 ** 2) - 1.0]
    q = np.arange(1, 8) / 8.0
    f += list(np.quantile(z1, q)) + list(np.quantile(z2, q))
    ev = np.linalg.eigvalsh(Sx)
    f += [Sx[0, 1] / math.sqrt(Sx[0, 0] * Sx[1, 1]), math.log(ev[1] / ev[0]), math.log10(n)]
    return np.array(f)


def to_target(H, X) -> np.ndarray:
    c, L = frame(X)
    Li = np.linalg.inv(L)
    return S.to_theta(Li @ np.asarray(H) @ Li.T / c)


def from_target(t, X) -> np.ndarray:
    c, L = frame(X)
    H = c * L @ S.from_theta(np.asarray(t, dtype=np.float64), 2) @ L.T
    return 0.5 * (H + H.T)


def grid_for(X, M: int = 256):
    """Grid box: the data range widened by 3 marginal normal-scale bandwidth SDs."""
    c, L = frame(X)
    H = c * L @ L.T
    return K.grid_tuple(K.kde_grid_from_data(X, 0.5 * (H + H.T), M, 3.0))


def mixtures(count: int, seed: int, n_range=(1e3, 1e5)):
    """2-D normal mixtures with 2-5 components (means in [-4, 4]^2, random SPD
    covariances with eigenvalue ratio up to 10, random weights), n log-uniform."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(rng.integers(2, 6))
        means = rng.uniform(-4, 4, size=(k, 2))
        covs = []
        for _ in range(k):
            Q, _ = np.linalg.qr(rng.normal(size=(2, 2)))
            lam = rng.uniform(0.1, 0.5) * np.array([1.0, rng.uniform(1.0, 10.0)])
            covs.append((Q * lam) @ Q.T)
        w = rng.dirichlet(np.ones(k))
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        comp = rng.choice(k, size=n, p=w)
        Z = rng.normal(size=(n, 2))
        X = np.empty((n, 2))
        for c in range(k):
            idx = comp == c
            X[idx] = means[c] + Z[idx] @ np.linalg.cholesky(covs[c]).T
        out.append(X)
    return out


def label(samples, M: int = 256, iters: int = 60, chunk: int = 256, device="cuda:0", **opts):
    """LSCV-optimal H of every sample by the lockstep batched search, started at normal scale."""
    out = []
    t0 = time.perf_counter()
    evals = 0
    for s in range(0, len(samples), chunk):
        part = samples[s:s + chunk]
        Xs = [torch.as_tensor(X, device=device) for X in part]
        grids = [grid_for(X, M) for X in part]
        res = S.lscv_search_batch(Xs, grids, iters=iters, **opts)
        out += [r["H"] for r in res]
        evals += sum(r["evals"] for r in res)
    torch.cuda.synchronize()
    return out, {"seconds": time.perf_counter() - t0, "evals": evals}


class Proposal:
    """Trained network plus the feature standardisation it was trained with."""

    def __init__(self, net: K.MlpNet, mu: np.ndarray, sd: np.ndarray):
        self.net, self.mu, self.sd = net, mu, sd

    def inputs(self, F: np.ndarray) -> torch.Tensor:
        return torch.as_tensor(((F - self.mu) / self.sd).astype(np.float32), device=self.net.device).contiguous()

    def predict(self, samples, F=None, M: int | None = 256):
        """Proposed H per sample; with a grid size M, moved into the search
        domain of that sample's grid (eigenvalues floored at one bin width^2)."""
        F = np.stack([features(X) for X in samples]) if F is None else F
        Y = self.net.forward(self.inputs(F)).cpu().numpy().astype(np.float64)
        Hs = [from_target(y, X) for y, X in zip(Y, samples)]
        if M is not None:
            Hs = [S.project(H, grid_for(X, M)) for H, X in zip(Hs, samples)]
        return Hs


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, small biases, padded rows / columns zero; output layer scaled down."""
    info = K.mlp_query()
    rng = np.random.default_rng(seed)
    shapes = [(32, 128), (128, 128), (128, 128), (128, 16)]
    parts = []
    for i, (k, n) in enumerate(shapes):
        W = rng.normal(size=(k, n)) * math.sqrt(2.0 / k) * (0.1 if i == 3 else 1.0)
        b = np.zeros(n)
        if i == 0:
            W[N_FEATURES:, :] = 0
        if i == 3:
            W[:, 3:] = 0
        parts += [W.ravel(), b]
    p = np.concatenate(parts)
    assert p.size == info["n_params"]
    return p


def train(F: np.ndarray, T: np.ndarray, epochs: int = 200, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          device="cuda:0"):
    """Adam on the mean squared error of the targets; returns (Proposal, losses per epoch)."""
    mu, sd = F.mean(axis=0), F.std(axis=0) + 1e-9
    net = K.MlpNet(init_params(seed), device=device)
    P = Proposal(net, mu, sd)
    Xd = P.inputs(F)
    Td = torch.as_tensor(T.astype(np.float32), device=device)
    rng = np.random.default_rng(seed)
    loss = torch.empty(1, dtype=torch.float32, device=device)
    losses = []
    step = 0
    n = F.shape[0]
    for _ in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device=device)
        Xp, Tp = Xd[perm].contiguous(), Td[perm].contiguous()
        acc = 0.0
        nb = 0
        for b in range(0, n - batch + 1, batch):
            step += 1
            net.train_step(Xp[b:b + batch], Tp[b:b + batch], lr, step, loss)
            acc += loss
            nb += 1
        losses.append(float((acc / nb).cpu()[0]) if nb else float("nan"))
    return P, losses


def lscv_at(samples, Hs, M: int = 256, **opts) -> np.ndarray:
    """Binned LSCV of each sample at its H (one batched evaluation)."""
    probs = []
    for X, H in zip(samples, Hs):
        Xd = torch.as_tensor(X, device="cuda:0")
        g = grid_for(X, M)
        C, _ = K.kde_bin(Xd, g)
        probs.append((C, X.shape[0], H, g))
    return S.lscv_values_batch(probs, **opts)
