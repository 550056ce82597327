"""Plain least-squares cross-validation (LSCV) bandwidth search.

The objective is evaluated on the GPU (``kde_lscv`` for one problem,
``kde_lscv_batch_create`` for many, each combining its terms on the device);
this module holds only the host-side search: a Nelder-Mead simplex over the Cholesky
coordinates of H, started from the normal-scale matrix.

Coordinates: H = R R' with R lower triangular, theta = (log R_11, R_21,
log R_22, R_31, R_32, log R_33) (row by row), so every theta is a valid SPD H.

Search domain: the binned objective treats samples that share a bin as
coincident, so for bandwidths much below the bin width its second term grows
like phi_H(0) and the objective runs off to minus infinity. The search
therefore only admits H whose smallest eigenvalue is at least
(min_bins * max_k delta_k)^2 (one bin width by default) and whose 2H still
fits the padded-length limit; other points evaluate to +inf.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import kde as K


def to_theta(H) -> np.ndarray:
    R = np.linalg.cholesky(np.asarray(H, dtype=np.float64))
    d = R.shape[0]
    return np.array([math.log(R[i, i]) if i == j else R[i, j] for i in range(d) for j in range(i + 1)])


def from_theta(theta, d: int) -> np.ndarray:
    """H = R R' from the Cholesky coordinates, summed in plain double arithmetic
    (exactly symmetric; a search evaluates this once per point, so no array
    machinery)."""
    R = [[0.0] * d for _ in range(d)]
    k = 0
    for i in range(d):
        for j in range(i + 1):
            R[i][j] = math.exp(theta[k]) if i == j else float(theta[k])
            k += 1
    H = np.empty((d, d))
    for i in range(d):
        for j in range(i + 1):
            s = 0.0
            for m in range(j + 1):
                s += R[i][m] * R[j][m]
            H[i, j] = H[j, i] = s
    return H


def normal_scale(X: np.ndarray) -> np.ndarray:
    """(4 / (d + 2))^(2 / (d + 4)) n^(-2 / (d + 4)) times the sample covariance."""
    n, d = X.shape
    S = np.atleast_2d(np.cov(X, rowvar=False))
    return (4.0 / (d + 2.0)) ** (2.0 / (d + 4.0)) * n ** (-2.0 / (d + 4.0)) * S


def nelder_mead(x0, step: float = 0.25, iters: int = 100, tol: float = 1e-7):
    """Nelder-Mead as a generator: yields points, receives their values; returns (x, f(x), evals)."""
    x0 = np.asarray(x0, dtype=np.float64)
    m = x0.size
    pts = [x0.copy()] + [x0 + step * e for e in np.eye(m)]
    vals = []
    for p in pts:
        vals.append((yield p))
    evals = m + 1
    for _ in range(iters):
        idx = sorted(range(m + 1), key=lambda i: vals[i])
        pts = [pts[i] for i in idx]
        vals = [vals[i] for i in idx]
        if abs(vals[-1] - vals[0]) <= tol * abs(vals[0]):
            break
        c = pts[0]                      # centroid of all but the worst, summed in order
        for q in pts[1:-1]:
            c = c + q
        c = c / m
        worst = pts[-1]
        xr = 2.0 * c - worst
        fr = yield xr
        evals += 1
        if fr < vals[0]:
            xe = 3.0 * c - 2.0 * worst
            fe = yield xe
            evals += 1
            pts[-1], vals[-1] = (xe, fe) if fe < fr else (xr, fr)
        elif fr < vals[-2]:
            pts[-1], vals[-1] = xr, fr
        else:
            xc = 0.5 * (c + worst)
            fc = yield xc
            evals += 1
            if fc < vals[-1]:
                pts[-1], vals[-1] = xc, fc
            else:
                for i in range(1, m + 1):
                    pts[i] = 0.5 * (pts[0] + pts[i])
                    vals[i] = yield pts[i]
                    evals += 1
    i = int(np.argmin(vals))
    return pts[i], vals[i], evals


def project(H, grid, min_bins: float = 1.0, margin: float = 1.01) -> np.ndarray:
    """The nearest H (same eigenvectors) whose eigenvalues respect the search domain's floor."""
    g = K._grid(grid)
    dmax = max((g.hi[k] - g.lo[k]) / (g.M[k] - 1) for k in range(g.d))
    lam, V = np.linalg.eigh(np.asarray(H, dtype=np.float64))
    lam = np.maximum(lam, margin * (min_bins * dmax) ** 2)
    Hp = (V * lam) @ V.T
    return 0.5 * (Hp + Hp.T)


def _min_eig(H: np.ndarray) -> float:
    if H.shape == (1, 1):
        return float(H[0, 0])
    if H.shape == (2, 2):   # closed form; LAPACK's call overhead dominates at this size
        a, b, c = float(H[0, 0]), 0.5 * (float(H[0, 1]) + float(H[1, 0])), float(H[1, 1])
        return 0.5 * (a + c) - math.hypot(0.5 * (a - c), b)
    return float(np.linalg.eigvalsh(H)[0])


def _admissible_phi0(H, n, grid, opts, min_bins: float = 1.0):
    """(admissible, phi_H(0)) from one plan query: admissible H have smallest eigenvalue
    >= (min_bins max delta)^2 and plan (with 2H) within the transform limits; phi_H(0) is
    formed as the library forms it (n k_0), so host and device combine identically."""
    g = K._grid(grid)
    dmax = max((g.hi[k] - g.lo[k]) / (g.M[k] - 1) for k in range(g.d))
    if _min_eig(np.asarray(H, dtype=np.float64)) < (min_bins * dmax) ** 2:
        return False, math.nan
    try:
        p = K.kde_plan_query(H, n, grid, **{k: v for k, v in opts.items() if k in K._PLAN_OPTS})
    except K.KdeError:
        return False, math.nan
    return p["lscv_ws_bytes"] > 0, p["norm"] * n


def _admissible(H, n, grid, opts, min_bins: float = 1.0) -> bool:
    return _admissible_phi0(H, n, grid, opts, min_bins)[0]


def lscv_search(X: torch.Tensor, grid, H0=None, iters: int = 100, step: float = 0.25, min_bins: float = 1.0,
                **opts) -> dict:
    """Minimise the binned LSCV objective for one sample (X: (n, d) float64 CUDA tensor)."""
    g = K._grid(grid)
    n, d = X.shape
    counts, _ = K.kde_bin(X, g, **{k: v for k, v in opts.items() if k in ("Q", "tile")})
    Xh = X.cpu().numpy()
    H0 = normal_scale(Xh) if H0 is None else np.asarray(H0, dtype=np.float64)
    out = torch.empty(3, dtype=torch.float64, device=X.device)
    plan = K.kde_plan_query(H0, n, g, **{k: v for k, v in opts.items() if k in K._PLAN_OPTS})
    ws = torch.empty(max(plan["lscv_ws_bytes"], 1), dtype=torch.uint8, device=X.device)
    gen = nelder_mead(to_theta(H0), step=step, iters=iters)
    theta = next(gen)
    evals = 0
    try:
        while True:
            H = from_theta(theta, d)
            if not _admissible(H, n, g, opts, min_bins):
                val = math.inf
            else:
                need = K.kde_plan_query(H, n, g, **{k: v for k, v in opts.items() if k in K._PLAN_OPTS})
                if need["lscv_ws_bytes"] > ws.numel():
                    ws = torch.empty(need["lscv_ws_bytes"], dtype=torch.uint8, device=X.device)
                K.kde_lscv(counts, n, H, g, out=out, ws=ws, **opts)
                val = float(out[0].item())
            evals += 1
            theta = gen.send(val)
    except StopIteration as stop:
        x, v, _ = stop.value
    return {"H": from_theta(x, d), "lscv": v, "evals": evals, "H0": H0}


def lscv_values_batch(problems, min_bins: float = 1.0, **opts) -> np.ndarray:
    """LSCV(H) of many (counts, n, H, grid) problems through one batched pipeline
    (kde_lscv_batch_create: two convolutions and dots per problem, combined on
    the device); inadmissible H give +inf."""
    items, idx = [], []
    out = np.full(len(problems), math.inf)
    for p, (C, n, H, grid) in enumerate(problems):
        H = np.asarray(H, dtype=np.float64)
        if not _admissible(H, n, grid, opts, min_bins):
            continue
        items.append((C, n, H, grid))
        idx.append(p)
    if not items:
        return out
    B = K.KdeLscvBatch(items, **opts)
    B.eval()
    vals = B.out[:, 0].cpu().numpy()
    B.close()
    out[np.asarray(idx)] = vals
    return out


def lscv_search_batch(samples, grids, H0s=None, iters: int = 100, step: float = 0.25, min_bins: float = 1.0,
                      **opts) -> list:
    """LSCV search for many samples in lockstep: every round evaluates the
    pending simplex point of every unfinished search in one batched launch."""
    count = len(samples)
    gs = [K._grid(g) for g in grids]
    counts = [K.kde_bin(X, g, **{k: v for k, v in opts.items() if k in ("Q", "tile")})[0] for X, g in zip(samples, gs)]
    ns = [int(X.shape[0]) for X in samples]
    ds = [int(X.shape[1]) for X in samples]
    if H0s is None:
        H0s = [normal_scale(X.cpu().numpy()) for X in samples]
    gens = [nelder_mead(to_theta(H0), step=step, iters=iters) for H0 in H0s]
    pending = [next(gen) for gen in gens]
    results = [None] * count
    evals = [0] * count
    rounds = 0
    active = list(range(count))
    while active:
        rounds += 1
        vals = lscv_values_batch([(counts[i], ns[i], from_theta(pending[i], ds[i]), gs[i]) for i in active],
                                 min_bins=min_bins, **opts)
        still = []
        for i, v in zip(active, vals):
            evals[i] += 1
            try:
                pending[i] = gens[i].send(float(v))
                still.append(i)
            except StopIteration as stop:
                x, fx, _ = stop.value
                results[i] = {"H": from_theta(x, ds[i]), "lscv": fx, "evals": evals[i], "H0": H0s[i]}
        active = still
    for r in results:
        r["rounds"] = rounds
    return results
