"""FP64 CPU oracle of the least-squares cross-validation (LSCV) objective.

TEST INFRASTRUCTURE, like kde_oracle: imported only by the tests, the package
smoke check and the benchmark's CPU-baseline leg.

The paper closes (Section 5) by pointing at bandwidth selection as the next
use of the binned FFT machinery, for a class of functionals whose
computation has the same convolution form as Eq. (5)-(7). LSCV is the
textbook member of that class for a Gaussian kernel with a full H:

    LSCV(H) = int f^2 - 2 n^-1 sum_i f_{-i}(X_i)
            = n^-2 sum_{i,j} phi_{2H}(X_i - X_j) - 2 [n (n - 1)]^-1 sum_{i != j} phi_H(X_i - X_j),

phi_A the N(0, A) density (K_A of Eq. 1), f the estimate of Eq. (1) and
f_{-i} the estimate without sample i. The first line is the definition; the
second uses that the convolution of two N(0, H) densities is N(0, 2H).

Binned form (the reading adopted here; the paper gives no formula):
each double sum over sample pairs becomes a double sum over grid counts,

    S(A) = sum_j c_j sum_{|l_k| <= L_k(A)} c_{j-l} phi_A(delta l),

i.e. Eq. (7) with k_l = phi_A(delta l) (no 1/n) and L from Eq. (15) with the
largest eigenvalue of A, followed by a dot product with the counts. The
i = j pairs of the second sum are removed as n phi_H(0), their exact value:

    LSCV_binned(H) = n^-2 S(2H) - 2 [n (n - 1)]^-1 (S(H) - n phi_H(0)).
"""
from __future__ import annotations

import math

import numpy as np

from .kde_oracle import TAU_DEFAULT, bin_fixed, bin_width, check_bandwidth, conv_direct, counts_to_c, \
    default_Q, gaussian_KH, lag_weights, truncation_L


def pair_sum(X, A, include_diagonal: bool) -> float:
    """sum over ordered sample pairs (i, j) of phi_A(X_i - X_j), optionally without i = j."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    total = 0.0
    step = max(1, 2_000_000 // max(n, 1))
    for s in range(0, n, step):
        U = (X[s:s + step, None, :] - X[None, :, :]).reshape(-1, d)
        total += float(np.sum(gaussian_KH(U, A)))
    if not include_diagonal:
        total -= n * float(gaussian_KH(np.zeros((1, d)), A)[0])
    return total


def lscv_direct(X, H) -> float:
    """LSCV(H) from the sample pairs (second line of the module docstring), O(n^2)."""
    H = check_bandwidth(H)
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if n < 2:
        raise ValueError("LSCV needs n >= 2")
    return pair_sum(X, 2.0 * H, True) / n ** 2 - 2.0 * pair_sum(X, H, False) / (n * (n - 1))


def binned_pair_sum(c, A, delta, M, tau: float = TAU_DEFAULT) -> float:
    """S(A): Eq. (7) with weights phi_A(delta l) on the box of Eq. (15) for A, dotted with c."""
    L = truncation_L(A, delta, M, tau)
    k = lag_weights(A, delta, L, 1)
    return float(np.sum(c * conv_direct(c, k, L)))


def lscv_binned_terms(X, H, lo, hi, M, tau: float = TAU_DEFAULT, Q=None):
    """(LSCV, first term n^-2 S(2H), second term 2 [n(n-1)]^-1 (S(H) - n phi_H(0)))."""
    H = check_bandwidth(H)
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    if n < 2:
        raise ValueError("LSCV needs n >= 2")
    M = tuple(int(m) for m in M)
    if Q is None:
        Q = default_Q(d)
    counts, _ = bin_fixed(X, lo, hi, M, Q)
    c = counts_to_c(counts, d, Q)
    delta = bin_width(lo, hi, M)
    t1 = binned_pair_sum(c, 2.0 * H, delta, M, tau) / n ** 2
    phi0 = 1.0 / math.sqrt(np.linalg.det(H)) / (2.0 * math.pi) ** (d / 2.0)
    t2 = 2.0 * (binned_pair_sum(c, H, delta, M, tau) - n * phi0) / (n * (n - 1))
    return t1 - t2, t1, t2


def lscv_binned(X, H, lo, hi, M, tau: float = TAU_DEFAULT, Q=None) -> float:
    return lscv_binned_terms(X, H, lo, hi, M, tau, Q)[0]


def chol_params(H) -> np.ndarray:
    """Search coordinates of an SPD H: (log R_11, R_21, log R_22, ...) of H = R R', R lower triangular."""
    R = np.linalg.cholesky(np.asarray(H, dtype=np.float64))
    d = R.shape[0]
    out = []
    for i in range(d):
        for j in range(i + 1):
            out.append(math.log(R[i, j]) if i == j else R[i, j])
    return np.array(out)


def from_chol_params(theta, d: int) -> np.ndarray:
    R = np.zeros((d, d))
    it = iter(theta)
    for i in range(d):
        for j in range(i + 1):
            v = next(it)
            R[i, j] = math.exp(v) if i == j else v
    return R @ R.T


def nelder_mead(f, x0, step: float = 0.25, iters: int = 200, tol: float = 1e-10):
    """Plain Nelder-Mead (reflection 1, expansion 2, contraction 1/2, shrink 1/2), minimising f."""
    x0 = np.asarray(x0, dtype=np.float64)
    m = x0.size
    simplex = [x0] + [x0 + step * np.eye(m)[k] for k in range(m)]
    vals = [f(x) for x in simplex]
    for _ in range(iters):
        order = np.argsort(vals, kind="stable")
        simplex = [simplex[i] for i in order]
        vals = [vals[i] for i in order]
        if abs(vals[-1] - vals[0]) <= tol * (abs(vals[0]) + 1e-300):
            break
        centroid = np.mean(simplex[:-1], axis=0)
        xr = centroid + (centroid - simplex[-1])
        fr = f(xr)
        if vals[0] <= fr < vals[-2]:
            simplex[-1], vals[-1] = xr, fr
            continue
        if fr < vals[0]:
            xe = centroid + 2.0 * (centroid - simplex[-1])
            fe = f(xe)
            simplex[-1], vals[-1] = (xe, fe) if fe < fr else (xr, fr)
            continue
        xc = centroid + 0.5 * (simplex[-1] - centroid)
        fc = f(xc)
        if fc < vals[-1]:
            simplex[-1], vals[-1] = xc, fc
            continue
        for k in range(1, m + 1):
            simplex[k] = simplex[0] + 0.5 * (simplex[k] - simplex[0])
            vals[k] = f(simplex[k])
    i = int(np.argmin(vals))
    return simplex[i], vals[i]
