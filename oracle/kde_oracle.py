"""Plain FP64 CPU oracle for binned FFT kernel density estimation with an
unconstrained (full, symmetric positive definite) bandwidth matrix H.

TEST INFRASTRUCTURE. Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module. The GPU library never
calls it and shares no code, table or helper with it.

Source: A. Gramacki and J. Gramacki, "FFT-Based Fast Computation of
Multivariate Kernel Density Estimators with Unconstrained Bandwidth Matrices"
(arXiv 1508.02766). Section and equation numbers below are the paper's:

* Eq. (1)  f(x, H) = n^-1 sum_i K_H(x - X_i), K_H(u) = |H|^-1/2 K(H^-1/2 u),
           K the standard normal density (Section 1).
* Eq. (2)  binned estimate on grid points g_j with grid counts c_l (Section 2).
* Eq. (3), (4)  equally spaced grid and bin width delta_k (Section 2).
* Eq. (5), (6)  the binned estimate as a convolution with k_l = n^-1 K_H(delta * l).
* Eq. (7)  the same convolution truncated to |l_k| <= L_k (Section 2).
* Eq. (8)-(9), (10), (11)  Wand's wrap-around kernel array, zero-padded counts,
           discrete convolution theorem and extraction (Section 4.1).
* Eq. (12)-(14)  the corrected zero-padded layout of k and c and its extraction
           window (Section 4.2).
* Eq. (15) L_k = min(M_k - 1, ceil(tau sqrt|lambda| / delta_k)), lambda the
           largest eigenvalue of H, tau about 3.7 (Section 4.2).

The primary result is Eq. (7) written out as a direct sum (``conv_direct``);
the FFT forms are the paper's algorithms, kept as cross-checks.

Readings where the paper is silent (each one is also listed in the design
notes):

* Linear binning (Section 2 only names it): multilinear tent weights to the
  2^d surrounding nodes, so each sample contributes total weight 1 and the
  counts sum to n as the Section 3 footnote requires.
* Binning is done in integer fixed point: t = u - floor(u) is rounded to
  q = rint(t 2^Q) (ties to even) and the corner weights are integer products
  of q and 2^Q - q, accumulated in uint64. Count c_l = counts_l 2^-dQ.
  Default Q = floor(32 / d).
* u = (X_ik - lo_k) / delta_k is one IEEE FP64 subtraction and one FP64
  division. A sample with u < 0, u > M_k - 1 or u NaN on any axis is dropped
  and counted; the normalisation still uses the total n. A sample on the last
  node (u = M_k - 1) takes j_k = M_k - 2, t_k = 1.
* tau = 3.7 on every dimension; one lambda (largest eigenvalue) for all axes.
* The result is Eq. (7) on the grid; the FFT layout used to reach it is free.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

TAU_DEFAULT = 3.7   # Section 4.2, after Eq. (15)


# --------------------------------------------------------------------------
# validation and grid (Eq. 3, 4)
# --------------------------------------------------------------------------

def check_bandwidth(H) -> np.ndarray:
    """H must be a symmetric positive definite d x d matrix (Section 1, Eq. 1)."""
    H = np.asarray(H, dtype=np.float64)
    if H.ndim != 2 or H.shape[0] != H.shape[1] or H.shape[0] not in (1, 2, 3, 4):
        raise ValueError("H must be d x d with d in {1, 2, 3, 4}")
    if not np.all(np.isfinite(H)):
        raise ValueError("H must be finite")
    if np.max(np.abs(H - H.T)) > 1e-12 * np.max(np.abs(H)):
        raise ValueError("H must be symmetric")
    if np.linalg.eigvalsh(H)[0] <= 0.0:
        raise ValueError("H must be positive definite")
    return H


def default_Q(d: int) -> int:
    return 32 // d


def bin_width(lo, hi, M) -> np.ndarray:
    """delta_k = (g_kM - g_k1) / (M_k - 1), Eq. (4)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    return (hi - lo) / (M - 1.0)


def grid_axes(lo, hi, M):
    """Grid coordinates g_kj = lo_k + j delta_k, j = 0..M_k-1 (Eq. 3, 0-based)."""
    delta = bin_width(lo, hi, M)
    return [lo[k] + np.arange(M[k], dtype=np.float64) * delta[k] for k in range(len(M))]


# --------------------------------------------------------------------------
# linear binning (Section 2, step one; Section 3 footnote: counts sum to n)
# --------------------------------------------------------------------------

def bin_fixed(X, lo, hi, M, Q: int | None = None):
    """Fixed-point multilinear binning.

    Returns (counts, n_dropped); counts is a uint64 array of shape M in units
    of 2^-dQ, so c_l = counts_l / 2^(dQ).
    """
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    M = tuple(int(m) for m in M)
    if Q is None:
        Q = default_Q(d)
    lo = np.asarray(lo, dtype=np.float64)
    delta = bin_width(lo, hi, M)
    counts = np.zeros(M, dtype=np.uint64)
    if n == 0:
        return counts, 0
    u = (X - lo) / delta                      # IEEE subtract, then divide
    top = np.asarray(M, dtype=np.float64) - 1.0
    keep = np.all((u >= 0.0) & (u <= top), axis=1)   # NaN compares false
    n_dropped = int(n - np.count_nonzero(keep))
    u = u[keep]
    j = np.floor(u)
    j = np.minimum(j, top - 1.0)              # sample on the last node
    t = u - j                                 # exact in FP64
    one = np.uint64(1) << np.uint64(Q)
    q = np.rint(t * float(2 ** Q)).astype(np.uint64)
    jj = j.astype(np.int64)
    for corner in itertools.product((0, 1), repeat=d):
        w = np.ones(u.shape[0], dtype=np.uint64)
        for k in range(d):
            w = w * (q[:, k] if corner[k] else one - q[:, k])
        idx = tuple(jj[:, k] + corner[k] for k in range(d))
        np.add.at(counts, idx, w)
    return counts, n_dropped


def counts_to_c(counts, d: int, Q: int | None = None) -> np.ndarray:
    """Grid counts c_l = counts_l / 2^dQ as FP64 (exact while counts_l < 2^53)."""
    if Q is None:
        Q = default_Q(d)
    return np.asarray(counts, dtype=np.float64) / float(2 ** (d * Q))


# --------------------------------------------------------------------------
# truncation (Eq. 15) and kernel weights (Eq. 6 with Eq. 1)
# --------------------------------------------------------------------------

def lambda_max(H) -> float:
    """Largest eigenvalue of H (LAPACK symmetric eigensolver)."""
    return float(np.linalg.eigvalsh(np.asarray(H, dtype=np.float64))[-1])


def truncation_L(H, delta, M, tau: float = TAU_DEFAULT, extent: str = "eigen"):
    """L_k = min(M_k - 1, ceil(tau sqrt(|lambda|) / delta_k)), Eq. (15).

    extent = "marginal": tau sqrt(H_kk) instead of tau sqrt(|lambda|), the
    half width along axis k of the ellipsoid u' H^-1 u <= tau^2.
    """
    H = np.asarray(H, dtype=np.float64)
    lam = lambda_max(H)
    half = [math.sqrt(H[k, k]) if extent == "marginal" else math.sqrt(abs(lam)) for k in range(len(M))]
    return tuple(int(min(int(M[k]) - 1, math.ceil(tau * half[k] / float(delta[k]))))
                 for k in range(len(M)))


def gaussian_KH(U, H) -> np.ndarray:
    """K_H(u) = |H|^-1/2 (2 pi)^-d/2 exp(-u' H^-1 u / 2) for rows u of U (Eq. 1)."""
    H = np.asarray(H, dtype=np.float64)
    d = H.shape[0]
    U = np.asarray(U, dtype=np.float64).reshape(-1, d)
    Hinv = np.linalg.inv(H)
    quad = np.einsum("ij,jk,ik->i", U, Hinv, U)
    return np.exp(-0.5 * quad) / math.sqrt(np.linalg.det(H)) / (2.0 * math.pi) ** (d / 2.0)


def lag_weights(H, delta, L, n: int) -> np.ndarray:
    """k_l = n^-1 K_H(delta_1 l_1, ..., delta_d l_d) for l in the box [-L, L] (Eq. 6).

    Returned with shape (2 L_1 + 1, ..., 2 L_d + 1); entry [L_1 + l_1, ...] is k_l.
    """
    d = len(L)
    axes = [np.arange(-L[k], L[k] + 1, dtype=np.float64) * float(delta[k]) for k in range(d)]
    mesh = np.meshgrid(*axes, indexing="ij")
    U = np.stack([m.ravel() for m in mesh], axis=1)
    return (gaussian_KH(U, H) / float(n)).reshape(tuple(2 * l + 1 for l in L))


# --------------------------------------------------------------------------
# the truncated binned estimate, Eq. (7): the oracle's primary result
# --------------------------------------------------------------------------

def conv_direct(c, k, L) -> np.ndarray:
    """f_j = sum_{|l_k| <= L_k} c_{j-l} k_l for every grid index j, c = 0 off the grid."""
    c = np.asarray(c, dtype=np.float64)
    M = c.shape
    d = c.ndim
    f = np.zeros(M, dtype=np.float64)
    for lag in itertools.product(*[range(-L[a], L[a] + 1) for a in range(d)]):
        w = k[tuple(lag[a] + L[a] for a in range(d))]
        # f[j] += c[j - lag] * w over the j for which j - lag lies on the grid
        dst, src = [], []
        for a in range(d):
            l = lag[a]
            if l >= M[a] or -l >= M[a]:
                break
            dst.append(slice(max(l, 0), M[a] + min(l, 0)))
            src.append(slice(max(-l, 0), M[a] - max(l, 0)))
        else:
            f[tuple(dst)] += w * c[tuple(src)]
    return f


def conv_direct_at(c, k, L, points) -> np.ndarray:
    """Eq. (7) at selected grid indices only (rows of ``points``), one by one."""
    c = np.asarray(c, dtype=np.float64)
    M = c.shape
    d = c.ndim
    out = np.empty(len(points), dtype=np.float64)
    for i, j in enumerate(points):
        acc = 0.0
        lo_l = [max(-L[a], j[a] - (M[a] - 1)) for a in range(d)]
        hi_l = [min(L[a], j[a]) for a in range(d)]
        if any(lo_l[a] > hi_l[a] for a in range(d)):
            out[i] = 0.0
            continue
        # lags l with 0 <= j - l < M, |l| <= L
        csl = tuple(slice(j[a] - hi_l[a], j[a] - lo_l[a] + 1) for a in range(d))
        ksl = tuple(slice(lo_l[a] + L[a], hi_l[a] + L[a] + 1) for a in range(d))
        cs = c[csl]
        ks = k[ksl]
        # c index runs j-hi .. j-lo while the lag runs hi .. lo: flip every axis
        acc = float(np.sum(cs[tuple(slice(None, None, -1) for _ in range(d))] * ks))
        out[i] = acc
    return out


# --------------------------------------------------------------------------
# the paper's FFT algorithms (Section 4)
# --------------------------------------------------------------------------

def _pow2_at_least(x: int) -> int:
    p = 1
    while p < x:
        p *= 2
    return p


def conv_fft_corrected(c, k, L, P=None, workers=None) -> np.ndarray:
    """Corrected FFT algorithm, Eq. (12)-(14), with the discrete convolution theorem (Eq. 10).

    k_new holds the whole signed lag box at its top-left corner (lag -L_k at
    index 0), c_new holds c with c_1 at 1-based position M_k (0-based
    offset M_k - 1), both zero padded to P_k. The estimate is read at
    0-based positions j + L_k + M_k - 1; for L_k = M_k - 1 that is the 1-based
    window (2M_k - 1) : (3M_k - 2) of Eq. (14). numpy's inverse FFT already
    divides by prod P_k. ``workers``: run the same transforms through scipy.fft with that
    many threads (used to time the oracle on several host cores).
    """
    c = np.asarray(c, dtype=np.float64)
    M = c.shape
    d = c.ndim
    if P is None:
        P = tuple(_pow2_at_least(2 * L[a] + 2 * M[a] - 1) for a in range(d))
    k_new = np.zeros(P)
    k_new[tuple(slice(0, 2 * L[a] + 1) for a in range(d))] = k
    c_new = np.zeros(P)
    c_new[tuple(slice(M[a] - 1, 2 * M[a] - 1) for a in range(d))] = c
    if workers:
        import scipy.fft as sf
        s = sf.ifftn(sf.fftn(c_new, workers=workers) * sf.fftn(k_new, workers=workers), workers=workers).real
    else:
        s = np.fft.ifftn(np.fft.fftn(c_new) * np.fft.fftn(k_new)).real
    return s[tuple(slice(L[a] + M[a] - 1, L[a] + 2 * M[a] - 1) for a in range(d))].copy()


def conv_fft_wand(c, k, L, P=None) -> np.ndarray:
    """Wand's original wrap-around ordering, Eq. (8), (9), (11) (the defective form).

    Only the non-negative lag orthant of k is used; the positions of negative
    lags receive the weight of the mirrored positive lag k_{|l_1|, ..., |l_d|}.
    The estimate is s[1:M_1, ..., 1:M_d] / prod P_k (Eq. 11).
    """
    c = np.asarray(c, dtype=np.float64)
    M = c.shape
    d = c.ndim
    if P is None:
        P = tuple(_pow2_at_least(M[a] + L[a]) for a in range(d))
    kw = np.zeros(P)
    for pos in itertools.product(*[list(range(0, L[a] + 1)) + list(range(P[a] - L[a], P[a]))
                                   for a in range(d)]):
        absl = tuple(pos[a] if pos[a] <= L[a] else P[a] - pos[a] for a in range(d))
        kw[pos] = k[tuple(absl[a] + L[a] for a in range(d))]
    c_pad = np.zeros(P)
    c_pad[tuple(slice(0, M[a]) for a in range(d))] = c
    s = np.fft.ifftn(np.fft.fftn(c_pad) * np.fft.fftn(kw)).real
    return s[tuple(slice(0, M[a]) for a in range(d))].copy()


# --------------------------------------------------------------------------
# test-only references: Eq. (1) and Eq. (2)
# --------------------------------------------------------------------------

def kde_direct(X, H, points) -> np.ndarray:
    """Eq. (1) evaluated directly at ``points`` (m x d): O(m n) kernel evaluations."""
    X = np.asarray(X, dtype=np.float64)
    points = np.asarray(points, dtype=np.float64)
    n = X.shape[0]
    out = np.empty(points.shape[0], dtype=np.float64)
    step = max(1, 2_000_000 // max(n, 1))
    for s in range(0, points.shape[0], step):
        P = points[s:s + step]
        U = (P[:, None, :] - X[None, :, :]).reshape(-1, X.shape[1])
        out[s:s + step] = gaussian_KH(U, H).reshape(P.shape[0], n).sum(axis=1) / n
    return out


def bkde_double_sum(c, H, lo, hi, n: int) -> np.ndarray:
    """Eq. (2): f(g_j) = n^-1 sum over every grid node l of K_H(g_j - g_l) c_l."""
    c = np.asarray(c, dtype=np.float64)
    M = c.shape
    axes = grid_axes(np.asarray(lo, float), np.asarray(hi, float), M)
    G = np.stack([m.ravel() for m in np.meshgrid(*axes, indexing="ij")], axis=1)
    cf = c.ravel()
    out = np.empty(G.shape[0])
    for j in range(G.shape[0]):
        out[j] = np.sum(gaussian_KH(G[j] - G, H) * cf) / n
    return out.reshape(M)


# --------------------------------------------------------------------------
# the whole path
# --------------------------------------------------------------------------

def plan(H, lo, hi, M, n, tau: float = TAU_DEFAULT, L=None, Q=None, extent: str = "eigen"):
    """Grid spacing, truncation and fixed-point scale for one problem."""
    H = check_bandwidth(H)
    d = H.shape[0]
    M = tuple(int(m) for m in M)
    if len(M) != d or any(m < 2 for m in M):
        raise ValueError("need M_k >= 2 on each of the d axes")
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if not np.all(hi > lo):
        raise ValueError("need hi_k > lo_k")
    delta = bin_width(lo, hi, M)
    if L is None:
        L = truncation_L(H, delta, M, tau, extent)
    L = tuple(int(x) for x in L)
    if Q is None:
        Q = default_Q(d)
    return {"d": d, "M": M, "delta": delta, "L": L, "Q": Q, "n": int(n)}


def kde_binned(X, H, lo, hi, M, tau: float = TAU_DEFAULT, L=None, Q=None, method: str = "direct",
               extent: str = "eigen", workers=None):
    """Binned estimate on the grid: linear binning, weights on the lag box, Eq. (7).

    Returns (density, info) where info carries counts, n_dropped, L, delta.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if n == 0:
        raise ValueError("the estimate needs n >= 1 (Eq. 1 divides by n)")
    p = plan(H, lo, hi, M, n, tau=tau, L=L, Q=Q, extent=extent)
    counts, n_dropped = bin_fixed(X, lo, hi, p["M"], p["Q"])
    c = counts_to_c(counts, p["d"], p["Q"])
    k = lag_weights(H, p["delta"], p["L"], n)
    if method == "direct":
        f = conv_direct(c, k, p["L"])
    elif method == "fft":
        f = conv_fft_corrected(c, k, p["L"], workers=workers)
    else:
        raise ValueError(method)
    info = dict(p)
    info.update(counts=counts, n_dropped=n_dropped, k=k, c=c)
    return f, info
