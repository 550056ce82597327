"""Pins of the LSCV oracle (CPU, no GPU): the objective is checked against
things fixed by the mathematics, not against its own formula retyped.

* n = 2: the whole objective in closed form from SciPy's normal densities;
* the first term is the integral of the squared estimate (quadrature of
  SciPy densities), the second the leave-one-out sum written as a loop;
* exact scaling LSCV(aX, a^2 H) = a^-d LSCV(X, H);
* the binned pair sum with L = M - 1 is the brute-force double sum over grid
  nodes, and the binned objective tends to the direct one as the grid refines;
* planted mistakes (H for 2H, the diagonal kept, n^2 for n(n-1)) fail a pin;
* the search routine and its coordinates.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O
import workloads as W


def _phi(u, A):
    A = np.atleast_2d(A)
    return stats.multivariate_normal(mean=np.zeros(A.shape[0]), cov=A).pdf(np.atleast_1d(u))


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_two_samples_closed_form(d):
    rng = np.random.default_rng(5 + d)
    X = rng.normal(size=(2, d))
    H = W.random_spd(rng, d, lam_min=(0.2, 0.6), ratio=(1.0, 4.0))
    D = X[0] - X[1]
    ref = 0.5 * (_phi(np.zeros(d), 2 * H) + _phi(D, 2 * H)) - 2.0 * _phi(D, H)
    assert O.lscv_direct(X, H) == pytest.approx(ref, rel=1e-12, abs=1e-15)


def _integral_f2_1d(X, h2):
    f = lambda x: np.mean(stats.norm.pdf(x, loc=X, scale=math.sqrt(h2)))
    lo, hi = X.min() - 12 * math.sqrt(h2), X.max() + 12 * math.sqrt(h2)
    return integrate.quad(lambda x: f(x) ** 2, lo, hi, limit=400, epsabs=1e-13, epsrel=1e-11)[0]


def _loo(X, H):
    n = X.shape[0]
    s = 0.0
    for i in range(n):
        rest = np.delete(X, i, axis=0)
        s += np.mean([_phi(X[i] - r, H) for r in rest])
    return s / n


def test_terms_are_integral_and_leave_one_out_1d():
    rng = np.random.default_rng(11)
    X = rng.normal(size=(7, 1)) * 1.3
    h2 = 0.21
    H = np.array([[h2]])
    t1 = O.pair_sum(X, 2 * H, True) / 49
    assert t1 == pytest.approx(_integral_f2_1d(X[:, 0], h2), rel=1e-9)
    assert O.lscv_direct(X, H) == pytest.approx(_integral_f2_1d(X[:, 0], h2) - 2 * _loo(X, H), rel=1e-9)


def test_terms_are_integral_and_leave_one_out_2d():
    rng = np.random.default_rng(12)
    X = rng.normal(size=(6, 2))
    H = np.array([[0.3, 0.12], [0.12, 0.2]])
    # trapezoid rule on a wide box: spectrally accurate for this smooth, decaying integrand
    ax = [np.linspace(X[:, k].min() - 6, X[:, k].max() + 6, 801) for k in range(2)]
    G = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1).reshape(-1, 2)
    f = np.mean([stats.multivariate_normal(mean=x, cov=H).pdf(G) for x in X], axis=0)
    integral = float(np.sum(f ** 2) * (ax[0][1] - ax[0][0]) * (ax[1][1] - ax[1][0]))
    assert O.pair_sum(X, 2 * H, True) / 36 == pytest.approx(integral, rel=1e-8)
    assert O.lscv_direct(X, H) == pytest.approx(integral - 2 * _loo(X, H), rel=1e-7)


@pytest.mark.parametrize("d", [1, 2, 4])
def test_scaling_law(d):
    rng = np.random.default_rng(20 + d)
    X = rng.normal(size=(40, d))
    H = W.random_spd(rng, d, lam_min=(0.1, 0.3))
    a = 4.0                                   # a power of two keeps the binning inputs exact
    assert O.lscv_direct(a * X, a * a * H) == pytest.approx(O.lscv_direct(X, H) / a ** d, rel=1e-12)
    lo, hi = X.min(0) - 2, X.max(0) + 2
    M = (40,) * d if d < 4 else (10,) * 4
    b1 = O.lscv_binned(X, H, lo, hi, M)
    b2 = O.lscv_binned(a * X, a * a * H, a * lo, a * hi, M)
    assert b2 == pytest.approx(b1 / a ** d, rel=1e-12)


def test_binned_pair_sum_full_box_is_grid_double_sum():
    rng = np.random.default_rng(31)
    M = (12, 10)
    lo, hi = np.array([-2.0, -1.5]), np.array([2.5, 2.0])
    X = rng.uniform(lo, hi, size=(300, 2))
    c = O.counts_to_c(O.bin_fixed(X, lo, hi, M)[0], 2)
    A = np.array([[0.4, 0.15], [0.15, 0.3]])
    delta = O.bin_width(lo, hi, M)
    got = O.binned_pair_sum(c, A, delta, M, tau=1e6)     # L = M - 1: no truncation
    g = np.stack(np.meshgrid(*O.grid_axes(lo, hi, M), indexing="ij"), axis=-1).reshape(-1, 2)
    mvn = stats.multivariate_normal(mean=[0, 0], cov=A)
    brute = 0.0
    cf = c.ravel()
    for j in range(g.shape[0]):
        brute += cf[j] * float(np.sum(cf * mvn.pdf(g[j] - g)))
    assert got == pytest.approx(brute, rel=1e-12)


def test_binned_tends_to_direct():
    w = W.small_mixture(3, 2, 400, 16)
    H = w.H
    ref = O.lscv_direct(w.X, H)
    errs = [abs(O.lscv_binned(w.X, H, w.lo, w.hi, (m, m)) - ref) for m in (24, 48, 96)]
    assert errs[2] < errs[1] < errs[0]
    assert errs[0] / errs[2] > 6          # about O(delta^2): 16 for two halvings
    assert errs[2] < 1e-2 * abs(ref)


def _mutants():
    def first_term_H(X, H):
        n = X.shape[0]
        return O.pair_sum(X, H, True) / n ** 2 - 2.0 * O.pair_sum(X, H, False) / (n * (n - 1))

    def diagonal_kept(X, H):
        n = X.shape[0]
        return O.pair_sum(X, 2 * H, True) / n ** 2 - 2.0 * O.pair_sum(X, H, True) / (n * (n - 1))

    def n_squared(X, H):
        n = X.shape[0]
        return O.pair_sum(X, 2 * H, True) / n ** 2 - 2.0 * O.pair_sum(X, H, False) / n ** 2

    return [first_term_H, diagonal_kept, n_squared]


@pytest.mark.parametrize("mutant", _mutants())
def test_planted_mistakes_are_caught(mutant):
    rng = np.random.default_rng(41)
    X = rng.normal(size=(2, 2))
    H = np.array([[0.5, 0.1], [0.1, 0.4]])
    D = X[0] - X[1]
    ref = 0.5 * (_phi(np.zeros(2), 2 * H) + _phi(D, 2 * H)) - 2.0 * _phi(D, H)
    assert abs(mutant(X, H) - ref) > 1e-6 * abs(ref)


def test_search_coordinates_and_nelder_mead():
    rng = np.random.default_rng(50)
    for d in (1, 2, 3):
        H = W.random_spd(rng, d)
        assert np.allclose(O.from_chol_params(O.chol_params(H), d), H, rtol=1e-13, atol=1e-15)
    a = np.array([0.3, -1.2, 2.0])
    x, v = O.nelder_mead(lambda t: float(np.sum((t - a) ** 2)) + 1.0, np.zeros(3), iters=400, tol=1e-14)
    assert np.allclose(x, a, atol=1e-5) and v == pytest.approx(1.0, abs=1e-9)


def test_lscv_minimum_near_normal_scale_for_normal_data():
    """For normal data the LSCV minimiser is a consistent estimate of the MISE
    optimum, which the normal-scale rule also targets: same order of magnitude."""
    rng = np.random.default_rng(60)
    X = rng.multivariate_normal([0, 0], [[1.0, 0.6], [0.6, 1.0]], size=600)
    Hns = W.normal_scale_H(X)
    lo, hi = X.min(0) - 2, X.max(0) + 2
    f = lambda t: O.lscv_binned(X, O.from_chol_params(t, 2), lo, hi, (48, 48))
    t, v = O.nelder_mead(f, O.chol_params(Hns), iters=60)
    Hopt = O.from_chol_params(t, 2)
    r = np.linalg.det(Hopt) / np.linalg.det(Hns)
    assert 0.1 < r < 10 and v <= f(O.chol_params(Hns))
