"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper it pins (section / equation) and the
independent source of truth: hand-derived integers, a closed form, a SciPy or
NumPy library routine, brute force, or an invariant the paper states. A
plausible slip in the oracle (a dropped factor, a transposed operand, a wrong
sign or index, floor for rint, the mirrored Wand ordering) fails at least one
of them; ``test_planted_mistakes_are_caught`` checks that on planted copies.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.signal
import scipy.stats

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# linear binning (Section 2 step one; Section 3 footnote)
# --------------------------------------------------------------------------

def test_binning_hand_cases_2d():
    """Hand-derived fixed-point weights on a unit-spaced 4x4 grid (Q = 16)."""
    one = 2 ** 16
    X = np.array([
        [1.0, 1.0],                 # on a node: all weight there
        [1.5, 2.5],                 # cell centre: a quarter to each corner
        [3.0, 3.0],                 # on the last node: j clamped to M-2, t = 1
        [0.25, 0.0],                # t = (1/4, 0)
        [0.1, 2.0],                 # 0.1 * 2^16 = 6553.6000000000004 -> 6554
        [1.0 + 3.0 / 2 ** 17, 0.0],  # t 2^Q = 1.5 exactly -> ties to even -> 2
        [1.0 + 5.0 / 2 ** 17, 1.0],  # t 2^Q = 2.5 exactly -> ties to even -> 2
        [-0.1, 1.0],                # outside: dropped
        [1.0, 3.0000000001],        # outside: dropped
        [np.nan, 1.0],              # NaN: dropped
        [np.inf, 0.0],              # infinite: dropped
    ])
    counts, nd = O.bin_fixed(X, [0.0, 0.0], [3.0, 3.0], (4, 4))
    exp = np.zeros((4, 4), dtype=object)
    exp[1, 1] += one * one
    for c in [(1, 2), (2, 2), (1, 3), (2, 3)]:
        exp[c] += 2 ** 30
    exp[3, 3] += one * one
    exp[0, 0] += (one - 16384) * one
    exp[1, 0] += 16384 * one
    exp[0, 2] += (one - 6554) * one
    exp[1, 2] += 6554 * one
    exp[1, 0] += (one - 2) * one
    exp[2, 0] += 2 * one
    exp[1, 1] += (one - 2) * one
    exp[2, 1] += 2 * one
    assert nd == 4
    assert [[int(v) for v in row] for row in counts] == [[int(v) for v in row] for row in exp]


def test_binning_hand_cases_1d_3d():
    c1, nd1 = O.bin_fixed(np.array([[0.75]]), [0.0], [1.0], (2,))      # Q = 32
    assert nd1 == 0 and [int(v) for v in c1] == [2 ** 32 - 3 * 2 ** 30, 3 * 2 ** 30]
    c3, nd3 = O.bin_fixed(np.array([[0.5, 0.5, 0.5]]), [0.0] * 3, [2.0] * 3, (3, 3, 3))  # Q = 10
    assert nd3 == 0
    for corner in itertools.product((0, 1), repeat=3):
        assert int(c3[corner]) == 512 ** 3
    assert int(c3.sum()) == 2 ** 30


def test_binning_hand_case_4d():
    """d = 4, Q = 8: fractions (1/4, 1/2, 0, 3/4) give the per-axis weight pairs (192, 64),
    (128, 128), (256, 0), (64, 192); corner b receives their product."""
    c4, nd4 = O.bin_fixed(np.array([[0.25, 0.5, 0.0, 0.75]]), [0.0] * 4, [1.0] * 4, (2, 2, 2, 2))
    assert nd4 == 0 and O.default_Q(4) == 8
    assert int(c4[0, 0, 0, 0]) == 402_653_184        # 192 128 256 64
    assert int(c4[0, 0, 0, 1]) == 1_207_959_552      # 192 128 256 192
    assert int(c4[1, 1, 0, 0]) == 134_217_728        # 64 128 256 64
    assert int(c4[1, 0, 0, 1]) == 402_653_184        # 64 128 256 192
    assert not c4[:, :, 1, :].any()                  # q = 0 on axis 3: nothing on the upper face
    assert int(c4.sum()) == 2 ** 32


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_binning_counts_sum_to_n(d):
    """Grid counts sum to n (Section 3 footnote), here n - n_dropped exactly in units 2^-dQ."""
    rng = np.random.default_rng(5 + d)
    n = 20000
    X = rng.normal(size=(n, d)) * 1.5
    lo, hi = -np.full(d, 3.0), np.full(d, 3.0)
    counts, nd = O.bin_fixed(X, lo, hi, (33,) * d)
    inside = np.all((X >= -3.0) & (X <= 3.0), axis=1)
    assert nd == n - inside.sum() and nd > 0
    assert int(counts.sum(dtype=np.uint64)) == (n - nd) * 2 ** (d * O.default_Q(d))


def test_binning_first_moment_4d():
    """The same in d = 4 (Q = 8) on every axis: a transposed or shifted corner index fails it."""
    w = W.small_mixture(seed=61, d=4, n=5000, M=(9, 12, 7, 10))
    counts, nd = O.bin_fixed(w.X, w.lo, w.hi, w.M)
    assert nd == 0
    c = O.counts_to_c(counts, 4)
    g = O.grid_axes(w.lo, w.hi, w.M)
    delta = O.bin_width(w.lo, w.hi, w.M)
    for a in range(4):
        marg = c.sum(axis=tuple(b for b in range(4) if b != a))
        tol = w.n * delta[a] * 2.0 ** -(8 + 1) + 1e-9
        assert abs((marg * g[a]).sum() - w.X[:, a].sum()) <= tol, a


def test_binning_first_moment():
    """Linear interpolation reproduces linear functions: sum_l c_l g_l = sum_i X_i,
    up to the position quantisation delta 2^-(Q+1) per sample."""
    w = W.mix2d_small()
    counts, nd = O.bin_fixed(w.X, w.lo, w.hi, w.M)
    assert nd == 0
    c = O.counts_to_c(counts, 2)
    g = O.grid_axes(w.lo, w.hi, w.M)
    delta = O.bin_width(w.lo, w.hi, w.M)
    m1 = (c.sum(axis=1) * g[0]).sum()
    m2 = (c.sum(axis=0) * g[1]).sum()
    tol = w.n * delta * 2.0 ** -(16 + 1) + 1e-9
    assert abs(m1 - w.X[:, 0].sum()) <= tol[0]
    assert abs(m2 - w.X[:, 1].sum()) <= tol[1]


# --------------------------------------------------------------------------
# Eq. (15): truncation
# --------------------------------------------------------------------------

def test_lambda_max_closed_form_2x2():
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    tr, det = np.trace(H), np.linalg.det(H)
    lam = (tr + math.sqrt(tr * tr - 4 * det)) / 2
    assert O.lambda_max(H) == pytest.approx(lam, rel=1e-14)
    assert lam == pytest.approx(0.145207973, abs=1e-8)
    # Eq. (15) on the grid [-4, 4]^2 with 64 nodes: delta = 8/63
    L = O.truncation_L(H, np.array([8 / 63, 8 / 63]), (64, 64), 3.7)
    assert L == (math.ceil(3.7 * math.sqrt(lam) / (8 / 63)),) * 2 == (12, 12)
    # the min(M - 1, .) branch
    assert O.truncation_L(H, np.array([8 / 63, 0.001]), (64, 64), 3.7) == (12, 63)


def test_paper_constants_fixture():
    """tau (Section 4.2, after Eq. 15) and the Eq. (14) window, as printed in the paper."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        g = json.load(fh)
    assert O.TAU_DEFAULT == g["tau"]
    a, b = g["extract_window_1based"]        # coefficients of M: (2M - 1) : (3M - 2)
    for M in (4, 64, 512):
        L = M - 1
        first0, last0 = L + M - 1, L + 2 * M - 2   # the oracle's 0-based read-out
        assert first0 + 1 == a[0] * M + a[1] and last0 + 1 == b[0] * M + b[1]


# --------------------------------------------------------------------------
# Eq. (6) with Eq. (1): lag weights
# --------------------------------------------------------------------------

@pytest.mark.parametrize("H", [
    np.array([[0.09, 0.06], [0.06, 0.08]]),
    np.array([[0.5, -0.2, 0.1], [-0.2, 0.3, 0.05], [0.1, 0.05, 0.2]]),
    np.array([[0.04]]),
    np.array([[0.5, -0.2, 0.1, 0.05], [-0.2, 0.3, 0.05, -0.1], [0.1, 0.05, 0.2, 0.02], [0.05, -0.1, 0.02, 0.25]]),
])
def test_lag_weights_vs_scipy_mvn(H):
    d = H.shape[0]
    delta = np.array([0.11, 0.07, 0.13, 0.09][:d])
    L = tuple([4, 5, 3, 2][:d])
    n = 37
    k = O.lag_weights(H, delta, L, n)
    mvn = scipy.stats.multivariate_normal(mean=np.zeros(d), cov=H)
    for lag in itertools.product(*[range(-l, l + 1) for l in L]):
        ref = mvn.pdf(np.array(lag) * delta) / n
        assert k[tuple(lag[a] + L[a] for a in range(d))] == pytest.approx(ref, rel=1e-12)
    # closed form at the origin: n^-1 (2 pi)^-d/2 |H|^-1/2
    assert k[tuple(L)] == pytest.approx(1 / n / (2 * np.pi) ** (d / 2) / np.sqrt(np.linalg.det(H)), rel=1e-13)


def test_lag_symmetries():
    """k_-l = k_l always; per-axis reflection k_(-l1,l2) = k_(l1,l2) only for diagonal H (Section 4.1)."""
    delta = np.array([0.1, 0.1])
    L = (6, 6)
    Hf = np.array([[0.09, 0.06], [0.06, 0.08]])
    Hd = np.diag(np.diag(Hf))
    kf = O.lag_weights(Hf, delta, L, 1)
    kd = O.lag_weights(Hd, delta, L, 1)
    assert np.array_equal(kf, kf[::-1, ::-1]) or np.allclose(kf, kf[::-1, ::-1], rtol=1e-14, atol=0)
    assert np.allclose(kd, kd[::-1, :], rtol=1e-14, atol=0)
    assert not np.allclose(kf, kf[::-1, :], rtol=1e-3, atol=0)


# --------------------------------------------------------------------------
# Eq. (7): the direct truncated convolution
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape,L", [((13,), (4,)), ((9, 14), (3, 5)), ((6, 7, 5), (2, 3, 1)), ((5, 4), (4, 3)),
                                     ((5, 4, 6, 3), (2, 1, 2, 1))])
def test_conv_direct_vs_scipy_convolve(shape, L):
    """Eq. (7) with an arbitrary (asymmetric) weight box equals the 'full'
    linear convolution sliced at offset L (library routine)."""
    rng = np.random.default_rng(11)
    c = rng.random(shape)
    k = rng.random(tuple(2 * l + 1 for l in L))
    f = O.conv_direct(c, k, L)
    full = scipy.signal.convolve(c, k, mode="full", method="direct")
    ref = full[tuple(slice(L[a], L[a] + shape[a]) for a in range(len(shape)))]
    assert np.allclose(f, ref, rtol=1e-13, atol=1e-13)
    pts = [tuple(rng.integers(0, s) for s in shape) for _ in range(20)] + [tuple(0 for _ in shape),
                                                                           tuple(s - 1 for s in shape)]
    assert np.allclose(O.conv_direct_at(c, k, L, pts), [ref[p] for p in pts], rtol=1e-13, atol=1e-13)


def test_eq7_full_box_equals_eq2_double_sum():
    """Eq. (7) with L_k = M_k - 1 is Eq. (5), a rewrite of Eq. (2) (brute-force double sum)."""
    rng = np.random.default_rng(3)
    X = rng.normal(size=(60, 2)) * 0.8
    H = np.array([[0.2, -0.12], [-0.12, 0.15]])
    lo, hi, M = np.array([-3.0, -2.5]), np.array([3.0, 2.5]), (12, 9)
    counts, nd = O.bin_fixed(X, lo, hi, M)
    c = O.counts_to_c(counts, 2)
    delta = O.bin_width(lo, hi, M)
    L = (M[0] - 1, M[1] - 1)
    f7 = O.conv_direct(c, O.lag_weights(H, delta, L, 60), L)
    f2 = O.bkde_double_sum(c, H, lo, hi, 60)
    assert np.max(np.abs(f7 - f2)) <= 1e-13 * np.max(f2)


def test_single_sample_on_node_is_gaussian():
    """n = 1 on node j1: f_j = K_H(g_j - X_1) for |j - j1| <= L componentwise, 0 outside."""
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    lo, hi, M = np.array([-2.0, -2.0]), np.array([2.0, 2.0]), (41, 41)
    g = O.grid_axes(lo, hi, M)
    j1 = (17, 23)
    X = np.array([[g[0][j1[0]], g[1][j1[1]]]])
    f, info = O.kde_binned(X, H, lo, hi, M)
    L = info["L"]
    mvn = scipy.stats.multivariate_normal(mean=X[0], cov=H)
    for j in itertools.product(range(M[0]), range(M[1])):
        inside = abs(j[0] - j1[0]) <= L[0] and abs(j[1] - j1[1]) <= L[1]
        ref = mvn.pdf([g[0][j[0]], g[1][j[1]]]) if inside else 0.0
        assert f[j] == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_single_sample_off_node_closed_form():
    """n = 1 off node: the 2^d corner weights times shifted kernels (closed form, Eq. 2 + binning)."""
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    lo, hi, M = np.array([0.0, 0.0]), np.array([3.0, 3.0]), (31, 31)   # delta = 0.1
    X = np.array([[1.025, 1.975]])
    f, info = O.kde_binned(X, H, lo, hi, M, L=(30, 30))
    g = O.grid_axes(lo, hi, M)
    u = (X[0] - lo) / 0.1
    j = np.floor(u).astype(int)
    t = u - j
    q = np.rint(t * 2 ** 16) / 2 ** 16
    ref = np.zeros(M)
    G0, G1 = np.meshgrid(g[0], g[1], indexing="ij")
    for b in itertools.product((0, 1), repeat=2):
        wgt = np.prod([q[a] if b[a] else 1 - q[a] for a in range(2)])
        node = [g[0][j[0] + b[0]], g[1][j[1] + b[1]]]
        ref += wgt * scipy.stats.multivariate_normal(mean=node, cov=H).pdf(np.dstack([G0, G1]))
    assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(ref)


def test_total_mass():
    """sum_j f_j prod delta_k ~ 1: exact to Riemann-sum accuracy with the full box,
    and short by at most the normal tail outside the tau = 3.7 ellipse (Eq. 15)."""
    w = W.mix2d_small()
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M)
    mass = f.sum() * np.prod(info["delta"])
    tail = math.exp(-3.7 ** 2 / 2)      # chi^2_2 tail beyond radius 3.7
    assert 1 - tail <= mass <= 1 + 1e-6
    X = np.array([[0.3, -0.2], [0.1, 0.4], [-0.5, 0.0]])
    H = np.array([[0.05, 0.02], [0.02, 0.04]])
    lo, hi, M = np.array([-4.0, -4.0]), np.array([4.0, 4.0]), (161, 161)
    f2, _ = O.kde_binned(X, H, lo, hi, M, L=(160, 160))
    assert f2.sum() * 0.05 * 0.05 == pytest.approx(1.0, abs=1e-9)


def test_translation_by_whole_cells():
    w = W.mix2d_small()
    delta = O.bin_width(w.lo, w.hi, w.M)
    lo, hi = w.lo - 10 * delta, w.hi + 10 * delta
    M = (w.M[0] + 20, w.M[1] + 20)
    f0, i0 = O.kde_binned(w.X, w.H, lo, hi, M, L=(10, 10))
    f1, i1 = O.kde_binned(w.X, w.H, lo - np.array([3, -2]) * i0["delta"],
                          hi - np.array([3, -2]) * i0["delta"], M, L=(10, 10))
    # moving the grid by (-3, +2) cells moves the estimate by (+3, -2) indices
    a, b = f0[3:-5, 5:-2], f1[6:-2, 3:-4]
    assert np.max(np.abs(a - b)) <= 1e-9 * np.max(f0)


# --------------------------------------------------------------------------
# Section 4: the FFT algorithms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_corrected_fft_equals_direct(d):
    """The corrected algorithm (Eq. 12-14) gives Eq. (7) for any H (Section 5)."""
    M = (24, 19, 15)[:d] if d < 4 else (11, 9, 8, 10)
    w = W.small_mixture(seed=d, d=d, n=3000, M=M)
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M)
    g = O.conv_fft_corrected(info["c"], info["k"], info["L"])
    assert np.max(np.abs(f - g)) <= 1e-13 * np.max(f)


def test_corrected_fft_lengths_not_powers_of_two():
    """The corrected layout (Eq. 12-14) is exact for any P_k with no wrap-around at all,
    P_k >= 2 M_k + 2 L_k - 1 (at that odd length and at a 3-smooth one), and still at the
    shortest length that holds the window, P_k = 2 M_k + L_k - 1: the linear convolution
    then wraps only onto indices below the window."""
    w = W.small_mixture(seed=44, d=3, n=3000, M=(14, 11, 9))
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M)
    ML = list(zip(w.M, info["L"]))
    need = tuple(2 * m + 2 * l - 1 for m, l in ML)
    for P in (need, tuple(3 * ((x + 2) // 3) for x in need), tuple(2 * m + l - 1 for m, l in ML)):
        g = O.conv_fft_corrected(info["c"], info["k"], info["L"], P=P)
        assert np.max(np.abs(f - g)) <= 1e-13 * np.max(f), P


def test_corrected_fft_extraction_window_full_box():
    """Eq. (14) window (2M-1):(3M-2) (1-based) with L = M - 1 and P >= 3M - 2."""
    rng = np.random.default_rng(8)
    M = (7, 6)
    c = rng.random(M)
    k = rng.random((13, 11))
    L = (6, 5)
    P = (32, 32)
    k_new = np.zeros(P)
    k_new[:13, :11] = k
    c_new = np.zeros(P)
    c_new[M[0] - 1:2 * M[0] - 1, M[1] - 1:2 * M[1] - 1] = c      # c_11 at 1-based row M1, col M2
    s = np.real(np.fft.ifft2(np.fft.fft2(c_new) * np.fft.fft2(k_new)))
    window = s[2 * M[0] - 2:3 * M[0] - 2, 2 * M[1] - 2:3 * M[1] - 2]
    assert np.allclose(window, O.conv_direct(c, k, L), rtol=1e-12, atol=1e-13)
    assert np.allclose(O.conv_fft_corrected(c, k, L, P), window, rtol=1e-12, atol=1e-13)


def test_wand_ordering_diagonal_ok_full_wrong():
    """Wand's mirrored ordering (Eq. 8) matches Eq. (7) for diagonal H and not for full H (Section 3)."""
    w = W.mix2d_small()
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M)
    wand = O.conv_fft_wand(info["c"], info["k"], info["L"])
    assert np.max(np.abs(wand - f)) >= 0.2 * np.max(f)
    Hd = np.diag(np.diag(w.H))
    fd, infod = O.kde_binned(w.X, Hd, w.lo, w.hi, w.M)
    wandd = O.conv_fft_wand(infod["c"], infod["k"], infod["L"])
    assert np.max(np.abs(wandd - fd)) <= 1e-13 * np.max(fd)
    # and the defective full-H result looks like the diagonal one more than the true one
    assert np.max(np.abs(wand - fd)) < np.max(np.abs(wand - f))


def test_univariate_reduces_to_textbook():
    """d = 1 is the textbook binned estimate: a plain 1-D convolution (np.convolve), and
    Wand's ordering is exact there (Section 4.1)."""
    rng = np.random.default_rng(21)
    X = rng.normal(size=(500, 1))
    H = np.array([[0.09]])
    lo, hi, M = np.array([-4.0]), np.array([4.0]), (200,)
    f, info = O.kde_binned(X, H, lo, hi, M)
    L = info["L"][0]
    ref = np.convolve(info["c"], info["k"])[L:L + M[0]]
    assert np.allclose(f, ref, rtol=1e-13, atol=1e-16)
    assert np.allclose(O.conv_fft_wand(info["c"], info["k"], info["L"]), f, rtol=1e-10, atol=1e-14)


def test_binned_converges_to_eq1():
    """The binned estimate approaches Eq. (1) with O(delta^2) error (Section 2): the error at
    the grid nodes shrinks by a factor of about 4 per halving of delta."""
    w = W.mix2d_small()
    errs = []
    for M in (64, 128, 256):
        f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, (M, M), L=None)
        g = O.grid_axes(w.lo, w.hi, (M, M))
        sub = 8 * (M // 64)   # compare on a common coarse lattice of nodes
        G = np.stack(np.meshgrid(g[0][::sub], g[1][::sub], indexing="ij"), axis=-1).reshape(-1, 2)
        direct = O.kde_direct(w.X, w.H, G).reshape(f[::sub, ::sub].shape)
        errs.append(np.max(np.abs(f[::sub, ::sub] - direct)) / np.max(direct))
    assert errs[0] <= 0.04
    assert 3.0 <= errs[0] / errs[1] <= 5.0
    assert 3.0 <= errs[1] / errs[2] <= 5.0


def test_diagonal_H_4d_is_separable():
    """d = 4 with diagonal H: K_H is the product of four 1-D normal densities, so Eq. (7) is four
    1-D convolutions in turn, each the textbook np.convolve with a scipy normal density."""
    w = W.small_mixture(seed=62, d=4, n=4000, M=(12, 9, 10, 8), diagonal_H=True)
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M)
    L, delta = info["L"], info["delta"]
    g = info["c"] / w.n
    for a in range(4):
        lags = np.arange(-L[a], L[a] + 1) * delta[a]
        ker = scipy.stats.norm(scale=math.sqrt(w.H[a, a])).pdf(lags)
        g = np.apply_along_axis(lambda v: np.convolve(v, ker, mode="full")[L[a]:L[a] + v.size], a, g)
    assert np.max(np.abs(f - g)) <= 1e-13 * np.max(f)


def test_total_mass_4d():
    """sum_j f_j prod delta_k ~ 1 in d = 4, short by at most the normal tail outside the
    tau = 3.7 ellipsoid (chi^2 with 4 degrees of freedom)."""
    w = W.small_mixture(seed=63, d=4, n=3000, M=(24, 24, 24, 24))
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M, method="fft")
    mass = f.sum() * np.prod(info["delta"])
    r2 = 3.7 ** 2
    tail = math.exp(-r2 / 2) * (1 + r2 / 2)          # P(chi^2_4 > r^2)
    assert 1 - tail - 1e-3 <= mass <= 1 + 1e-3


# --------------------------------------------------------------------------
# planted mistakes must trip the pins
# --------------------------------------------------------------------------

def _weights_ok(fn):
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    delta = np.array([0.11, 0.07])
    L = (4, 5)
    k = fn(H, delta, L, 37)
    mvn = scipy.stats.multivariate_normal(mean=np.zeros(2), cov=H)
    ref = np.array([[mvn.pdf(np.array([a, b]) * delta) / 37 for b in range(-5, 6)] for a in range(-4, 5)])
    return np.allclose(k, ref, rtol=1e-12, atol=0)


def _conv_ok(fn):
    rng = np.random.default_rng(11)
    c = rng.random((9, 14))
    k = rng.random((7, 11))
    full = scipy.signal.convolve(c, k, mode="full", method="direct")
    return np.allclose(fn(c, k, (3, 5)), full[3:12, 5:19], rtol=1e-13, atol=1e-13)


def _binning_ok(fn):
    X = np.array([[0.1, 2.0], [1.0 + 3.0 / 2 ** 17, 0.0], [1.0 + 5.0 / 2 ** 17, 1.0], [3.0, 3.0]])
    counts, _ = fn(X, [0.0, 0.0], [3.0, 3.0], (4, 4))
    one = 2 ** 16
    return (int(counts[0, 2]) == (one - 6554) * one and int(counts[1, 0]) == (one - 2) * one
            and int(counts[1, 1]) == (one - 2) * one and int(counts[3, 3]) == one * one)


def test_planted_mistakes_are_caught():
    assert _weights_ok(O.lag_weights) and _conv_ok(O.conv_direct) and _binning_ok(O.bin_fixed)

    def w_H_not_inverse(H, delta, L, n):          # uses H where H^-1 belongs
        return O.lag_weights(np.linalg.inv(H), delta, L, n) * np.sqrt(np.linalg.det(np.linalg.inv(H))) \
            / np.sqrt(np.linalg.det(H))

    def w_no_2pi(H, delta, L, n):                 # drops the (2 pi)^-d/2 factor
        return O.lag_weights(H, delta, L, n) * (2 * np.pi)

    def w_mirrored(H, delta, L, n):               # Wand's mirrored negative lags
        k = O.lag_weights(H, delta, L, n)
        k[:L[0], :] = k[L[0] + 1:, :][::-1, :]
        return k

    def w_transposed(H, delta, L, n):             # delta applied to the wrong axes
        return O.lag_weights(H, delta[::-1], L, n)

    for bad in (w_H_not_inverse, w_no_2pi, w_mirrored, w_transposed):
        assert not _weights_ok(bad), bad.__name__

    def c_sign(c, k, L):                          # c_{j+l} instead of c_{j-l}
        return O.conv_direct(c, k[::-1, ::-1], L)

    def c_transposed(c, k, L):                    # lag box axes swapped
        kk = np.zeros_like(k)
        m = min(k.shape)
        kk[:m, :m] = k[:m, :m].T
        return O.conv_direct(c, kk, L)

    for bad in (c_sign, c_transposed):
        assert not _conv_ok(bad), bad.__name__

    def b_floor(X, lo, hi, M, Q=None):            # truncation instead of round-to-nearest-even
        X = np.asarray(X, float)
        counts = np.zeros(M, dtype=np.uint64)
        delta = O.bin_width(lo, hi, M)
        u = (X - np.asarray(lo)) / delta
        j = np.minimum(np.floor(u), np.asarray(M) - 2.0)
        q = np.floor((u - j) * 2 ** 16).astype(np.uint64)
        one = np.uint64(2 ** 16)
        for b in itertools.product((0, 1), repeat=2):
            wgt = (q[:, 0] if b[0] else one - q[:, 0]) * (q[:, 1] if b[1] else one - q[:, 1])
            np.add.at(counts, (j[:, 0].astype(int) + b[0], j[:, 1].astype(int) + b[1]), wgt)
        return counts, 0

    def b_round_half_up(X, lo, hi, M, Q=None):    # ties away from zero
        X = np.asarray(X, float)
        counts = np.zeros(M, dtype=np.uint64)
        delta = O.bin_width(lo, hi, M)
        u = (X - np.asarray(lo)) / delta
        j = np.minimum(np.floor(u), np.asarray(M) - 2.0)
        q = np.floor((u - j) * 2 ** 16 + 0.5).astype(np.uint64)
        one = np.uint64(2 ** 16)
        for b in itertools.product((0, 1), repeat=2):
            wgt = (q[:, 0] if b[0] else one - q[:, 0]) * (q[:, 1] if b[1] else one - q[:, 1])
            np.add.at(counts, (j[:, 0].astype(int) + b[0], j[:, 1].astype(int) + b[1]), wgt)
        return counts, 0

    for bad in (b_floor, b_round_half_up):
        assert not _binning_ok(bad), bad.__name__


def test_marginal_extent_is_the_ellipsoid_bounding_box():
    """tau sqrt(H_kk) is the largest |u_k| on the ellipsoid u' H^-1 u = tau^2 (found here by
    dense sampling of its boundary), and it never exceeds the Eq. (15) half width."""
    rng = np.random.default_rng(77)
    for d in (2, 3):
        H = W.random_spd(rng, d, ratio=(1.0, 20.0))
        tau = 3.7
        V = rng.normal(size=(200_000, d))
        V /= np.linalg.norm(V, axis=1, keepdims=True)
        U = tau * V @ np.linalg.cholesky(H).T          # u' H^-1 u = tau^2 for every row
        box = np.max(np.abs(U), axis=0)
        assert np.allclose(box, tau * np.sqrt(np.diag(H)), rtol=2e-3)
        delta = np.full(d, 0.05)
        Le = O.truncation_L(H, delta, (1000,) * d, tau)
        Lm = O.truncation_L(H, delta, (1000,) * d, tau, extent="marginal")
        assert all(m <= e for m, e in zip(Lm, Le)) and any(m < e for m, e in zip(Lm, Le))
