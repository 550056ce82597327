"""Host-side checks of the C ABI (no device work): the library loads, exports
every function include/kde.h declares, and its FP64 planner agrees with the
oracle on delta (Eq. 4), lambda_max and L (Eq. 15), |H| and k_0 (Eq. 6), and
rejects invalid problems with the documented status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1508_02766_amd as K
import workloads as W
from paper_1508_02766_amd import kde as KB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "kde.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kde_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = K.lib()
    declared = _header_functions()
    assert declared == sorted(K.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_strerror():
    assert K.kde_strerror(0) == "ok"
    for code in (-1, -2, -3, -4, -5, -6):
        assert K.kde_strerror(code) != "unknown status"
    assert K.kde_strerror(-99) == "unknown status"


@pytest.mark.parametrize("name", ["mix2d_small", "mix2d_512", "mix3d_128"])
def test_plan_matches_oracle(name):
    w = W.WORKLOADS[name]()
    plan = K.kde_plan_query(w.H, w.n, (w.lo, w.hi, w.M))
    op = O.plan(w.H, w.lo, w.hi, w.M, w.n)
    assert plan["L"] == op["L"]
    assert np.allclose(plan["delta"], op["delta"], rtol=0, atol=0)
    assert plan["lambda_max"] == pytest.approx(O.lambda_max(w.H), rel=1e-13)
    assert plan["det_H"] == pytest.approx(np.linalg.det(w.H), rel=1e-12)
    k0 = O.lag_weights(w.H, op["delta"], (0,) * w.d, w.n).ravel()[0]
    assert plan["norm"] == pytest.approx(k0, rel=1e-13)
    for k in range(w.d):
        P = plan["P"][k]
        assert P >= w.M[k] + plan["L"][k] and P >= 16 and P & (P - 1) == 0 and P // 2 < max(16, w.M[k] + plan["L"][k])


def test_plan_random_spd_matches_oracle():
    rng = np.random.default_rng(4)
    for trial in range(200):
        d = int(rng.integers(1, 4))
        H = W.random_spd(rng, d, lam_min=(0.01, 0.5), ratio=(1.0, 50.0))
        M = tuple(int(m) for m in rng.integers(2, 200, size=d))
        lo = rng.uniform(-5, 0, size=d)
        hi = lo + rng.uniform(0.5, 10, size=d)
        n = int(rng.integers(1, 10 ** 6))
        plan = K.kde_plan_query(H, n, (lo, hi, M))
        op = O.plan(H, lo, hi, M, n)
        assert plan["L"] == op["L"], (trial, plan["L"], op["L"])
        assert plan["lambda_max"] == pytest.approx(O.lambda_max(H), rel=1e-12)


def test_plan_binning_only():
    """With H = NULL the planner fills the binning quantities and accepts n = 0."""
    g = ([-1.0, -1.0], [1.0, 1.0], [512, 512])
    p = K.kde_plan_query(None, 10 ** 6, g)
    assert p["Q"] == 16 and p["bin_ws_bytes"] > 8 * 4 * 10 ** 6 and p["L"] == (0, 0)
    assert K.kde_plan_query(None, 0, g)["bin_ws_bytes"] == 0
    # Q too large for a 64-bit record falls back to atomics: no workspace
    assert K.kde_plan_query(None, 10, g, Q=30)["bin_ws_bytes"] == 0


def test_plan_overrides_and_precision():
    w = W.mix2d_small()
    g = (w.lo, w.hi, w.M)
    p = K.kde_plan_query(w.H, w.n, g, L=(5, 63), prec="f64", Q=12, tau=2.0)
    assert p["L"] == (5, 63) and p["P"] == (128, 128) and p["prec"] == 2 and p["Q"] == 12
    assert p["lag_bytes"] == 11 * 127 * 8
    p = K.kde_plan_query(w.H, w.n, g, tau=2.0)
    assert p["L"] == O.truncation_L(w.H, O.bin_width(w.lo, w.hi, w.M), w.M, 2.0)


def _code(H, n, grid, **opts):
    try:
        K.kde_plan_query(H, n, grid, **opts)
    except K.KdeError as e:
        return e.code
    return 0


def test_plan_errors():
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    good = ([-1.0, -1.0], [1.0, 1.0], [32, 32])
    assert _code(H, 10, good) == 0
    assert _code(H, 0, good) == -1                                   # n < 1
    assert _code(H, 10, ([-1, -1], [1, 1], [1, 32])) == -1             # M < 2
    assert _code(H, 10, ([1, -1], [1, 1], [32, 32])) == -1             # hi == lo
    assert _code(H, 10, ([np.nan, -1], [1, 1], [32, 32])) == -1        # non-finite box
    assert _code(H, 10, good, L=(32, 1)) == -1                         # L > M - 1
    assert _code(H, 10, good, prec=3) == -1                            # bad precision
    assert _code(H, 10, good, Q=40) == -1                              # d Q > 62
    assert _code(np.array([[0.09, 0.07], [0.06, 0.08]]), 10, good) == -2   # asymmetric
    assert _code(np.array([[0.09, 0.2], [0.2, 0.08]]), 10, good) == -2     # indefinite
    assert _code(np.array([[0.09, np.inf], [np.inf, 0.08]]), 10, good) == -2
    assert _code(np.zeros((2, 2)), 10, good) == -2
    assert _code(H, 2 ** 33, good) == -3                               # n 2^32 overflows
    assert _code(H, 10, ([-1, -1], [1, 1], [4000, 32])) == -5          # P > 4096
    g4 = K.make_grid([0.0] * 3, [1.0] * 3, [4] * 3)
    g4.d = 4                                                           # d outside {1, 2, 3}
    out = KB.KdePlan()
    H4 = np.eye(4).ctypes.data_as(ctypes.c_void_p)
    assert K.lib().kde_plan_query(H4, 10, ctypes.byref(g4), None, ctypes.byref(out)) == -1


def test_device_entry_points_reject_before_enqueue():
    """Invalid arguments return before any HIP call, so these run without a GPU."""
    lib = K.lib()
    g = K.make_grid([-1.0, -1.0], [1.0, 1.0], [32, 32])
    bad = K.make_grid([-1.0, -1.0], [1.0, 1.0], [1, 32])
    p = KB.KdeParams()
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    Hp = H.ctypes.data_as(ctypes.c_void_p)
    null = ctypes.c_void_p(0)
    assert lib.kde_bin(null, 10, ctypes.byref(bad), ctypes.byref(p), ctypes.c_void_p(8), null, null, 0, null) == -1
    assert lib.kde_bin(null, 10, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(8), null, null, 0, null) == -1
    # the tiled binning needs its workspace: missing / misaligned / too small
    assert lib.kde_bin(ctypes.c_void_p(8), 10, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(8), null, null, 0,
                       null) == -1
    assert lib.kde_bin(ctypes.c_void_p(8), 10, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(8), null,
                       ctypes.c_void_p(100), 1 << 30, null) == -1
    assert lib.kde_bin(ctypes.c_void_p(8), 10, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(8), null,
                       ctypes.c_void_p(256), 16, null) == -4
    assert lib.kde_eval(ctypes.c_void_p(8), 0, Hp, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(8),
                        ctypes.c_void_p(256), 1 << 30, null, null) == -1      # n = 0
    assert lib.kde_eval(ctypes.c_void_p(8), 10, Hp, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(8),
                        ctypes.c_void_p(256), 16, null, null) == -4           # workspace too small
    assert lib.kde_conv(ctypes.c_void_p(8), 10, Hp, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(8),
                        ctypes.c_void_p(100), 1 << 30, null) == -1            # misaligned workspace
    assert lib.kde_kernel_grid(Hp, 10, ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(8), 4, null) == -4
