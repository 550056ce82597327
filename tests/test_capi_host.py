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
        assert plan["P"][k] == _padded_length(w.M[k] + plan["L"][k], w.d)


# Padded lengths (highly composite, Section 4.1): 2^k in [16, 4096], and in 3-D and 4-D
# also 3 x 2^k in [48, 3072].
def _padded_length(need: int, d: int) -> int:
    """The shortest admissible length that holds M_k + L_k (the window and the lags of
    the circular layout)."""
    lengths = [2 ** k for k in range(4, 13)] + ([3 * 2 ** k for k in range(4, 11)] if d >= 3 else [])
    return min(P for P in lengths if P >= need)


def test_plan_random_spd_matches_oracle():
    rng = np.random.default_rng(4)
    for trial in range(200):
        d = int(rng.integers(1, 5))
        H = W.random_spd(rng, d, lam_min=(0.01, 0.5), ratio=(1.0, 50.0))
        M = tuple(int(m) for m in rng.integers(2, 200, size=d))
        lo = rng.uniform(-5, 0, size=d)
        hi = lo + rng.uniform(0.5, 10, size=d)
        n = int(rng.integers(1, 10 ** 6))
        plan = K.kde_plan_query(H, n, (lo, hi, M))
        op = O.plan(H, lo, hi, M, n)
        assert plan["L"] == op["L"], (trial, plan["L"], op["L"])
        assert plan["P"] == tuple(_padded_length(m + l, d) for m, l in zip(M, plan["L"]))
        assert plan["lambda_max"] == pytest.approx(O.lambda_max(H), rel=1e-12)


def test_plan_4d_matches_oracle():
    """d = 4: Eq. (15) with lambda_max from the cyclic Jacobi rotations, |H|, k_0, the default
    8^4 binning tile (record: 4 x 9 fraction bits + 4 x 4 corner bits) and a workspace."""
    w = W.small_mixture(seed=70, d=4, n=20_000, M=(24, 20, 18, 30))
    plan = K.kde_plan_query(w.H, w.n, (w.lo, w.hi, w.M))
    op = O.plan(w.H, w.lo, w.hi, w.M, w.n)
    assert plan["d"] == 4 and plan["Q"] == 8 and plan["L"] == op["L"]
    assert plan["lambda_max"] == pytest.approx(np.linalg.eigvalsh(w.H)[-1], rel=1e-13)
    assert plan["det_H"] == pytest.approx(np.linalg.det(w.H), rel=1e-12)
    k0 = O.lag_weights(w.H, op["delta"], (0,) * 4, w.n).ravel()[0]
    assert plan["norm"] == pytest.approx(k0, rel=1e-13)
    assert plan["bin_ws_bytes"] > 0 and plan["conv_ws_bytes"] > 0
    assert plan["lag_count"] == np.prod([2 * l + 1 for l in op["L"]])


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


@pytest.mark.parametrize("d,M", [(2, (80, 60)), (3, (20, 24, 18)), (4, (10, 12, 8, 9))])
def test_plan_stored_spectrum_workspace(d, M):
    """A stored spectrum adds P_1 .. P_(d-1) x pitch(P_d) reals (pitch: P/2 + 1 rounded up to 16)
    of the precision to the convolution workspace and changes nothing else of the plan."""
    w = W.small_mixture(400 + d, d, 5_000, M)
    g = (w.lo, w.hi, w.M)
    for prec, rs in (("f32", 4), ("f64", 8)):
        a = K.kde_plan_query(w.H, w.n, g, prec=prec)
        b = K.kde_plan_query(w.H, w.n, g, prec=prec, store_spectrum=True)
        pitch = (a["P"][-1] // 2 + 1 + 15) // 16 * 16
        extra = int(np.prod(a["P"][:-1])) * pitch * rs
        assert b["conv_ws_bytes"] - a["conv_ws_bytes"] == (extra + 255) // 256 * 256
        assert b["eval_ws_bytes"] - a["eval_ws_bytes"] == b["conv_ws_bytes"] - a["conv_ws_bytes"]
        assert a["L"] == b["L"] and a["P"] == b["P"] and a["bin_ws_bytes"] == b["bin_ws_bytes"]
    one = W.small_mixture(410, 1, 5_000, (300,))
    g1 = (one.lo, one.hi, one.M)
    assert K.kde_plan_query(one.H, one.n, g1, store_spectrum=True) == K.kde_plan_query(one.H, one.n, g1)


def test_plan_length_options():
    """kde_params.lengths: 0 = 2^k (3 x 2^k in 3-D and 4-D where shorter), 1 = 3 x 2^k also
    in 2-D, 2 = 2^k only; other values are rejected."""
    w2, w3 = W.mix2d_512(n=10_000), W.mix3d_128(n=10_000)
    for w, auto, comp, pow2 in ((w2, (1024, 1024), (768, 768), (1024, 1024)),
                                (w3, (192, 192, 192), (192, 192, 192), (256, 256, 256))):
        g = (w.lo, w.hi, w.M)
        assert K.kde_plan_query(w.H, w.n, g)["P"] == auto
        assert K.kde_plan_query(w.H, w.n, g, lengths="composite")["P"] == comp
        assert K.kde_plan_query(w.H, w.n, g, lengths="pow2")["P"] == pow2
    one = W.small_mixture(411, 1, 5_000, (300,))
    assert K.kde_plan_query(one.H, one.n, (one.lo, one.hi, one.M), lengths="composite")["P"] == (512,)
    assert _code(w2.H, w2.n, (w2.lo, w2.hi, w2.M), lengths=3) == -1


def test_stored_spectrum_rejections():
    """store_spectrum takes 0 or 1, and batches refuse it."""
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    good = ([-1.0, -1.0], [1.0, 1.0], [32, 32])
    p = KB.KdeParams()
    p.store_spectrum = 2
    out = KB.KdePlan()
    Hc = (ctypes.c_double * 4)(*H.ravel())
    assert K.lib().kde_plan_query(Hc, 10, ctypes.byref(K.make_grid(*good)), ctypes.byref(p), ctypes.byref(out)) == -1
    ok = _batch_items([(1000, H.tolist(), ((-3, -3), (3, 3), (64, 64)))])
    q = KB.KdeParams()
    q.store_spectrum = 1
    assert _batch_info(ok, q)[0] == -1


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
    g5 = K.make_grid([0.0] * 4, [1.0] * 4, [4] * 4)
    g5.d = 5                                                           # d outside {1, 2, 3, 4}
    out = KB.KdePlan()
    H5 = np.eye(5)
    assert K.lib().kde_plan_query(H5.ctypes.data_as(ctypes.c_void_p), 10, ctypes.byref(g5), None,
                                  ctypes.byref(out)) == -1


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


# --------------------------------------------------------------------------
# batched planning (kde_batch_create / _query / _destroy do no device work)
# --------------------------------------------------------------------------

def _batch_items(probs):
    """ctypes items with placeholder device addresses (never dereferenced on the host)."""
    arr = (KB.KdeBatchItem * len(probs))()
    for i, (n, H, grid) in enumerate(probs):
        g = KB.make_grid(*grid)
        arr[i].X = 0x10000 + i * 0x1000
        arr[i].n = n
        Hn = np.asarray(H, dtype=np.float64).reshape(g.d, g.d)
        for a in range(g.d):
            for b in range(g.d):
                arr[i].H[a * g.d + b] = Hn[a, b]
        arr[i].grid = g
        arr[i].density = 0x90000 + i * 0x1000
    return arr


def _batch_info(arr, params=None):
    lib = K.lib()
    h = ctypes.c_void_p()
    rc = lib.kde_batch_create(arr, len(arr), ctypes.byref(params) if params is not None else None, ctypes.byref(h))
    if rc != 0:
        return rc, None
    info = KB.KdeBatchInfo()
    assert lib.kde_batch_query(h, ctypes.byref(info)) == 0
    assert lib.kde_batch_eval(h, None) == -1          # not bound: rejected before any HIP call
    lib.kde_batch_destroy(h)
    return 0, info


def test_batch_plan_sizes_and_launch_count():
    H2 = [[0.09, 0.06], [0.06, 0.08]]
    probs = [(1000, H2, ((-3, -3), (3, 3), (64, 64))), (250_000, H2, ((-3, -3), (3, 3), (64, 64))),
             (40_000, H2, ((-4, -3), (4, 3), (128, 128)))]
    rc, info = _batch_info(_batch_items(probs))
    assert rc == 0 and info.count == 3
    need = sum(K.kde_plan_query(H, n, g)["eval_ws_bytes"] for n, H, g in probs)
    assert info.ws_bytes >= need
    assert info.launches == 4 + 4 * 2                 # two padded lengths (128, 256)
    # d = 1, 2, 3 together: one launch per (pass, template) group
    probs = [(5000, [[0.2]], ((-3,), (3,), (300,))), (5000, H2, ((-3, -3), (3, 3), (64, 64))),
             (5000, np.eye(3) * 0.3, ((-3,) * 3, (3,) * 3, (20, 20, 20)))]
    rc, info = _batch_info(_batch_items(probs))
    assert rc == 0
    # binning 4 per d; d=1: kspec, counts, product; d=2: kspec, counts, conv, c2r;
    # d=3: kspec_r2c, kspec_col2, counts_r2c, counts_col2, conv_col1, inv_col2, c2r
    assert info.launches == 12 + 3 + 4 + 7


def test_batch_plan_errors():
    H2 = [[0.09, 0.06], [0.06, 0.08]]
    lib = K.lib()
    h = ctypes.c_void_p()
    ok = _batch_items([(1000, H2, ((-3, -3), (3, 3), (64, 64)))])
    assert lib.kde_batch_create(ok, 0, None, ctypes.byref(h)) == -1
    assert lib.kde_batch_create(None, 1, None, ctypes.byref(h)) == -1
    assert lib.kde_batch_create(ok, 1, None, None) == -1
    bad = _batch_items([(1000, H2, ((-3, -3), (3, 3), (64, 64))), (1000, [[1, 2], [2, 1]], ((-3, -3), (3, 3), (64, 64)))])
    assert _batch_info(bad)[0] == -2
    noX = _batch_items([(1000, H2, ((-3, -3), (3, 3), (64, 64)))])
    noX[0].X = 0
    assert _batch_info(noX)[0] == -1
    zero_n = _batch_items([(0, H2, ((-3, -3), (3, 3), (64, 64)))])
    assert _batch_info(zero_n)[0] == -1
    p = KB.KdeParams()
    p.tile[0], p.tile[1] = 48, 32                     # not a power of two
    assert _batch_info(ok, p)[0] == -1
    p.tile[0], p.tile[1] = 128, 64                    # 8192 cells
    assert _batch_info(ok, p)[0] == -1
    p.tile[0], p.tile[1] = 16, 64
    rc, info = _batch_info(ok, p)
    assert rc == 0 and tuple(info.tile) == (16, 64, 0, 0)
    assert lib.kde_batch_query(None, ctypes.byref(KB.KdeBatchInfo())) == -1


def test_tile_override_in_plan():
    H2 = [[0.09, 0.06], [0.06, 0.08]]
    g = ((-3, -3), (3, 3), (512, 512))
    base = K.kde_plan_query(None, 100_000, g)["bin_ws_bytes"]
    wide = K.kde_plan_query(None, 100_000, g, tile=(64, 64))["bin_ws_bytes"]
    assert base > 0 and wide > 0 and wide != base
    with pytest.raises(K.KdeError):
        K.kde_plan_query(H2, 1000, g, tile=(3, 32))


def test_lscv_plan_and_rejections():
    lib = K.lib()
    H2 = [[0.09, 0.06], [0.06, 0.08]]
    g = ((-3, -3), (3, 3), (64, 64))
    p = K.kde_plan_query(H2, 1000, g)
    assert p["lscv_ws_bytes"] > p["density_bytes"]
    assert K.kde_plan_query(H2, 1, g)["lscv_ws_bytes"] == 0
    grid = KB.make_grid(*g)
    Hn = np.ascontiguousarray(np.array(H2, dtype=np.float64))
    Hp = Hn.ctypes.data_as(ctypes.c_void_p)
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)
    need = p["lscv_ws_bytes"]
    call = lambda counts, n, H, out, wsp, nbytes: lib.kde_lscv(counts, n, H, ctypes.byref(grid), None, out, wsp,
                                                                nbytes, None)
    assert call(fake, 1, Hp, fake, ws, need) == -1           # n < 2
    assert call(None, 1000, Hp, fake, ws, need) == -1        # no counts
    assert call(fake, 1000, Hp, None, ws, need) == -1        # no output
    assert call(fake, 1000, Hp, fake, ctypes.c_void_p(0x200010), need) == -1   # misaligned workspace
    assert call(fake, 1000, Hp, fake, ws, need - 1) == -4    # workspace too small
    bad = np.ascontiguousarray(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert call(fake, 1000, bad.ctypes.data_as(ctypes.c_void_p), fake, ws, need) == -2


def test_search_helpers_on_host():
    from paper_1508_02766_amd import lscv as S
    rng = np.random.default_rng(3)
    for d in (1, 2, 3):
        H = W.random_spd(rng, d)
        assert np.allclose(S.from_theta(S.to_theta(H), d), H, rtol=1e-13, atol=1e-15)
    a = np.array([0.5, -0.7, 1.5])
    gen = S.nelder_mead(np.zeros(3), iters=400, tol=1e-15)
    x = next(gen)
    try:
        while True:
            x = gen.send(float(np.sum((x - a) ** 2)) + 2.0)
    except StopIteration as stop:
        xb, vb, evals = stop.value
    assert np.allclose(xb, a, atol=1e-5) and abs(vb - 2.0) < 1e-9 and evals > 10
    # smallest eigenvalue of the admissibility test (closed form for 2 x 2) against LAPACK
    for d in (1, 2, 3):
        for _ in range(200):
            H = W.random_spd(rng, d, ratio=(1.0, 50.0))
            assert abs(S._min_eig(H) - np.linalg.eigvalsh(H)[0]) <= 1e-12 * np.abs(H).max()
    # one plan query gives both the admissibility and phi_H(0) = n k_0 of the library
    g = ((-3.0, -3.0), (3.0, 3.0), (256, 256))
    H = np.array([[0.05, 0.01], [0.01, 0.04]])
    ok, f0 = S._admissible_phi0(H, 5000, g, {})
    assert ok and f0 == K.kde_plan_query(H, 5000, g)["norm"] * 5000
    assert not S._admissible_phi0(H * 1e-6, 5000, g, {})[0]


def test_plan_marginal_extent_matches_oracle():
    rng = np.random.default_rng(78)
    for d in (1, 2, 3):
        H = W.random_spd(rng, d, ratio=(1.0, 20.0))
        M = (70, 50, 40)[:d]
        lo, hi = -np.ones(d) * 3, np.ones(d) * 3
        p = K.kde_plan_query(H, 1000, (lo, hi, M), extent="marginal")
        ref = O.truncation_L(H, O.bin_width(lo, hi, M), M, extent="marginal")
        assert tuple(p["L"]) == ref
    with pytest.raises(K.KdeError):
        K.kde_plan_query(np.eye(2), 10, ((-1, -1), (1, 1), (8, 8)), extent=2)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more, it says so and exits with status 2
    before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_counter_record_names_the_sources():
    """The committed HBM byte counters carry the hash of the device sources they were taken
    with; bench.py reports them only while that hash matches (else traffic is null)."""
    import bench
    import json
    with open(bench.COUNTERS) as fh:
        c = json.load(fh)
    assert len(c["source_sha256"]) == 64
    for wl in ("mix2d_512", "mix3d_128"):
        cal = c["copy_calibration"][wl]
        assert 1.5 < cal["fetch_factor"] < 2.5 and 0.5 < cal["write_factor"] < 1.5
        assert all(k["FETCH_SIZE"] > 0 for k in c["workloads"][wl].values())
    if c["source_sha256"] == bench.kernel_source_hash():
        assert bench.measured_traffic("mix2d_512", "bin_scatter") > 0
    else:
        assert bench.measured_traffic("mix2d_512", "bin_scatter") is None


# --------------------------------------------------------------------------
# grid rule (Eq. 3-4 with the data-range reading) and batched LSCV planning
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["mix2d_small", "mix2d_512", "mix3d_128"])
def test_grid_from_data_matches_workload_boxes(name):
    """The library's grid rule reproduces the boxes the workloads use, bit for bit."""
    w = W.WORKLOADS[name]()
    g = K.kde_grid_from_data(w.X, w.H, w.M[0], 3.0)
    lo, hi, M = K.grid_tuple(g)
    assert np.array_equal(lo, w.lo) and np.array_equal(hi, w.hi) and M == tuple(w.M)


def test_grid_from_data_hand_values():
    X = np.array([[0.0, 1.0], [2.0, -1.0], [1.0, 5.0], [np.nan, 100.0], [1.0, np.inf]])
    H = np.array([[0.25, 0.1], [0.1, 4.0]])
    lo, hi, M = K.grid_tuple(K.kde_grid_from_data(X, H, 40, 2.0))
    # non-finite samples ignored; sqrt(H_kk) = 0.5 and 2, times 2
    assert np.array_equal(lo, [0.0 - 1.0, -1.0 - 4.0]) and np.array_equal(hi, [2.0 + 1.0, 5.0 + 4.0])
    assert M == (40, 40)
    lo, hi, _ = K.grid_tuple(K.kde_grid_from_data(X[:3, :1], [[0.04]], 8, 0.0))
    assert lo[0] == 0.0 and hi[0] == 2.0
    # d = 4: sqrt(H_kk) = 0.5, 1, 2, 0.25 (off-diagonal entries do not enter), times 3
    X4 = np.array([[0.0, 1.0, -2.0, 3.0], [1.0, -1.0, 2.0, 3.5], [0.5, 0.0, 0.0, 2.0]])
    H4 = np.diag([0.25, 1.0, 4.0, 0.0625])
    H4[0, 1] = H4[1, 0] = 0.1
    lo, hi, M = K.grid_tuple(K.kde_grid_from_data(X4, H4, 24, 3.0))
    assert np.array_equal(lo, [-1.5, -4.0, -8.0, 1.25]) and np.array_equal(hi, [2.5, 4.0, 8.0, 4.25])
    assert M == (24, 24, 24, 24)


def test_grid_from_data_errors():
    lib = K.lib()
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    X = np.array([[0.0, 1.0], [2.0, -1.0]])
    Xp, Hp = X.ctypes.data_as(ctypes.c_void_p), H.ctypes.data_as(ctypes.c_void_p)
    g = KB.KdeGrid()
    call = lambda Xq, n, d, Hq, nsd, M, out: lib.kde_grid_from_data(Xq, n, d, Hq, nsd, M, out)
    assert call(Xp, 2, 2, Hp, 3.0, 64, ctypes.byref(g)) == 0 and g.d == 2
    assert call(None, 2, 2, Hp, 3.0, 64, ctypes.byref(g)) == -1          # no samples
    assert call(Xp, 0, 2, Hp, 3.0, 64, ctypes.byref(g)) == -1            # n < 1
    assert call(Xp, 2, 5, Hp, 3.0, 64, ctypes.byref(g)) == -1            # d outside {1, 2, 3, 4}
    assert call(Xp, 2, 2, Hp, 3.0, 1, ctypes.byref(g)) == -1             # M < 2
    assert call(Xp, 2, 2, Hp, -1.0, 64, ctypes.byref(g)) == -1           # negative nsd
    assert call(Xp, 2, 2, Hp, float("nan"), 64, ctypes.byref(g)) == -1
    assert call(Xp, 2, 2, Hp, 3.0, 64, None) == -1
    one = np.array([[1.0, 1.0]])
    assert call(one.ctypes.data_as(ctypes.c_void_p), 1, 2, Hp, 0.0, 64, ctypes.byref(g)) == -1   # hi == lo
    nanX = np.full((3, 2), np.nan)
    assert call(nanX.ctypes.data_as(ctypes.c_void_p), 3, 2, Hp, 3.0, 64, ctypes.byref(g)) == -1  # no finite sample
    bad = np.array([[0.09, 0.2], [0.2, 0.08]])
    assert call(Xp, 2, 2, bad.ctypes.data_as(ctypes.c_void_p), 3.0, 64, ctypes.byref(g)) == -2


def _lscv_items(probs):
    arr = (KB.KdeLscvItem * len(probs))()
    for i, (n, H, grid) in enumerate(probs):
        g = KB.make_grid(*grid)
        arr[i].counts = 0x10000 + i * 0x1000
        arr[i].n = n
        Hn = np.asarray(H, dtype=np.float64).reshape(g.d, g.d)
        arr[i].H[:g.d * g.d] = Hn.ravel().tolist()
        arr[i].grid = g
        arr[i].out = 0x90000 + i * 0x100
    return arr


def test_lscv_batch_plan_and_errors():
    lib = K.lib()
    H2 = [[0.09, 0.06], [0.06, 0.08]]
    g64, g128 = ((-3, -3), (3, 3), (64, 64)), ((-3, -3), (3, 3), (128, 128))
    arr = _lscv_items([(1000, H2, g64), (5000, H2, g128), (2000, np.array(H2) * 2, g64)])
    h = ctypes.c_void_p()
    assert lib.kde_lscv_batch_create(arr, 3, None, ctypes.byref(h)) == 0
    info = KB.KdeBatchInfo()
    assert lib.kde_batch_query(h, ctypes.byref(info)) == 0
    # two convolutions per problem: the workspace holds at least each problem's kde_lscv workspace
    need = sum(K.kde_plan_query(H, n, g)["lscv_ws_bytes"] for n, H, g in [(1000, H2, g64), (5000, H2, g128)])
    assert info.count == 6 and info.ws_bytes >= need
    assert lib.kde_batch_eval(h, None) == -1          # not bound
    lib.kde_batch_destroy(h)
    assert lib.kde_lscv_batch_create(arr, 0, None, ctypes.byref(h)) == -1
    assert lib.kde_lscv_batch_create(None, 1, None, ctypes.byref(h)) == -1
    one = _lscv_items([(1, H2, g64)])                  # n < 2
    assert lib.kde_lscv_batch_create(one, 1, None, ctypes.byref(h)) == -1
    nocounts = _lscv_items([(1000, H2, g64)])
    nocounts[0].counts = 0
    assert lib.kde_lscv_batch_create(nocounts, 1, None, ctypes.byref(h)) == -1
    noout = _lscv_items([(1000, H2, g64)])
    noout[0].out = 0
    assert lib.kde_lscv_batch_create(noout, 1, None, ctypes.byref(h)) == -1
    bad = _lscv_items([(1000, H2, g64), (1000, [[1, 2], [2, 1]], g64)])
    assert lib.kde_lscv_batch_create(bad, 2, None, ctypes.byref(h)) == -2
