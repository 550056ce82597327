"""Parity of the gfx950 path (through the C ABI) with the FP64 oracle.

Bars: grid counts bit-exact (integer fixed point); lag weights within 2e-6 of
k_0 in FP32 and 1e-14 in FP64; densities within 1e-5 of the grid maximum in
FP32 and 1e-12 in FP64. Sizes span several FFT tiles with ragged tails; the
full-size workloads are compared on every cell (2-D against the direct sum,
3-D against the oracle's FFT form of Eq. 7), the 3-D one also on sampled grid
points the oracle evaluates one by one.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1508_02766_amd as K
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}
DEV = "cuda:0"


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device=DEV)


def _counts(X, lo, hi, M, **opts):
    c, nd = K.kde_bin(_dev(X), (lo, hi, M), **opts)
    torch.cuda.synchronize()
    return c.cpu().numpy(), int(nd.cpu().numpy()[0])


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# --------------------------------------------------------------------------
# binning: bit-exact
# --------------------------------------------------------------------------

def test_bin_hand_cases_bit_exact():
    X = np.array([[1.0, 1.0], [1.5, 2.5], [3.0, 3.0], [0.25, 0.0], [0.1, 2.0], [1.0 + 3.0 / 2 ** 17, 0.0],
                  [1.0 + 5.0 / 2 ** 17, 1.0], [-0.1, 1.0], [1.0, 3.0000000001], [np.nan, 1.0], [np.inf, 0.0],
                  [0.0, 0.0], [2.9999999999999996, 0.5]])
    ref, rnd = O.bin_fixed(X, [0.0, 0.0], [3.0, 3.0], (4, 4))
    got, gnd = _counts(X, [0.0, 0.0], [3.0, 3.0], (4, 4))
    assert gnd == rnd == 4
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", ["mix2d_small", "mix2d_512", "mix3d_128", "mix4d_48"])
def test_bin_workloads_bit_exact(name):
    w = W.WORKLOADS[name]()
    ref, rnd = O.bin_fixed(w.X, w.lo, w.hi, w.M)
    got, gnd = _counts(w.X, w.lo, w.hi, w.M)
    assert gnd == rnd
    assert got.dtype == np.uint64 and np.array_equal(got, ref)
    assert int(got.sum(dtype=np.uint64)) == (w.n - gnd) * 2 ** (w.d * O.default_Q(w.d))


@pytest.mark.parametrize("d,M,Q", [(1, (1000,), None), (1, (7,), 20), (2, (37, 50), None), (2, (2, 2), None),
                                   (3, (5, 9, 17), None), (3, (40, 33, 2), 8), (2, (300, 3), 24),
                                   (4, (7, 9, 5, 11), None), (4, (24, 24, 24, 24), None), (4, (3, 40, 2, 17), 6)])
def test_bin_ragged_bit_exact(d, M, Q):
    rng = np.random.default_rng(100 + d)
    n = 50_000
    X = rng.normal(size=(n, d)) * 1.2
    X[:50] = np.nan
    lo, hi = np.full(d, -2.5), np.full(d, 2.5)
    # samples exactly on nodes and on the box faces
    g = O.grid_axes(lo, hi, M)
    for i in range(200):
        X[100 + i] = [g[k][rng.integers(0, M[k])] for k in range(d)]
    X[400] = hi
    X[401] = lo
    ref, rnd = O.bin_fixed(X, lo, hi, M, Q)
    got, gnd = _counts(X, lo, hi, M, Q=Q)
    assert gnd == rnd
    assert np.array_equal(got, ref)


def test_bin_tile_edges_bit_exact():
    """Samples whose cell straddles the edges of the 32 x 32 binning tiles (copied to each tile they touch)."""
    lo, hi, M = np.array([0.0, 0.0]), np.array([99.0, 99.0]), (100, 100)   # unit spacing
    rng = np.random.default_rng(3)
    edge = np.array([31.0, 31.5, 31.999, 32.0, 32.25, 63.5, 64.0, 95.75, 98.5, 99.0, 0.0, 0.5])
    X = np.stack(np.meshgrid(edge, edge, indexing="ij"), axis=-1).reshape(-1, 2)
    X = np.concatenate([X, rng.uniform(0, 99, size=(5000, 2)), np.repeat(X, 50, axis=0)])
    ref, rnd = O.bin_fixed(X, lo, hi, M)
    got, gnd = _counts(X, lo, hi, M)
    assert gnd == rnd == 0
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("d,M,Q", [(2, (300, 3), 27), (1, (50,), 60), (3, (9, 10, 11), 20), (4, (5, 6, 7, 8), 14)])
def test_bin_atomic_fallback_bit_exact(d, M, Q):
    """Records wider than 64 bits (large Q) take the global-atomic kernel; same results."""
    plan = K.kde_plan_query(None, 10, ([0.0] * d, [1.0] * d, M), Q=Q)
    assert plan["bin_ws_bytes"] == 0
    rng = np.random.default_rng(9)
    X = rng.uniform(-0.1, 1.1, size=(10, d))
    X[0] = 1.0
    ref, rnd = O.bin_fixed(X, [0.0] * d, [1.0] * d, M, Q)
    got, gnd = _counts(X, [0.0] * d, [1.0] * d, M, Q=Q)
    assert gnd == rnd
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("d,M,center", [(2, (512, 512), 0.0), (2, (100, 70), 0.97), (3, (40, 50, 37), 0.95),
                                         (1, (5000,), 0.99), (4, (24, 24, 24, 24), 0.9)])
def test_bin_heavy_tile_segments(d, M, center):
    """Most samples in one tile (also a ragged tile at the far edge of the grid): thousands of
    records in one bucket, summed by many segments into the zeroed counts with atomics."""
    rng = np.random.default_rng(5)
    X = rng.normal(center, 0.02, size=(300_000, d))
    lo, hi = -np.ones(d), np.ones(d)
    ref, rnd = O.bin_fixed(X, lo, hi, M)
    got, gnd = _counts(X, lo, hi, M)
    assert gnd == rnd
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 2, 511, 2047, 2048, 2049, 16_385])
def test_bin_chunk_boundaries(d, n):
    """Sample counts around the 2048-sample chunk of the histogram and scatter passes (a
    last chunk of one sample, exact multiples, one chunk short of a group of eight)."""
    rng = np.random.default_rng(700 + 10 * d)
    X = rng.normal(size=(n, d))
    lo, hi = np.full(d, -3.0), np.full(d, 3.0)
    M = {1: (300,), 2: (61, 70), 3: (20, 17, 33), 4: (9, 10, 11, 12)}[d]
    ref, rnd = O.bin_fixed(X, lo, hi, M)
    got, gnd = _counts(X, lo, hi, M)
    assert gnd == rnd
    assert np.array_equal(got, ref)


def test_bin_empty_and_order_independent():
    got, gnd = _counts(np.zeros((0, 2)), [0.0, 0.0], [1.0, 1.0], (8, 8))
    assert gnd == 0 and not got.any()
    w = W.mix2d_small()
    a, _ = _counts(w.X, w.lo, w.hi, w.M)
    perm = np.random.default_rng(0).permutation(w.n)
    b, _ = _counts(w.X[perm], w.lo, w.hi, w.M)
    assert np.array_equal(a, b)


# --------------------------------------------------------------------------
# lag weights (Eq. 6, Eq. 12)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", ["mix2d_small", "mix2d_512", "mix3d_128"])
def test_kernel_grid(prec, name):
    w = W.WORKLOADS[name]()
    p = O.plan(w.H, w.lo, w.hi, w.M, w.n)
    ref = O.lag_weights(w.H, p["delta"], p["L"], w.n)
    got = K.kde_kernel_grid(w.H, w.n, (w.lo, w.hi, w.M), prec=prec, device=DEV)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert got.shape == ref.shape
    tol = 2e-6 if prec == "f32" else 1e-14
    assert np.max(np.abs(got - ref)) <= tol * ref.max()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_kernel_grid_4d(prec):
    w = W.small_mixture(seed=71, d=4, n=20_000, M=(20, 24, 18, 30))
    p = O.plan(w.H, w.lo, w.hi, w.M, w.n)
    ref = O.lag_weights(w.H, p["delta"], p["L"], w.n)
    got = K.kde_kernel_grid(w.H, w.n, (w.lo, w.hi, w.M), prec=prec, device=DEV)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert got.shape == ref.shape
    tol = 2e-6 if prec == "f32" else 1e-14
    assert np.max(np.abs(got - ref)) <= tol * ref.max()


# --------------------------------------------------------------------------
# convolution from exact counts (Eq. 7): isolates the FFT path
# --------------------------------------------------------------------------

CONV_CASES = [
    # (d, M, seed, L override, H scale); the padded lengths P in the comments: 2^k, and in
    # 3-D and 4-D also 3 x 2^k where shorter
    (1, (200,), 1, None, 1.0),             # 256
    (1, (2000,), 2, None, 1.0),            # 4096 (largest length)
    (1, (1700,), 24, None, 1.0),           # 2048
    (1, (9,), 3, None, 1.0),               # 16 (smallest length)
    (2, (64, 64), 4, None, 1.0),           # (128, 128)
    (2, (37, 50), 5, None, 1.0),           # (64, 64): ragged, odd row count
    (2, (129, 300), 6, None, 3.0),         # (256, 512)
    (2, (2050, 12), 7, None, 0.5),         # (4096, 16)
    (2, (1000, 40), 12, None, 0.3),        # (2048, 64)
    (2, (40, 1700), 27, None, 0.5),        # (64, 2048): long rows
    (2, (24, 19), 8, (23, 18), 1.0),       # (64, 64): full lag box, L = M - 1
    (2, (230, 200), 30, None, 1.0),        # (256, 256): pruned first stages on both axes
    (2, (300, 257), 14, None, 1.0),        # (512, 512): 4 / 8 points per thread
    (2, (520, 700), 15, None, 1.0),        # (1024, 1024)
    (3, (20, 17, 23), 9, None, 1.0),       # (32, 32, 32)
    (3, (33, 40, 31), 10, None, 2.0),      # (48, 64, 48)
    (3, (6, 5, 4), 11, (5, 4, 3), 1.0),    # 16: separate row / column passes
    (3, (24, 40, 10), 13, None, 1.0),      # (32, 48, 16): P_2 != P_3, separate passes
    (3, (100, 9, 7), 28, None, 1.0),       # (128, 16, 16): the product pass on the longest axis
    (3, (70, 6, 5), 32, None, 1.0),        # (96, 16, 16)
    (3, (210, 12, 230), 31, None, 1.0),    # (256, 16, 384): both families in one problem
    (3, (7, 9, 300), 16, None, 1.0),       # P_3 = 384: row passes at 12 points per thread
    (3, (300, 7, 9), 17, None, 1.0),       # P_1 = 384: product pass at 12 points per thread
    (3, (680, 5, 4), 33, (60, 2, 2), 1.0),       # (768, 16, 16)
    (3, (1400, 5, 4), 34, (100, 2, 2), 1.0),     # (1536, 16, 16)
    (3, (2900, 5, 4), 35, (150, 2, 2), 1.0),     # (3072, 16, 16): largest 3 x 2^k
    (3, (4, 5, 700), 36, (2, 2, 50), 1.0),       # (16, 16, 768): long rows
    (3, (5, 4, 2900), 37, (2, 2, 150), 1.0),     # (16, 16, 3072)
    (4, (24, 24, 24, 24), 18, None, 1.0),  # 32: three strided passes each way
    (4, (20, 24, 18, 30), 19, None, 1.0),  # (32, 32, 32, 48): ragged, P_4 != P_1..3
    (4, (6, 5, 4, 7), 20, (5, 4, 3, 6), 1.0),   # 16: full lag box
    (4, (9, 12, 7, 40), 21, None, 2.0),    # (16, 16, 16, 64)
    (4, (40, 6, 5, 9), 22, None, 1.0),     # (64, 16, 16, 16): the product pass on the longest axis
    (4, (100, 6, 5, 9), 29, None, 1.0),    # (192, 16, 16, 16)
]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CONV_CASES, ids=[f"d{c[0]}-{'x'.join(map(str, c[1]))}" for c in CONV_CASES])
def test_conv_from_counts(prec, case):
    d, M, seed, Lovr, hs = case
    w = W.small_mixture(seed=seed, d=d, n=4000, M=M, H_scale=hs)
    # large grids: the oracle's FFT form of Eq. (7) (pinned to the direct sum on the CPU)
    method = "fft" if np.prod(M) > 200_000 else "direct"
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M, L=Lovr, method=method)
    counts = _dev(info["counts"])
    got = K.kde_conv(counts, w.n, w.H, (w.lo, w.hi, w.M), prec=prec, L=Lovr)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert got.shape == f.shape
    assert _rel(got, f) <= TOL[prec], (case, _rel(got, f))


# --------------------------------------------------------------------------
# the whole estimate
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_eval_small_workload(prec):
    w = W.mix2d_small()
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M)
    got, nd = K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), prec=prec)
    torch.cuda.synchronize()
    assert int(nd.cpu().numpy()[0]) == 0
    assert _rel(got.cpu().numpy(), f) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_eval_4d(prec):
    """The whole estimate in d = 4 on a 24^4 grid: every cell against the oracle's FFT form of
    Eq. (7), and sampled cells against the direct sum evaluated one by one."""
    w = W.small_mixture(seed=72, d=4, n=50_000, M=24)
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M, method="fft")
    got, nd = K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), prec=prec)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert int(nd.cpu().numpy()[0]) == info["n_dropped"] == 0
    assert _rel(got, f) <= TOL[prec]
    rng = np.random.default_rng(3)
    pts = [tuple(int(v) for v in rng.integers(0, 24, size=4)) for _ in range(40)]
    pts.append(tuple(int(v) for v in np.unravel_index(np.argmax(f), f.shape)))
    direct = O.conv_direct_at(info["c"], info["k"], info["L"], pts)
    assert np.max(np.abs(np.array([got[p] for p in pts]) - direct)) <= TOL[prec] * np.max(f)


def test_eval_small_diagonal_and_full_differ():
    w = W.mix2d_small()
    Hd = np.diag(np.diag(w.H))
    g = (w.lo, w.hi, w.M)
    full = K.kde_eval(_dev(w.X), w.H, g, prec="f64")[0].cpu().numpy()
    diag = K.kde_eval(_dev(w.X), Hd, g, prec="f64")[0].cpu().numpy()
    fd, _ = O.kde_binned(w.X, Hd, w.lo, w.hi, w.M)
    assert _rel(diag, fd) <= TOL["f64"]
    assert _rel(full, diag) > 0.05


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("d,M", [(2, (80, 60)), (3, (20, 24, 18)), (1, (300,))])
def test_eval_marginal_extent(prec, d, M):
    """The tighter per-axis lag box (extent = marginal) against the oracle with the same box."""
    w = W.small_mixture(200 + d, d, 20_000, M, ratio=(1.0, 20.0))
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M, extent="marginal")
    plan = K.kde_plan_query(w.H, w.n, (w.lo, w.hi, w.M), extent="marginal")
    assert tuple(plan["L"]) == tuple(info["L"])
    got, _ = K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), prec=prec, extent="marginal")
    torch.cuda.synchronize()
    assert _rel(got.cpu().numpy(), f) <= TOL[prec]


@pytest.mark.parametrize("name,M", [("2d", 256), ("3d", 48), ("1d", 1000)])
def test_reused_spectrum_matches_full_call(name, M):
    """A second estimate with the same H, n and grid reuses the spectrum left in the workspace:
    bit-identical to a full call on the same samples."""
    if name == "2d":
        w1, w2 = W.mix2d_512(n=100_000, M=M), W.mix2d_512(n=100_000, M=M, seed_offset=3)
    elif name == "3d":
        w1, w2 = W.mix3d_128(n=100_000, M=M), W.mix3d_128(n=100_000, M=M, seed_offset=3)
    else:
        w1 = W.small_mixture(31, 1, 50_000, M)
        w2 = W.small_mixture(32, 1, 50_000, M)
    g = (w1.lo, w1.hi, w1.M)
    plan = K.kde_plan_query(w1.H, w1.n, g)
    ws = torch.empty(plan["eval_ws_bytes"], dtype=torch.uint8, device=DEV)
    K.kde_eval(_dev(w1.X), w1.H, g, ws=ws)
    X2 = _dev(w2.X)
    reused = K.kde_eval(X2, w1.H, g, ws=ws, reuse_spectrum=True)[0]
    full = K.kde_eval(X2, w1.H, g)[0]
    torch.cuda.synchronize()
    assert torch.equal(reused, full)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("d,M", [(2, (300, 200)), (2, (512, 512)), (3, (48, 40, 36)), (3, (128, 128, 128)),
                                 (4, (16, 20, 12, 18))])
def test_stored_spectrum_matches_default(prec, d, M):
    """Storing the real spectrum on the padded grid (one more spectrum pass; the product pass
    reads it instead of transforming the lag columns) gives the default path's bits: for a full
    estimate, for a stored spectrum reused on new samples, and for kde_conv."""
    w = W.small_mixture(500 + d, d, 60_000, M, ratio=(1.0, 20.0))
    w2 = W.small_mixture(520 + d, d, 60_000, M, ratio=(1.0, 20.0))
    g = (w.lo, w.hi, w.M)
    X, X2 = _dev(w.X), _dev(w2.X)
    plan = K.kde_plan_query(w.H, w.n, g, prec=prec, store_spectrum=True)
    ws = torch.empty(plan["eval_ws_bytes"], dtype=torch.uint8, device=DEV)
    ref = K.kde_eval(X, w.H, g, prec=prec)[0]
    got = K.kde_eval(X, w.H, g, prec=prec, ws=ws, store_spectrum=True)[0]
    reused = K.kde_eval(X2, w.H, g, prec=prec, ws=ws, store_spectrum=True, reuse_spectrum=True)[0]
    full2 = K.kde_eval(X2, w.H, g, prec=prec)[0]
    counts, _ = K.kde_bin(X, g)
    conv = K.kde_conv(counts, w.n, w.H, g, prec=prec, store_spectrum=True)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert torch.equal(reused, full2)
    assert torch.equal(conv, ref)
    if d <= 3 and max(M) <= 300:
        lscv_s = K.kde_lscv(counts, w.n, w.H, g, prec=prec, store_spectrum=True)
        lscv_d = K.kde_lscv(counts, w.n, w.H, g, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(lscv_s, lscv_d)
    if int(np.prod(M)) <= 200_000:
        f, _ = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M)
        assert _rel(got.cpu().numpy(), f) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("d,M,lengths,P", [(2, (300, 257), "composite", (384, 384)),
                                           (3, (48, 40, 36), "pow2", (64, 64, 64)),
                                           (3, (48, 40, 36), "composite", (64, 48, 48))])
def test_eval_length_options(prec, d, M, lengths, P):
    """kde_params.lengths (3 x 2^k also in 2-D, or 2^k only) changes the padded lengths and
    not the estimate beyond rounding."""
    w = W.small_mixture(600 + d, d, 40_000, M, ratio=(1.0, 20.0))
    g = (w.lo, w.hi, w.M)
    assert K.kde_plan_query(w.H, w.n, g, lengths=lengths)["P"] == P
    got = K.kde_eval(_dev(w.X), w.H, g, prec=prec, lengths=lengths)[0]
    torch.cuda.synchronize()
    f, _ = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M)
    assert _rel(got.cpu().numpy(), f) <= TOL[prec]


@pytest.fixture(scope="module")
def ref2d512():
    w = W.mix2d_512()
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M)
    return w, f, info


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_eval_2d_512_full(ref2d512, prec):
    w, f, info = ref2d512
    got, nd = K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), prec=prec)
    torch.cuda.synchronize()
    assert int(nd.cpu().numpy()[0]) == info["n_dropped"]
    assert _rel(got.cpu().numpy(), f) <= TOL[prec]


@pytest.fixture(scope="module")
def ref3d128():
    w = W.mix3d_128()
    p = O.plan(w.H, w.lo, w.hi, w.M, w.n)
    counts, nd = O.bin_fixed(w.X, w.lo, w.hi, w.M)
    c = O.counts_to_c(counts, 3)
    k = O.lag_weights(w.H, p["delta"], p["L"], w.n)
    return w, p, counts, c, k


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_eval_3d_128_sampled(ref3d128, prec):
    w, p, counts, c, k = ref3d128
    got, nd = K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), prec=prec)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    rng = np.random.default_rng(7)
    pts = [tuple(int(v) for v in rng.integers(0, 128, size=3)) for _ in range(1500)]
    imax = np.unravel_index(np.argmax(got), got.shape)
    pts += [tuple(int(v) for v in imax), (0, 0, 0), (127, 127, 127), (0, 127, 64)]
    # points near the mass: a box around the maximum
    for dd in range(-3, 4):
        pts.append(tuple(int(np.clip(imax[a] + dd * (a + 1), 0, 127)) for a in range(3)))
    ref = O.conv_direct_at(c, k, p["L"], pts)
    gmax = float(np.max(got))
    err = np.max(np.abs(np.array([got[q] for q in pts]) - ref))
    assert err <= TOL[prec] * gmax, err / gmax
    # total mass: at most the normal tail beyond tau is lost
    mass = got.sum(dtype=np.float64) * np.prod(p["delta"])
    assert 0.99 <= mass <= 1.0 + 1e-4


def _smooth_at_least(x: int) -> int:
    """Smallest 2^a 3^b >= x (a length numpy's FFT handles quickly)."""
    best = 1 << (x - 1).bit_length()
    p3 = 1
    while p3 < best:
        v = p3
        while v < x:
            v *= 2
        best = min(best, v)
        p3 *= 3
    return best


@pytest.fixture(scope="module")
def full3d128(ref3d128):
    """The whole 128^3 estimate from the oracle's FFT form of Eq. (7) (the paper's layout,
    Eq. 12-14, with P_k >= 2 M_k + 2 L_k - 1, pinned on the CPU to the direct sum)."""
    w, p, counts, c, k = ref3d128
    P = tuple(_smooth_at_least(2 * m + 2 * l - 1) for m, l in zip(w.M, p["L"]))
    return O.conv_fft_corrected(c, k, p["L"], P=P)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_eval_3d_128_full_grid(ref3d128, full3d128, prec):
    """Every one of the 2.1M cells of the 3-D estimate (P = 192 on all three axes)
    element by element against the oracle."""
    w, p, counts, c, k = ref3d128
    got, nd = K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), prec=prec)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert got.shape == full3d128.shape
    assert _rel(got, full3d128) <= TOL[prec], _rel(got, full3d128)
    # the FFT form itself agrees with the direct sum where the latter is evaluated
    pts = [(64, 64, 64), (0, 0, 0), (127, 3, 90), (17, 127, 0)]
    ref = O.conv_direct_at(c, k, p["L"], pts)
    assert np.max(np.abs(np.array([full3d128[q] for q in pts]) - ref)) <= 1e-14 * full3d128.max()


@pytest.fixture(scope="module")
def ref4d48():
    """The 4-D bench workload (n = 1e6, 48^4) through the oracle: counts, weights and the
    FFT form of Eq. (7) (Eq. 12-14 at P_k >= M_k + L_k, pinned on the CPU to the direct sum)."""
    import os
    w = W.mix4d_48()
    f, info = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M, method="fft", workers=min(16, os.cpu_count() or 1))
    return w, info, f


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_eval_4d_48_full_grid(ref4d48, prec):
    """Every one of the 5.3M cells of the 4-D estimate against the oracle, and sampled cells
    against the direct sum evaluated one by one."""
    w, info, f = ref4d48
    got, nd = K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), prec=prec)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert int(nd.cpu().numpy()[0]) == info["n_dropped"]
    assert got.shape == f.shape
    assert _rel(got, f) <= TOL[prec], _rel(got, f)
    rng = np.random.default_rng(9)
    pts = [tuple(int(v) for v in rng.integers(0, 48, size=4)) for _ in range(200)]
    pts.append(tuple(int(v) for v in np.unravel_index(np.argmax(f), f.shape)))
    ref = O.conv_direct_at(info["c"], info["k"], info["L"], pts)
    assert np.max(np.abs(np.array([got[q] for q in pts]) - ref)) <= TOL[prec] * f.max()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("d,M", [(2, (64, 48)), (3, (24, 20, 30)), (1, (200,))])
def test_eval_with_dropped_samples(prec, d, M):
    """A grid box narrower than the data: samples outside it are dropped and counted, and
    the estimate keeps the total n in the 1/n of Eq. (1)."""
    w = W.small_mixture(600 + d, d, 20_000, M)
    span = w.hi - w.lo
    lo, hi = w.lo + 0.2 * span, w.hi - 0.15 * span
    f, info = O.kde_binned(w.X, w.H, lo, hi, w.M)
    assert info["n_dropped"] > 0
    got, nd = K.kde_eval(_dev(w.X), w.H, (lo, hi, w.M), prec=prec)
    torch.cuda.synchronize()
    assert int(nd.cpu().numpy()[0]) == info["n_dropped"]
    assert _rel(got.cpu().numpy(), f) <= TOL[prec]


def test_eval_3d_128_bins_exact_inside_eval(ref3d128):
    """kde_eval bins into its workspace with the same kernel: the counts it convolves are the oracle's."""
    w, p, counts, c, k = ref3d128
    plan = K.kde_plan_query(w.H, w.n, (w.lo, w.hi, w.M))
    ws = torch.empty(plan["eval_ws_bytes"], dtype=torch.uint8, device=DEV)
    K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), ws=ws)
    torch.cuda.synchronize()
    ncell = int(np.prod(w.M))
    got = ws[: ncell * 8].view(torch.uint64).cpu().numpy().reshape(w.M)
    assert np.array_equal(got, counts)


def test_eval_deterministic():
    w = W.mix2d_512(n=200_000, M=256)
    g = (w.lo, w.hi, w.M)
    X = _dev(w.X)
    a = K.kde_eval(X, w.H, g)[0].cpu().numpy()
    b = K.kde_eval(X, w.H, g)[0].cpu().numpy()
    assert np.array_equal(a, b)


def test_eval_single_sample_is_gaussian():
    """n = 1 on a node gives exactly N(X_1, H) inside the lag box (closed form)."""
    H = np.array([[0.09, 0.06], [0.06, 0.08]])
    lo, hi, M = np.array([-2.0, -2.0]), np.array([2.0, 2.0]), (41, 41)
    g = O.grid_axes(lo, hi, M)
    X = np.array([[g[0][17], g[1][23]]])
    f, info = O.kde_binned(X, H, lo, hi, M)
    got = K.kde_eval(_dev(X), H, (lo, hi, M), prec="f64")[0].cpu().numpy()
    assert _rel(got, f) <= 1e-12


def test_eval_errors_on_gpu():
    w = W.mix2d_small()
    X = _dev(w.X)
    with pytest.raises(ValueError):
        K.kde_eval(X, w.H, (w.lo, w.hi, w.M), ws=torch.empty(64, dtype=torch.uint8, device=DEV))
    with pytest.raises(K.KdeError) as e:
        K.kde_eval(X, np.array([[0.09, 0.2], [0.2, 0.08]]), (w.lo, w.hi, w.M))
    assert e.value.code == -2


def test_trace_events_record_every_kernel():
    import ctypes
    hip = K.lib()          # hipEvent* resolved in the runtime the library links
    evs = []
    for _ in range(16):
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        evs.append(e.value)
    w = W.mix2d_small()
    tr = {}
    K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), trace_events=evs, trace=tr)
    torch.cuda.synchronize()
    assert tr["count"] == len(tr["names"])
    # 2-D: the spectrum's row pass shares the histogram's launch
    assert tr["names"] == ["hist_kspec", "bin_scan", "bin_scatter", "bin_accum", "counts_r2c", "conv_col", "c2r"]

    def ms(a, b):
        v = ctypes.c_float()
        assert hip.hipEventElapsedTime(ctypes.byref(v), ctypes.c_void_p(a), ctypes.c_void_p(b)) == 0
        return v.value

    # each pair brackets one kernel: positive durations, kernels in stream order,
    # together no longer than the span from the first start to the last end
    dur = [ms(evs[2 * i], evs[2 * i + 1]) for i in range(tr["count"])]
    assert all(t > 0.0 for t in dur)
    span = ms(evs[0], evs[2 * tr["count"] - 1])
    assert sum(dur) <= span * 1.001 + 1e-3
    for i in range(tr["count"] - 1):
        assert ms(evs[2 * i + 1], evs[2 * i + 2]) >= 0.0
    # capacity for fewer passes than the call has: the first ones are stamped
    tr2 = {}
    K.kde_eval(_dev(w.X), w.H, (w.lo, w.hi, w.M), trace_events=evs[:6], trace=tr2)
    torch.cuda.synchronize()
    assert tr2["names"] == tr["names"][:3]
    for e in evs:
        hip.hipEventDestroy(ctypes.c_void_p(e))


def _hip_events(n):
    import ctypes
    hip = K.lib()
    evs = []
    for _ in range(n):
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        evs.append(e.value)
    return evs


def test_overlapped_spectrum_matches_serial():
    """Untraced calls compute the kernel spectrum on a second stream; traced calls run
    serially on one stream. Same kernels, same arithmetic: bit-identical densities."""
    for name, M in (("2d", 256), ("3d", 64)):
        w = W.mix2d_512(n=200_000, M=M) if name == "2d" else W.mix3d_128(n=200_000, M=M)
        g = (w.lo, w.hi, w.M)
        X = _dev(w.X)
        a = K.kde_eval(X, w.H, g)[0].cpu().numpy()
        tr = {}
        b = K.kde_eval(X, w.H, g, trace_events=_hip_events(32), trace=tr)[0].cpu().numpy()
        assert tr["count"] > 5
        assert np.array_equal(a, b)
        f = K.kde_conv(K.kde_bin(X, g)[0], w.n, w.H, g).cpu().numpy()
        assert np.array_equal(a, f)


def test_graph_capture_replays_match_eager():
    """The whole estimate captured in a HIP graph: every replay (with eager work and
    synchronisations in between) reproduces the eager result exactly."""
    w = W.mix2d_512(n=100_000, M=128)
    g = (w.lo, w.hi, w.M)
    X = _dev(w.X)
    plan = K.kde_plan_query(w.H, w.n, g)
    ws = torch.empty(plan["eval_ws_bytes"], dtype=torch.uint8, device=DEV)
    out = torch.empty(w.M, dtype=torch.float32, device=DEV)
    nd = torch.empty(1, dtype=torch.uint64, device=DEV)
    K.kde_eval(X, w.H, g, out=out, ws=ws, n_dropped=nd)
    torch.cuda.synchronize()
    ref = out.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        K.kde_eval(X, w.H, g, out=out, ws=ws, n_dropped=nd)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        K.kde_eval(X, w.H, g, out=out, ws=ws, n_dropped=nd)
    w2 = W.mix2d_512(n=50_000, M=96, seed_offset=1)
    X2 = _dev(w2.X)
    for rep in range(3):
        out.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        other = K.kde_eval(X2, w2.H, (w2.lo, w2.hi, w2.M))[0]     # eager work between replays
        torch.cuda.synchronize()
        assert float(other.sum()) > 0
