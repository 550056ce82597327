"""Batched evaluation (kde_batch_*) through the C ABI.

A batch must reproduce, bit for bit, what kde_eval gives for each item with
the same options (the batched launches run the same device code on the same
workspace layout), and therefore the oracle to the single-instance bars. The
cases mix grid sizes (several padded lengths per pass), sample counts (one to
hundreds of binning chunks), dimensions, and the atomic binning fallback.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1508_02766_amd as K
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f32": 1e-5, "f64": 1e-12}


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device=DEV)


def _items(wl):
    return [(_dev(w.X), w.H, (w.lo, w.hi, w.M)) for w in wl]


def _assert_matches_single(B, items, **opts):
    for i, (X, H, g) in enumerate(items):
        ref, nd = K.kde_eval(X, H, g, **opts)
        torch.cuda.synchronize()
        assert torch.equal(B.densities[i], ref), i
        if B.n_dropped:
            assert int(B.n_dropped[i].cpu()[0]) == int(nd.cpu()[0]), i


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_matches_single_bit_identical(prec):
    wl = W.batch2d(20, seed_offset=11, n_range=(1e3, 6e4), sides=(64, 128, 256))
    # grid side 512 (P = 1024 on both axes, the largest batched lengths) at the full
    # sample count, and a second 512^2 item of another size
    wl += [W.mix2d_512(), W.mix2d_512(n=300_000, seed_offset=5)]
    items = _items(wl)
    B = K.KdeBatch(items, n_dropped=True, prec=prec)
    B.eval()
    torch.cuda.synchronize()
    _assert_matches_single(B, items, prec=prec)
    info = B.info()
    plans = [K.kde_plan_query(w.H, w.n, (w.lo, w.hi, w.M), prec=prec) for w in wl]
    p0, p1 = {p["P"][0] for p in plans}, {p["P"][1] for p in plans}
    # four binning stages, then one launch per padded length for each of the four FFT
    # passes: spectrum rows, count rows and the inverse rows over P_2, the product over P_1
    assert info["launches"] == 4 + 3 * len(p1) + len(p0)


def test_batch_composite_lengths_match_single_calls():
    """With kde_params.lengths = composite the 2-D items pad to 3 x 2^k where shorter (side
    512: P = 768); the batch gives the bits of single calls with the same option, and the
    oracle's estimate within the FP32 bound."""
    wl = W.batch2d(6, seed_offset=21, n_range=(1e3, 3e4), sides=(64, 128, 256))
    wl.append(W.mix2d_512(n=200_000, seed_offset=6))
    items = _items(wl)
    B = K.KdeBatch(items, n_dropped=True, prec="f32", lengths="composite")
    B.eval()
    torch.cuda.synchronize()
    _assert_matches_single(B, items, prec="f32", lengths="composite")
    assert K.kde_plan_query(wl[-1].H, wl[-1].n, (wl[-1].lo, wl[-1].hi, wl[-1].M), lengths="composite")["P"] == (768, 768)
    for i in (0, len(wl) - 1):
        w = wl[i]
        f, _ = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M, method="fft" if w.M[0] > 256 else "direct")
        got = B.densities[i].cpu().numpy()
        assert np.max(np.abs(got - f)) <= 1e-5 * np.max(np.abs(f)), i


def test_batch_matches_oracle():
    wl = W.batch2d(6, seed_offset=12, n_range=(500, 4000), sides=(64, 96))
    wl.append(W.mix2d_512(n=100_000, seed_offset=7))        # 512^2: P = 1024 row and column passes
    items = _items(wl)
    B = K.KdeBatch(items, prec="f32")
    B.eval()
    torch.cuda.synchronize()
    for i, w in enumerate(wl):
        ref, _ = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M, method="fft")
        got = B.densities[i].double().cpu().numpy()
        assert float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))) <= TOL["f32"], i


def test_batch_mixed_dimensions_and_atomic_fallback():
    """d = 1, 2, 3 items in one batch; Q = 16 sends the 3-D items to the atomic
    binning (their packed records would exceed 64 bits) while the others tile."""
    wl = [W.small_mixture(70 + i, d, n, M) for i, (d, n, M) in enumerate(
        [(1, 3000, 300), (2, 20000, (40, 70)), (3, 8000, (12, 20, 9)), (2, 500, 33), (1, 100, 17),
         (3, 30000, 24), (2, 70000, 128)])]
    items = _items(wl)
    for Q in (None, 16):
        opts = {"prec": "f32"} if Q is None else {"prec": "f32", "Q": Q}
        B = K.KdeBatch(items, n_dropped=True, **opts)
        B.eval()
        torch.cuda.synchronize()
        _assert_matches_single(B, items, **opts)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_four_dimensional_items(prec):
    """d = 4 items (three strided passes per transform direction) beside 2-D and 3-D ones;
    Q = 12 sends the 4-D items to the atomic binning (4 x 13 fraction bits plus the corner
    bits exceed a 64-bit record) while the others tile."""
    wl = [W.small_mixture(90 + i, d, n, M) for i, (d, n, M) in enumerate(
        [(4, 20000, (12, 10, 9, 14)), (2, 5000, (40, 33)), (4, 3000, 16), (3, 8000, (12, 20, 9)),
         (4, 40000, (20, 24, 18, 30))])]
    items = _items(wl)
    for Q in (None, 12):
        opts = {"prec": prec} if Q is None else {"prec": prec, "Q": Q}
        B = K.KdeBatch(items, n_dropped=True, **opts)
        B.eval()
        torch.cuda.synchronize()
        _assert_matches_single(B, items, **opts)
    for i in (0, 4):    # the last batch ran with Q = 12
        ref, _ = O.kde_binned(wl[i].X, wl[i].H, wl[i].lo, wl[i].hi, wl[i].M, Q=12, method="fft")
        got = B.densities[i].double().cpu().numpy()
        assert float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))) <= TOL[prec], i


def test_batch_graph_capture_replays_match_eager():
    wl = W.batch2d(12, seed_offset=13, n_range=(1e3, 3e4), sides=(64, 128, 256))
    items = _items(wl)
    B = K.KdeBatch(items, prec="f32")
    B.eval()
    torch.cuda.synchronize()
    ref = [d.clone() for d in B.densities]
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.eval()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        B.eval()
    other = W.mix2d_512(n=20_000, M=64, seed_offset=2)
    for rep in range(3):
        for d in B.densities:
            d.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        for i, d in enumerate(B.densities):
            assert torch.equal(d, ref[i]), (rep, i)
        o = K.kde_eval(_dev(other.X), other.H, (other.lo, other.hi, other.M))[0]   # eager work between replays
        torch.cuda.synchronize()
        assert float(o.sum()) > 0


def test_batch_new_data_in_bound_buffers():
    """The bound batch reads its items' X buffers at every eval."""
    wl = W.batch2d(5, seed_offset=14, n_range=(2e3, 2e4), sides=(64, 128))
    items = _items(wl)
    B = K.KdeBatch(items, prec="f32")
    B.eval()
    torch.cuda.synchronize()
    for (X, _, _), w in zip(items, wl):
        X.mul_(0.9)
    B.eval()
    torch.cuda.synchronize()
    _assert_matches_single(B, items, prec="f32")


def test_batch_tune_keeps_results():
    wl = W.batch2d(16, seed_offset=15, n_range=(1e3, 1e5), sides=(64, 128, 256, 512))
    items = _items(wl)
    B = K.KdeBatch(items, prec="f32")
    B.eval()
    torch.cuda.synchronize()
    ref = [d.clone() for d in B.densities]
    info = B.tune(reps=2)
    assert info["tile"] in [(0, 0, 0, 0), (16, 64, 0, 0), (64, 16, 0, 0), (64, 64, 0, 0), (16, 16, 0, 0)]
    B.eval()
    torch.cuda.synchronize()
    for i, d in enumerate(B.densities):
        assert torch.equal(d, ref[i]), i
    # every tile shape and both strided-pass shapes give identical results
    for tile in [(16, 64, 0), (64, 64, 0)]:
        C = K.KdeBatch(items, prec="f32", tile=tile)
        C.eval()
        torch.cuda.synchronize()
        for i, d in enumerate(C.densities):
            assert torch.equal(d, ref[i]), (tile, i)


def test_batch_trace_names_groups():
    wl = W.batch2d(4, seed_offset=16, n_range=(1e3, 5e3), sides=(64,))
    items = _items(wl)
    import ctypes
    hip = K.lib()
    evs = []
    for _ in range(32):
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        evs.append(e.value)
    B = K.KdeBatch(items, prec="f32", trace_events=evs, trace={})
    B.eval()
    torch.cuda.synchronize()
    t = B.trace()
    assert t["names"] == ["bin_hist", "bin_scan", "bin_scatter", "bin_accum", "counts_r2c",
                          "kspec_r2c", "conv_col", "c2r"]
    for i in range(t["count"]):
        ms = ctypes.c_float()
        assert hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(evs[2 * i]),
                                       ctypes.c_void_p(evs[2 * i + 1])) == 0
        assert ms.value > 0.0
    _assert_matches_single(B, items, prec="f32")
    for e in evs:
        hip.hipEventDestroy(ctypes.c_void_p(e))


def test_batch_errors():
    w = W.batch2d(2, seed_offset=17, n_range=(1e3, 2e3), sides=(64,))
    items = _items(w)
    bad = list(items)
    bad[1] = (items[1][0], np.array([[1.0, 2.0], [2.0, 1.0]]), items[1][2])
    with pytest.raises(K.KdeError) as e:
        K.KdeBatch(bad)
    assert e.value.code == -2
    with pytest.raises(K.KdeError):
        K.KdeBatch(items, tile=(48, 32, 0))
