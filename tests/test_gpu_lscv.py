"""LSCV objective and search on the GPU (through the C ABI) against the oracle.

Bars: each term of the objective within 1e-12 (FP64) / 2e-5 (FP32) of its own
magnitude against the FP64 oracle of the binned objective; the batched dot
products give bit-identical terms to the single-problem call; the search ends
at a point the oracle confirms as a local minimum of the binned objective.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1508_02766_amd as K
from paper_1508_02766_amd import lscv as S
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f32": 2e-5, "f64": 1e-12}
CASES = [(2, 2000, 64, 0.7), (2, 500, 40, 1.6), (1, 3000, 200, 1.0), (3, 1500, 20, 1.2), (2, 20000, 128, 0.5),
         (4, 2000, 12, 1.0)]


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device=DEV)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("d,n,M,scale", CASES)
def test_lscv_matches_oracle(prec, d, n, M, scale):
    w = W.small_mixture(90 + d + M, d, n, M, H_scale=scale)
    g = (w.lo, w.hi, w.M)
    counts, _ = K.kde_bin(_dev(w.X), g)
    got = K.kde_lscv(counts, n, w.H, g, prec=prec).cpu().numpy()
    ref = np.array(O.lscv_binned_terms(w.X, w.H, w.lo, w.hi, w.M))
    for k in (1, 2):
        assert abs(got[k] - ref[k]) <= TOL[prec] * abs(ref[k]), (k, got, ref)
    assert abs(got[0] - ref[0]) <= TOL[prec] * (abs(ref[1]) + abs(ref[2]))


def test_lscv_batch_terms_bit_identical_to_single():
    ws = [W.small_mixture(120 + i, 2, n, M) for i, (n, M) in enumerate([(1000, 64), (5000, 96), (300, 33), (40000, 128)])]
    probs = []
    singles = []
    for i, w in enumerate(ws):
        g = (w.lo, w.hi, w.M)
        C, _ = K.kde_bin(_dev(w.X), g)
        H = w.H * (0.6 + 0.3 * i)
        probs.append((C, w.n, H, g))
        singles.append(K.kde_lscv(C, w.n, H, g).cpu().numpy())
    vals = S.lscv_values_batch(probs)
    for v, s in zip(vals, singles):
        assert v == s[0]


def test_lscv_trace_pairs_time_each_pass():
    """Traced kde_lscv: one kernel-stamped event pair per pass, the two dot-product stages
    counted as one pass; the traced call gives the untraced call's bits."""
    import ctypes
    hip = K.lib()
    evs = []
    for _ in range(64):
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        evs.append(e.value)
    w = W.small_mixture(130, 2, 3000, 64)
    g = (w.lo, w.hi, w.M)
    counts, _ = K.kde_bin(_dev(w.X), g)
    plain = K.kde_lscv(counts, w.n, w.H, g).cpu().numpy()
    tr = {}
    got = K.kde_lscv(counts, w.n, w.H, g, trace_events=evs, trace=tr).cpu().numpy()
    assert np.array_equal(got, plain)
    names = tr["names"]
    assert names.count("dot") == 2 and names[-1] == "lscv_combine" and tr["count"] == len(names)
    for i in range(tr["count"]):
        ms = ctypes.c_float()
        assert hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(evs[2 * i]),
                                       ctypes.c_void_p(evs[2 * i + 1])) == 0
        assert ms.value > 0.0
    for e in evs:
        hip.hipEventDestroy(ctypes.c_void_p(e))


def test_lscv_rejects_bad_input():
    w = W.small_mixture(130, 2, 100, 32)
    g = (w.lo, w.hi, w.M)
    C, _ = K.kde_bin(_dev(w.X), g)
    with pytest.raises(ValueError):
        K.kde_lscv(C, 1, w.H, g)
    with pytest.raises(K.KdeError):
        K.kde_lscv(C, w.n, -w.H, g)
    small = torch.empty(64, dtype=torch.uint8, device=DEV)
    with pytest.raises(ValueError):
        K.kde_lscv(C, w.n, w.H, g, ws=small)


def test_lscv_search_reaches_oracle_local_minimum():
    """The search ends at a point where the oracle's binned objective is lower
    than at the start and than at every admissible neighbour."""
    w = W.small_mixture(140, 2, 800, 64, H_scale=2.5)
    X = _dev(w.X)
    g = (w.lo, w.hi, w.M)
    r = S.lscv_search(X, g, H0=w.H, iters=80, prec="f64")
    f = lambda H: O.lscv_binned(w.X, H, w.lo, w.hi, w.M)
    best = f(r["H"])
    assert best < f(w.H)
    assert best == pytest.approx(r["lscv"], rel=1e-10, abs=1e-14)
    dmax = float(np.max((w.hi - w.lo) / (np.array(w.M) - 1)))
    theta = S.to_theta(r["H"])
    checked = 0
    for k in range(theta.size):
        for s in (-0.05, 0.05):
            t = theta.copy()
            t[k] += s
            Hn = S.from_theta(t, 2)
            if np.linalg.eigvalsh(Hn)[0] < dmax ** 2:
                continue                      # outside the search domain
            checked += 1
            assert f(Hn) >= best - 1e-12 * abs(best)
    assert checked >= 4


def test_lscv_search_batch_equals_single_searches():
    ws = [W.small_mixture(150 + i, 2, 600 + 400 * i, 48) for i in range(4)]
    samples = [_dev(w.X) for w in ws]
    grids = [(w.lo, w.hi, w.M) for w in ws]
    batch = S.lscv_search_batch(samples, grids, iters=40)
    for X, g, b in zip(samples, grids, batch):
        single = S.lscv_search(X, g, iters=40)
        assert single["lscv"] == b["lscv"]
        assert np.array_equal(single["H"], b["H"])
        assert single["evals"] == b["evals"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_lscv_batch_bit_identical_to_single(prec):
    """kde_lscv_batch_create: every problem's {LSCV, t1, t2}, combined on the device,
    equals kde_lscv of that problem bit for bit (2-D of several sizes, 1-D and 3-D)."""
    probs = []
    for i, (d, M, n) in enumerate([(2, 64, 3000), (2, 128, 20_000), (2, 256, 50_000), (2, 512, 100_000),
                                   (1, 300, 4000), (3, 24, 5000)]):
        w = W.small_mixture(400 + i, d, n, M)
        g = (w.lo, w.hi, w.M)
        C, _ = K.kde_bin(_dev(w.X), g)
        probs.append((C, w.n, w.H, g))
    B = K.KdeLscvBatch(probs, prec=prec)
    B.eval()
    got = B.out.cpu().numpy()
    for k, (C, n, H, g) in enumerate(probs):
        ref = K.kde_lscv(C, n, H, g, prec=prec).cpu().numpy()
        assert np.array_equal(got[k], ref), k
        assert got[k][0] == got[k][1] - got[k][2]
    # a second eval after tuning gives the same values
    B.tune(reps=1)
    B.out.zero_()
    B.eval()
    assert np.array_equal(B.out.cpu().numpy(), got)
    B.close()


def test_lscv_batch_matches_oracle_terms():
    w = W.small_mixture(420, 2, 2500, 48)
    g = (w.lo, w.hi, w.M)
    C, _ = K.kde_bin(_dev(w.X), g)
    B = K.KdeLscvBatch([(C, w.n, w.H, g), (C, w.n, 1.5 * w.H, g)], prec="f64")
    B.eval()
    got = B.out.cpu().numpy()
    for k, s in enumerate((1.0, 1.5)):
        v, t1, t2 = O.lscv_binned_terms(w.X, s * w.H, w.lo, w.hi, w.M)
        assert got[k][1] == pytest.approx(t1, rel=1e-11)
        assert got[k][2] == pytest.approx(t2, rel=1e-11)
    B.close()
