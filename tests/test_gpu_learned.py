"""The learned bandwidth proposal end to end on the GPU: LSCV labels from the
batched search, training with the network kernels, and the comparison with
the plain search as reference. Reduced sizes (hundreds of mixtures, 128^2 grids) so the
test runs in seconds; the full-size run is ``python -m
paper_1508_02766_amd.learned_report``. Reports the LSCV gap and the search
time saved."""
import json
import time

import numpy as np
import pytest
import torch

import paper_1508_02766_amd.learned as L
from paper_1508_02766_amd import lscv as S

pytestmark = pytest.mark.gpu


def test_learned_proposal_beats_normal_scale_and_saves_search():
    M = 128
    train = L.mixtures(768, seed=1, n_range=(1e3, 1e4))
    test = L.mixtures(64, seed=2, n_range=(1e3, 1e4))
    Htr, _ = L.label(train, M=M, iters=40)
    F = np.stack([L.features(X) for X in train])
    T = np.stack([L.to_target(H, X) for H, X in zip(Htr, train)])
    P, losses = L.train(F, T, epochs=150, batch=256, lr=2e-3)
    assert losses[-1] < losses[0]
    t0 = time.perf_counter()
    Hml = P.predict(test, M=M)
    torch.cuda.synchronize()
    t_ml = time.perf_counter() - t0
    Hns = [L.from_target(np.zeros(3), X) for X in test]
    t0 = time.perf_counter()
    Hst, st = L.label(test, M=M, iters=40)
    t_search = time.perf_counter() - t0
    # warm start: the plain search from the proposal (fallback and refinement)
    Xs = [torch.as_tensor(X, device="cuda:0") for X in test]
    grids = [L.grid_for(X, M) for X in test]
    t0 = time.perf_counter()
    warm = S.lscv_search_batch(Xs, grids, H0s=Hml, iters=40, step=0.05)
    t_warm = time.perf_counter() - t0
    v_st = L.lscv_at(test, Hst, M)
    v_ml = L.lscv_at(test, Hml, M)
    v_ns = L.lscv_at(test, Hns, M)
    v_wm = np.array([r["lscv"] for r in warm])
    gap = lambda v: float(np.mean((v - v_st) / np.abs(v_st)))
    report = {"gap_learned": gap(v_ml), "gap_normal_scale": gap(v_ns), "gap_warm_start": gap(v_wm),
              "search_s": round(t_search, 3), "predict_s": round(t_ml, 4), "warm_search_s": round(t_warm, 3),
              "evals_cold": int(sum(r for r in [st["evals"]])), "evals_warm": int(sum(r["evals"] for r in warm)),
              "train_loss_first_last": [losses[0], losses[-1]]}
    print(json.dumps(report))
    assert report["gap_learned"] < report["gap_normal_scale"]
    assert report["gap_warm_start"] < 0.01
