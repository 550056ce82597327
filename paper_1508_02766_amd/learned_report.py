"""Full-size run of the learned bandwidth proposal, printed as one JSON line.

    python -m paper_1508_02766_amd.learned_report [--train 50000] [--test 1000] [--grid 256]

Training mixtures (2-5 components, n log-uniform in [1e3, 1e5]) are drawn,
featurised and labelled with the LSCV-optimal H of the plain batched search
chunk by chunk (samples are not kept). The network trains on the features and
labels; on held-out mixtures at the same grid size the plain search from the
normal-scale start is the reference: the report gives the mean relative LSCV gap
of the normal-scale rule, of the proposal alone and of the plain search
warm-started at the proposal, with the search evaluations and times.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import learned as L
from . import lscv as S


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=50_000)
    ap.add_argument("--test", type=int, default=1_000)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--seed", type=int, default=11)
    a = ap.parse_args(argv)
    M = a.grid
    t_all = time.perf_counter()
    F, T = [], []
    label_s = 0.0
    label_evals = 0
    for c in range(0, a.train, a.chunk):
        part = L.mixtures(min(a.chunk, a.train - c), seed=a.seed * 1_000_003 + c, n_range=(1e3, 1e5))
        F += [L.features(X) for X in part]
        H, st = L.label(part, M=M, iters=a.iters, chunk=a.chunk)
        label_s += st["seconds"]
        label_evals += st["evals"]
        T += [L.to_target(h, X) for h, X in zip(H, part)]
        print(f"[learned] labelled {c + len(part)} / {a.train} ({label_s:.1f} s of search)", file=sys.stderr,
              flush=True)
    F, T = np.stack(F), np.stack(T)
    t0 = time.perf_counter()
    P, losses = L.train(F, T, epochs=a.epochs, batch=256, lr=1e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    steps = a.epochs * (F.shape[0] // 256)
    print(f"[learned] trained {steps} steps in {train_s:.1f} s, loss {losses[0]:.4f} -> {losses[-1]:.4f}",
          file=sys.stderr, flush=True)
    test = L.mixtures(a.test, seed=a.seed * 7 + 1, n_range=(1e3, 1e5))
    Ft = np.stack([L.features(X) for X in test])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Hml = P.predict(test, F=Ft, M=M)
    torch.cuda.synchronize()
    predict_s = time.perf_counter() - t0
    Hst, st = L.label(test, M=M, iters=a.iters, chunk=a.chunk)
    Xs = [torch.as_tensor(X, device="cuda:0") for X in test]
    grids = [L.grid_for(X, M) for X in test]
    t0 = time.perf_counter()
    warm = []
    for c in range(0, a.test, a.chunk):
        warm += S.lscv_search_batch(Xs[c:c + a.chunk], grids[c:c + a.chunk], H0s=Hml[c:c + a.chunk],
                                    iters=a.iters, step=0.05)
    torch.cuda.synchronize()
    warm_s = time.perf_counter() - t0
    Hns = [L.from_target(np.zeros(3), X) for X in test]
    v_st = L.lscv_at(test, Hst, M)
    v_ml = L.lscv_at(test, Hml, M)
    v_ns = L.lscv_at(test, [S.project(H, g) for H, g in zip(Hns, grids)], M)
    v_wm = np.array([r["lscv"] for r in warm])
    rel = lambda v: (v - v_st) / np.abs(v_st)
    out = {
        "train_mixtures": a.train, "test_mixtures": a.test, "grid": [M, M], "search_iters": a.iters,
        "label_search_s": round(label_s, 2), "label_evals": int(label_evals), "train_steps": steps,
        "train_s": round(train_s, 2), "train_loss_first_last": [round(losses[0], 5), round(losses[-1], 5)],
        "gap_normal_scale_mean": float(np.mean(rel(v_ns))), "gap_learned_mean": float(np.mean(rel(v_ml))),
        "gap_learned_median": float(np.median(rel(v_ml))), "gap_warm_start_mean": float(np.mean(rel(v_wm))),
        "cold_search_s": round(st["seconds"], 3), "cold_search_evals": int(st["evals"]),
        "warm_search_s": round(warm_s, 3), "warm_search_evals": int(sum(r["evals"] for r in warm)),
        "predict_s_incl_features": round(predict_s, 4),
        "total_s": round(time.perf_counter() - t_all, 1),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
