"""Benchmark of the gfx950 binned FFT KDE on one MI355X.

One step = one whole estimate (kde_eval: zero + fixed-point binning of n
samples, lag-box fill, kernel spectrum, forward FFTs of the counts, product,
inverse FFTs, window) over inputs already resident in HBM. Default workload:
d = 2, n = 1,000,000 samples of a 5-component normal mixture, 512 x 512 grid,
full H with correlation 0.8, FP32 convolution. The JSON line also carries the
3-D 128^3, 4-D 48^4 and FP64 variants, the batched form (256 independent 2-D problems
of uneven size through kde_batch_*, autotuned, eager and graph-replayed), the
per-kernel roofline of the dominant kernel and the FP64 CPU oracle timed on
the host.

    python bench.py [--steps K] [--warmup W] [--workload mix2d_512|mix3d_128|mix4d_48] [--prec f32|f64]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters.json")


def kernel_source_hash() -> str:
    """SHA-256 over the device-code sources (kernels and the headers they include);
    host orchestration (kde_api.cpp) does not enter."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = glob.glob(os.path.join(ROOT, "paper_1508_02766_amd", "csrc", "*.hip"))
    files += glob.glob(os.path.join(ROOT, "paper_1508_02766_amd", "csrc", "*.h"))
    for f in sorted(files):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    readings, scaled by what the same counters read for a plain copy of known
    size; None when the kernels changed since the counters were taken."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except OSError:
        return None
    if c.get("source_sha256") != kernel_source_hash():
        return None
    k = c.get("workloads", {}).get(workload, {}).get(kernel)
    cal = c.get("copy_calibration", {}).get(workload)
    if not k or not cal:
        return None
    return int((k["FETCH_SIZE"] * cal["fetch_factor"] + k["WRITE_SIZE"] * cal["write_factor"]) * 1024)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="mix2d_512", choices=["mix2d_512", "mix3d_128", "mix4d_48"])
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-variants", action="store_true", help="skip the 3-D / 4-D / FP64 / batched side measurements")
    ap.add_argument("--variants", default="mix2d_512_f64,mix3d_128_f32,mix3d_128_f64,mix4d_48_f32,batch",
                    help="comma-separated side measurements to run")
    ap.add_argument("--batch", type=int, default=256, help="problems in the batched measurement (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-reps", type=int, default=9)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run 5 plain device copies of this many MiB (calibrates HBM byte counters)")
    return ap.parse_args()


# --------------------------------------------------------------------------
# HIP events through the runtime library (the library records them on its stream)
# --------------------------------------------------------------------------

class Hip:
    """hipEvent calls resolved through libkde.so, i.e. in the HIP runtime the library itself uses."""

    def __init__(self, kde_lib):
        self.lib = kde_lib

    def event(self) -> int:
        e = ctypes.c_void_p()
        if self.lib.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return e.value

    def elapsed_ms(self, a: int, b: int) -> float:
        ms = ctypes.c_float()
        if self.lib.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b)) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def destroy(self, e: int):
        self.lib.hipEventDestroy(ctypes.c_void_p(e))


# --------------------------------------------------------------------------
# HBM bytes per launch. `alg` counts the method's bytes only (the measurement
# contract of the path): binning reads X once and writes the counts once; the
# FFT convolution reads the u64 counts, moves the half-spectrum intermediates
# once per pass (r2c on the contiguous axis), reads a half-space real kernel
# spectrum once and writes the density. `design` adds what this design moves
# on top (binning records, histograms, the lag columns the product pass
# transforms in place).
# --------------------------------------------------------------------------

def conv_method_bytes(d, M, P, prec):
    """Method bytes of the FFT convolution (counts -> density), per pass, r2c form:
    2-D: 8 M^2 + 4 M H w_c + P H w_r + M^2 w_r; 3-D: 8 M^3 + 4 M^2 H w_c + 4 M P H w_c
    + P^2 H w_r + M^3 w_r, with H = P_d / 2 + 1 (1-D: 8 M + 2 H w_c + H w_r + M w_r; 4-D: each
    strided pass reads and writes its arrays once, and the product reads the real spectrum)."""
    rs = 4 if prec == "f32" else 8
    cs = 2 * rs
    H = P[-1] // 2 + 1
    cells = int(np.prod(M))
    if d == 1:
        return {"counts_r2c": cells * 8 + H * cs, "product_c2r": H * cs + H * rs + cells * rs}
    if d == 2:
        rows = M[0] * H * cs
        return {"counts_r2c": cells * 8 + rows, "conv_col": 2 * rows + P[0] * H * rs, "c2r": rows + cells * rs}
    if d == 4:
        z1 = M[0] * M[1] * M[2] * H * cs          # [M0][M1][M2] half spectra
        z2 = M[0] * M[1] * P[2] * H * cs          # [M0][M1][P2]
        z3 = M[0] * P[1] * P[2] * H * cs          # [M0][P1][P2]
        return {"counts_r2c": cells * 8 + z1, "counts_col3": z1 + z2, "counts_col2": z2 + z3,
                "conv_col1": 2 * z3 + P[0] * P[1] * P[2] * H * rs, "inv_col2": z3 + z2, "inv_col3": z2 + z1,
                "c2r": z1 + cells * rs}
    plane = M[0] * M[1] * H * cs
    mid = M[0] * P[1] * H * cs
    return {"counts_r2c": cells * 8 + plane, "counts_col2": plane + mid, "conv_col1": 2 * mid + P[0] * P[1] * H * rs,
            "inv_col2": mid + plane, "c2r": plane + cells * rs}


def spectrum_bytes(d, L, P, prec):
    """The kernel spectrum (computed once per H, n and grid): the strided passes of the
    lag box's transform, in + out (the row pass computes its weights in place)."""
    cs = 8 if prec == "f32" else 16
    H = P[-1] // 2 + 1
    nb = [2 * l + 1 for l in L]
    if d == 1:
        return {"kspec_r2c": H * cs // 2}
    if d == 2:
        return {"kspec_r2c": nb[0] * H * cs}
    if d == 4:
        k1 = nb[0] * nb[1] * nb[2] * H * cs
        k2 = nb[0] * nb[1] * P[2] * H * cs
        k3 = nb[0] * P[1] * P[2] * H * cs
        return {"kspec_r2c": k1, "kspec_col3": k1 + k2, "kspec_col2": k2 + k3}
    return {"kspec_r2c": nb[0] * nb[1] * H * cs, "kspec_col2": nb[0] * nb[1] * H * cs + nb[0] * P[1] * H * cs}


def kernel_bytes(name: str, w, plan: dict, prec: str) -> dict:
    """{"alg": method bytes, "design": bytes this design moves} of one launch."""
    rs = 4 if prec == "f32" else 8
    cs = 2 * rs
    d, M, L, P, n = w.d, w.M, plan["L"], plan["P"], w.n
    H = P[-1] // 2 + 1
    cells = int(np.prod(M))
    x_read, counts_write = n * d * 8, cells * 8
    records = n * 8            # about one packed 8-byte record per sample (more where cells straddle tiles)
    conv = conv_method_bytes(d, M, P, prec)
    spec = spectrum_bytes(d, L, P, prec)
    nb = [2 * l + 1 for l in L]
    # the product pass also reads its lag columns and transforms them in place
    lagcols = {}
    if d == 2:
        lagcols = {"conv_col": nb[0] * H * cs - P[0] * H * rs}
    elif d == 3:
        lagcols = {"conv_col1": nb[0] * P[1] * H * cs - P[0] * P[1] * H * rs}
    elif d == 4:
        lagcols = {"conv_col1": nb[0] * P[1] * P[2] * H * cs - P[0] * P[1] * P[2] * H * rs}
    # The method reads X once and writes the counts once. This design reads X twice (the
    # histogram counts records, the scatter places them); the method's read is credited to the
    # scatter, whose records the accumulation sums, and the histogram's read is design bytes.
    binning = {
        "zero_counts": (0, cells * 8), "zero_dropped": (0, 8), "bin": (x_read + counts_write, 0),
        "bin_hist": (0, x_read), "bin_scan": (0, 0), "bin_scatter": (x_read, records),
        "bin_accum": (counts_write, records),
    }
    if name in binning:
        a, extra = binning[name]
        return {"alg": a, "design": a + extra}
    if name == "hist_kspec":
        return {"alg": spec["kspec_r2c"], "design": x_read + spec["kspec_r2c"]}
    if name == "scan_kcol":
        return {"alg": spec["kspec_col2"], "design": spec["kspec_col2"]}
    if name == "kfill":
        return {"alg": int(np.prod(nb)) * rs, "design": int(np.prod(nb)) * rs}
    if name in spec:
        return {"alg": spec[name], "design": spec[name]}
    a = conv[name]
    return {"alg": a, "design": a + lagcols.get(name, 0)}


CONV_KERNELS = {"counts_r2c", "counts_col2", "counts_col3", "conv_col", "conv_col1", "inv_col2", "inv_col3", "c2r",
                "product_c2r"}
SPEC_KERNELS = {"kspec_r2c", "kspec_col2", "kspec_col3"}


def step_roofline(kern: dict, names, alg_bytes: int) -> dict:
    """Bytes of a whole step of the path over the summed kernel-stamped times of its launches."""
    us = sum(kern[k]["us"] for k in names if k in kern)
    if us <= 0:
        return None
    gbs = alg_bytes / (us * 1e-6) / 1e9
    return {"kernels": [k for k in names if k in kern], "us": round(us, 3), "alg_bytes": int(alg_bytes),
            "achieved_GBs": round(gbs, 1), "peak_GBs": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4)}


def measure(K, W, hip, name: str, prec: str, steps: int, warmup: int):
    import torch
    w = W.WORKLOADS[name]()
    dev = "cuda:0"
    X = torch.as_tensor(w.X, device=dev)
    grid = (w.lo, w.hi, w.M)
    plan = K.kde_plan_query(w.H, w.n, grid, prec=prec)
    ws = torch.empty(plan["eval_ws_bytes"], dtype=torch.uint8, device=dev)
    out = torch.empty(w.M, dtype=torch.float32 if prec == "f32" else torch.float64, device=dev)
    nd = torch.empty(1, dtype=torch.uint64, device=dev)
    cap = 32   # event pairs for up to 16 kernels
    plain = K.prepare_eval(X, w.H, grid, out, ws, nd, prec=prec)
    for _ in range(warmup):
        plain()
    torch.cuda.synchronize()
    # timed region: K whole steps as a caller runs them
    t0 = time.perf_counter()
    for _ in range(steps):
        plain()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # serving with a fixed H: the kernel spectrum left in the workspace is reused
    reuse = K.prepare_eval(X, w.H, grid, out, ws, nd, prec=prec, reuse_spectrum=True)
    torch.cuda.synchronize()
    r0 = time.perf_counter()
    for _ in range(steps):
        reuse()
    torch.cuda.synchronize()
    r1 = time.perf_counter()
    # the same step captured once in a HIP graph and replayed K times (no host launch
    # cost inside the timed region)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        K.prepare_eval(X, w.H, grid, out, ws, nd, prec=prec)()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        K.prepare_eval(X, w.H, grid, out, ws, nd, prec=prec)()
    for _ in range(3):
        graph.replay()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    del graph

    def traced(ws_, nsteps=steps, flush=None, **o):
        """nsteps steps with every kernel stamping an event pair with its own dispatch start and
        end (hipExtLaunchKernel); tracing keeps all kernels in order on one stream. With `flush`,
        a 512 MiB write before each step evicts the last-level cache (cold kernels)."""
        events = [[hip.event() for _ in range(cap)] for _ in range(nsteps)]
        calls = [K.prepare_eval(X, w.H, grid, out, ws_, nd, prec=prec, trace_events=events[s], **o)
                 for s in range(nsteps)]
        torch.cuda.synchronize()
        u0 = time.perf_counter()
        for c in calls:
            if flush is not None:
                flush.fill_(1)
            c()
        torch.cuda.synchronize()
        u1 = time.perf_counter()
        per = {}
        names = None
        for s in range(nsteps):
            tr = calls[s].trace()
            names = tr["names"]
            for i, nm in enumerate(names):
                per.setdefault(nm, []).append(hip.elapsed_ms(events[s][2 * i], events[s][2 * i + 1]))
        gpu_ms = float(np.mean([hip.elapsed_ms(events[s][0], events[s][2 * len(names) - 1]) for s in range(nsteps)]))
        for row in events:
            for e in row:
                hip.destroy(e)
        return names, {nm: float(np.mean(per[nm])) * 1e3 for nm in names}, gpu_ms, (u1 - u0) * 1e3 / nsteps

    # cold steps: a 512 MiB write before each step evicts the last-level cache, so the
    # step reads its inputs from HBM; each step is bracketed by events on the stream
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    cold = []
    for _ in range(10):
        flush.fill_(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plain()
        e1.record()
        e1.synchronize()
        cold.append(e0.elapsed_time(e1))
    _, cold_us, _, _ = traced(ws, nsteps=10, flush=flush)
    del flush
    # warm steps one by one, each bracketed by events on the stream (median of 50)
    ev = []
    for _ in range(50):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plain()
        e1.record()
        ev.append((e0, e1))
    torch.cuda.synchronize()
    ev_ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
    names, per_us, gpu_step_ms, ms_traced = traced(ws)
    # serving with the spectrum stored on the padded grid: after one full call, the product
    # pass reads the stored real spectrum instead of transforming each line's lag column
    plan_s = K.kde_plan_query(w.H, w.n, grid, prec=prec, store_spectrum=True)
    ws_s = torch.empty(plan_s["eval_ws_bytes"], dtype=torch.uint8, device=dev)
    K.prepare_eval(X, w.H, grid, out, ws_s, nd, prec=prec, store_spectrum=True)()
    stored = K.prepare_eval(X, w.H, grid, out, ws_s, nd, prec=prec, store_spectrum=True, reuse_spectrum=True)
    stored()
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for _ in range(steps):
        stored()
    torch.cuda.synchronize()
    s1 = time.perf_counter()
    s_names, s_us, _, _ = traced(ws_s, store_spectrum=True, reuse_spectrum=True)
    ms_step = (t1 - t0) * 1e3 / steps
    kern = {}
    for nm in names:
        us = per_us[nm]
        b = kernel_bytes(nm, w, plan, prec)
        uc = cold_us.get(nm)
        kern[nm] = {"us": round(us, 3), "alg_bytes": int(b["alg"]), "alg_GBs": round(b["alg"] / (us * 1e-6) / 1e9, 1),
                    "alg_frac": round(b["alg"] / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                    "us_cold": round(uc, 3) if uc else None,
                    "alg_frac_cold": round(b["alg"] / (uc * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if uc else None,
                    "design_bytes": int(b["design"])}
        hbm = measured_traffic(name, nm) if prec == "f32" else None
        if hbm is not None:
            kern[nm]["hbm_bytes"] = hbm
            kern[nm]["hbm_frac"] = round(hbm / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    conv_names = [k for k in names if k in CONV_KERNELS]
    bin_names = [k for k in names if k not in CONV_KERNELS and k not in SPEC_KERNELS]
    conv_us = sum(kern[k]["us"] for k in conv_names)
    bin_us = sum(kern[k]["us"] for k in bin_names)
    cells = int(np.prod(w.M))
    conv_alg = sum(conv_method_bytes(w.d, w.M, plan["P"], prec).values())
    bin_alg = w.n * w.d * 8 + cells * 8
    steps_roof = {"binning": step_roofline(kern, bin_names, bin_alg),
                  "fft_convolution": step_roofline(kern, conv_names, conv_alg)}
    # 3-D and 4-D plans pad to 3 x 2^j where shorter: beside the method bytes at the plan's
    # lengths, the same formula at the power-of-two lengths (the layout before that choice)
    pow2 = [max(16, 1 << (int(m) + int(l) - 1).bit_length()) for m, l in zip(w.M, plan["L"])]
    if steps_roof["fft_convolution"] and list(plan["P"]) != pow2:
        b2 = sum(conv_method_bytes(w.d, w.M, pow2, prec).values())
        c = steps_roof["fft_convolution"]
        c["pow2_P"] = pow2
        c["pow2_alg_bytes"] = int(b2)
        c["frac_on_pow2_alg_bytes"] = round(b2 / (c["us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    cold_kern = {k: {"us": v["us_cold"]} for k, v in kern.items() if v["us_cold"]}
    for key, nm_, alg in (("binning", bin_names, bin_alg), ("fft_convolution", conv_names, conv_alg)):
        c = step_roofline(cold_kern, nm_, alg)
        if steps_roof[key] and c:
            steps_roof[key]["us_cold"] = c["us"]
            steps_roof[key]["frac_cold"] = c["frac"]
    if w.d >= 2:
        # the same chain reading the stored spectrum (serving a fixed H): the method's bytes as
        # above; the stored spectrum read, prod P_k / P_d x pitch reals, is design traffic
        s_kern = {nm: {"us": round(s_us[nm], 3)} for nm in s_names}
        s_conv = [k for k in s_names if k in CONV_KERNELS]
        roof = step_roofline(s_kern, s_conv, conv_alg)
        if roof:
            rs = 4 if prec == "f32" else 8
            pitch = (plan["P"][-1] // 2 + 1 + 15) // 16 * 16
            roof["spectrum_read_bytes"] = int(np.prod(plan["P"][:-1])) * pitch * rs
            roof["kernel_us"] = {k: s_kern[k]["us"] for k in s_conv}
            steps_roof["fft_convolution_stored_spectrum"] = roof
    if steps_roof["binning"] and "hist_kspec" in kern:
        steps_roof["binning"]["note"] = "hist_kspec also runs the kernel spectrum's row pass beside the histogram"
    return {
        "workload": name, "prec": prec, "n": w.n, "M": list(w.M), "L": list(plan["L"]), "P": list(plan["P"]),
        "ms_per_step": ms_step, "ms_per_step_traced": ms_traced, "gpu_ms_per_step_traced": gpu_step_ms,
        "ms_per_step_cold": float(np.median(cold)), "ms_per_step_graph": (g1 - g0) * 1e3 / steps,
        "ms_per_step_event_median": ev_ms,
        "ms_per_step_reused_spectrum": (r1 - r0) * 1e3 / steps,
        "ms_per_step_stored_spectrum": (s1 - s0) * 1e3 / steps,
        "samples_per_s": w.n / (ms_step * 1e-3), "grid_pts_per_s": cells / (ms_step * 1e-3),
        "conv_us": round(conv_us, 3), "conv_grid_pts_per_s": cells / (conv_us * 1e-6),
        "bin_us": round(bin_us, 3), "bin_samples_per_s": w.n / (bin_us * 1e-6), "kernels": kern,
        "steps": steps_roof,
    }


def measure_batch(K, W, hip, count: int, steps: int, warmup: int):
    """The batched form: `count` independent 2-D problems (n log-uniform in
    [1e3, 1e6], grid side in {64, 128, 256, 512}, random SPD H) per step."""
    import torch
    wl = W.batch2d(count)
    dev = "cuda:0"
    items = [(torch.as_tensor(w.X, device=dev), w.H, (w.lo, w.hi, w.M)) for w in wl]
    B = K.KdeBatch(items, prec="f32")
    t0 = time.perf_counter()
    info = B.tune(reps=3)
    tune_s = time.perf_counter() - t0
    for _ in range(warmup):
        B.eval()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        B.eval()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3 / steps
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.eval()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        B.eval()
    for _ in range(3):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / steps
    # the same batch with 3 x 2^k padded lengths in 2-D as well (kde_params.lengths)
    Bc = K.KdeBatch(items, prec="f32", lengths="composite")
    Bc.tune(reps=3)
    for _ in range(warmup):
        Bc.eval()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        Bc.eval()
    torch.cuda.synchronize()
    composite_ms = (time.perf_counter() - t0) * 1e3 / steps
    Bc.close()
    # the same problems as one kde_eval call each
    plans = [K.kde_plan_query(w.H, w.n, (w.lo, w.hi, w.M)) for w in wl]
    wss = [torch.empty(p["eval_ws_bytes"], dtype=torch.uint8, device=dev) for p in plans]
    outs = [torch.empty(w.M, dtype=torch.float32, device=dev) for w in wl]
    calls = [K.prepare_eval(X, H, g, outs[i], wss[i]) for i, (X, H, g) in enumerate(items)]
    for c in calls:
        c()
    torch.cuda.synchronize()
    loop_steps = max(3, steps // 10)
    t0 = time.perf_counter()
    for _ in range(loop_steps):
        for c in calls:
            c()
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3 / loop_steps
    same = all(torch.equal(outs[i], B.densities[i]) for i in range(len(wl)))
    del wss, outs, calls
    # per-kernel times of the batched launches (traced: one stream, each launch stamping
    # an event pair with its dispatch start and end)
    evs = [hip.event() for _ in range(128)]
    T = K.KdeBatch(items, prec="f32", trace_events=evs, trace={}, tile=info["tile"] if any(info["tile"]) else None)
    T.eval()
    torch.cuda.synchronize()
    per = {}
    reps = max(5, steps // 10)
    for _ in range(reps):
        T.eval()
        torch.cuda.synchronize()
        names = T.trace()["names"]
        for i, nm in enumerate(names):
            per.setdefault(nm, []).append(hip.elapsed_ms(evs[2 * i], evs[2 * i + 1]))
    for e in evs:
        hip.destroy(e)
    T.close()
    alg, design = {}, {}
    for w in wl:
        plan = K.kde_plan_query(w.H, w.n, (w.lo, w.hi, w.M))
        for nm in set(per):
            b = kernel_bytes(nm, w, plan, "f32")
            alg[nm] = alg.get(nm, 0) + b["alg"]
            design[nm] = design.get(nm, 0) + b["design"]
    kern = {}
    for nm, v in per.items():
        us = float(np.sum(v)) / reps * 1e3        # a name can repeat (one launch per padded length)
        kern[nm] = {"us": round(us, 3), "alg_bytes": int(alg[nm]), "alg_GBs": round(alg[nm] / (us * 1e-6) / 1e9, 1),
                    "design_bytes": int(design[nm])}
    n_tot = int(sum(w.n for w in wl))
    cells = int(sum(np.prod(w.M) for w in wl))
    alg_tot = sum(v["alg_bytes"] for v in kern.values())
    best = min(eager_ms, graph_ms)
    B.close()
    return {
        "problems": count, "n_total": n_tot, "grid_pts_total": cells, "launches": info["launches"],
        "tuned_tile": list(info["tile"]), "tuned_narrow_mask": info["narrow_mask"], "tune_s": round(tune_s, 3),
        "ms_per_batch": round(eager_ms, 4), "ms_per_batch_graph": round(graph_ms, 4),
        "ms_per_batch_composite_lengths": round(composite_ms, 4),
        "samples_per_s": round(n_tot / (best * 1e-3), 1), "grid_pts_per_s": round(cells / (best * 1e-3), 1),
        "problems_per_s": round(count / (best * 1e-3), 1),
        "ms_per_item_calls": round(loop_ms, 4), "speedup_vs_item_calls": round(loop_ms / best, 2),
        "item_calls_bit_identical": bool(same),
        "alg_bytes_per_batch": int(alg_tot), "alg_GBs": round(alg_tot / (best * 1e-3) / 1e9, 1),
        "hbm_frac": round(alg_tot / (best * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "design_bytes_per_batch": int(sum(v["design_bytes"] for v in kern.values())), "kernels": kern,
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(W, name: str, reps: int, gpu_density=None):
    """The FP64 oracle on the host, over the same workload, in three legs: (i) the direct
    Eq. (7) sum (the oracle's primary result; `value`), single thread; (ii) the oracle's
    FFT form with NumPy's single-threaded FFT; (iii) the same FFT form through
    scipy.fft with one worker per host core. Each leg includes the oracle's binning and
    lag weights. `gpu_density` ({precision: host array}) is compared with leg (i)'s result:
    max |gpu - oracle| / max |oracle| per precision."""
    import oracle as O
    w = W.WORKLOADS[name]()
    ncpu = os.cpu_count() or 1
    last = {}

    def leg(method, workers, r):
        ts = []
        for _ in range(r):
            t0 = time.perf_counter()
            last[method] = O.kde_binned(w.X, w.H, w.lo, w.hi, w.M, method=method, workers=workers)[0]
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    t_direct = leg("direct", None, reps)
    acc = None
    if gpu_density:
        ref = last["direct"]
        acc = {p: float(np.max(np.abs(np.asarray(f, dtype=np.float64) - ref)) / float(np.max(np.abs(ref))))
               for p, f in gpu_density.items()}
    fft_reps = max(1, reps // 3)
    t_fft = leg("fft", None, fft_reps)
    t_fft_mt = leg("fft", ncpu, fft_reps)
    legs = {
        "direct_1thread": {"s_per_pass": round(t_direct, 4), "samples_per_s": round(w.n / t_direct, 1), "cores": 1,
                           "passes": reps},
        "fft_numpy_1thread": {"s_per_pass": round(t_fft, 4), "samples_per_s": round(w.n / t_fft, 1), "cores": 1,
                              "passes": fft_reps},
        f"fft_scipy_{ncpu}workers": {"s_per_pass": round(t_fft_mt, 4), "samples_per_s": round(w.n / t_fft_mt, 1),
                                     "cores": ncpu, "passes": fft_reps},
    }
    return {"value": round(w.n / t_direct, 1), "unit": "samples/s", "cores": 1, "kind": "oracle",
            "host_cpu": _cpu_model(), "host_cpu_count": ncpu, "legs": legs,
            "max_err_rel_vs_oracle": acc,
            "sample": f"{reps} full FP64 oracle passes over the {name} workload (n={w.n}, grid "
                      f"{'x'.join(map(str, w.M))}): fixed-point binning, lag weights, direct Eq. (7); median "
                      f"{t_direct:.2f} s per pass on one thread (value); beside it the oracle's FFT form "
                      f"(Eq. 12-14) with NumPy ({t_fft:.2f} s) and with scipy.fft on {ncpu} workers "
                      f"({t_fft_mt:.2f} s), {fft_reps} passes each"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {a.gpus}): independent KDEs or haloed slabs of one "
              "KDE would shard across GPUs, but this benchmark runs the single-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1508_02766_amd as K
    import workloads as W
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    hip = Hip(K.lib())
    main_run = measure(K, W, hip, a.workload, a.prec, a.steps, a.warmup)
    variants = {}
    if not a.no_variants:
        chosen = set(a.variants.split(","))
        for name, prec in (("mix2d_512", "f64"), ("mix3d_128", "f32"), ("mix3d_128", "f64"), ("mix4d_48", "f32")):
            if (name, prec) == (a.workload, a.prec) or f"{name}_{prec}" not in chosen:
                continue
            v = measure(K, W, hip, name, prec, max(20, a.steps // 4), 5)
            variants[f"{name}_{prec}"] = {k: v[k] for k in ("ms_per_step", "ms_per_step_traced", "ms_per_step_cold",
                                                            "ms_per_step_graph", "ms_per_step_event_median",
                                                            "ms_per_step_reused_spectrum",
                                                            "ms_per_step_stored_spectrum", "samples_per_s",
                                                            "grid_pts_per_s", "conv_us", "conv_grid_pts_per_s",
                                                            "bin_us", "bin_samples_per_s", "kernels", "steps")}
        if a.batch > 0 and "batch" in chosen:
            variants[f"batch2d_{a.batch}_f32"] = measure_batch(K, W, hip, a.batch, max(20, a.steps // 4), 5)
    # roofline of the dominant kernel of the main workload (method bytes per launch over its
    # kernel-stamped average duration), and of the two steps of the path
    kern = main_run["kernels"]
    dom = max(kern, key=lambda k: kern[k]["us"])
    ach = kern[dom]["alg_bytes"] / (kern[dom]["us"] * 1e-6) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(a.workload, dom) if a.prec == "f32" else None,
            "alg_bytes_per_launch": kern[dom]["alg_bytes"], "design_bytes_per_launch": kern[dom]["design_bytes"],
            "avg_launch_us": kern[dom]["us"], "steps": main_run["steps"]}
    conv_step = main_run["steps"]["fft_convolution"]
    if conv_step:
        roof["fft_convolution_target_frac"] = 0.5
        roof["fft_convolution_gap_to_target"] = round(0.5 - conv_step["frac"], 4)
    for key, v in variants.items():
        if "steps" in v:
            roof[f"steps_{key}"] = v["steps"]
    if a.copy_mb:
        src = torch.ones(a.copy_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cpu = None
    if not a.no_cpu:
        # the workload's density in both precisions, for the oracle comparison
        w = W.WORKLOADS[a.workload]()
        Xd = torch.as_tensor(w.X, device="cuda:0")
        dens = {p: K.kde_eval(Xd, w.H, (w.lo, w.hi, w.M), prec=p)[0].cpu().numpy() for p in ("f32", "f64")}
        del Xd
        cpu = cpu_baseline(W, a.workload, a.cpu_reps, dens)
    line = {
        "metric": "samples/s and grid pts/s for 2-D 512^2 / 3-D 128^3 KDE, FP32 vs FP64, % HBM peak",
        "value": round(main_run["samples_per_s"], 1), "unit": "samples/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(main_run["ms_per_step"], 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": a.prec, "data": "synthetic",
        "config": {"workload": a.workload, "n": main_run["n"], "grid": main_run["M"], "L": main_run["L"],
                   "P": main_run["P"], "H": "full SPD"},
        "grid_pts_per_s": round(main_run["grid_pts_per_s"], 1),
        "conv_grid_pts_per_s": round(main_run["conv_grid_pts_per_s"], 1),
        "bin_samples_per_s": round(main_run["bin_samples_per_s"], 1),
        "ms_per_step_traced": round(main_run["ms_per_step_traced"], 5),
        "ms_per_step_cold": round(main_run["ms_per_step_cold"], 5),
        "ms_per_step_graph": round(main_run["ms_per_step_graph"], 5),
        "ms_per_step_event_median": round(main_run["ms_per_step_event_median"], 5),
        "ms_per_step_reused_spectrum": round(main_run["ms_per_step_reused_spectrum"], 5),
        "ms_per_step_stored_spectrum": round(main_run["ms_per_step_stored_spectrum"], 5),
        "gpu_ms_per_step_traced": round(main_run["gpu_ms_per_step_traced"], 5),
        "kernels": kern, "roofline": roof, "cpu_baseline": cpu, "variants": variants,
    }
    if cpu and cpu.get("max_err_rel_vs_oracle"):
        # max |density - oracle's direct Eq. (7)| / max |oracle| over the whole grid, both precisions
        line["max_err_rel_vs_oracle"] = cpu["max_err_rel_vs_oracle"]
    # the same workload with FP64 transforms (the precision the paper computes in), beside the headline
    f64 = variants.get(f"{a.workload}_f64")
    if a.prec == "f32" and f64:
        line["fp64_same_workload"] = {"ms_per_step": round(f64["ms_per_step"], 5),
                                      "samples_per_s": round(f64["samples_per_s"], 1),
                                      "grid_pts_per_s": round(f64["grid_pts_per_s"], 1)}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
