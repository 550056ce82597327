"""ctypes binding of libkde.so, the gfx950 binned FFT KDE library.

Argument marshalling only: every step of the estimate runs in the library's
HIP kernels. PyTorch supplies device memory (tensors) and the current stream.
The names and semantics follow include/kde.h:

    kde_grid_from_data(X, H, M, nsd)            -> KdeGrid (host, data range +- nsd sqrt(H_kk))
    kde_plan_query(H, n, grid, **opts)          -> dict (host planner, no device work)
    kde_bin(X, grid, **opts)                    -> (counts, n_dropped)
    kde_kernel_grid(H, n, grid, **opts)         -> lag-box weights
    kde_conv(counts, n, H, grid, **opts)        -> density from counts
    kde_eval(X, H, grid, **opts)                -> (density, n_dropped)
    kde_lscv(counts, n, H, grid, **opts)        -> LSCV objective and its two terms
    KdeBatch(items, **opts)                     -> kde_batch_create / _bind / _eval / _tune
    KdeLscvBatch(problems, **opts)              -> kde_lscv_batch_create, then the same calls
    kde_strerror(code)                          -> str

``grid`` is ``(lo, hi, M)`` (per-axis sequences) or a ``KdeGrid``. Options:
``prec`` ("f32" default, or "f64"), ``tau``, ``L`` (per-axis override),
``Q`` (fixed-point bits), ``tile`` (binning tile per axis), ``extent`` ("eigen" = Eq. 15,
"marginal" = tau sqrt(H_kk) per axis), ``reuse_spectrum`` (the workspace holds the kernel spectrum
of an earlier call with the same H, n, grid and options), ``store_spectrum`` (keep the whole real
spectrum for the product pass), ``lengths`` ("auto", "composite": 3 x 2^k also in 2-D, "pow2"),
``trace_events`` (list of raw hipEvent_t handles
as ints, used in pairs: pass i stamps events 2i and 2i + 1 with its kernel's start and end) with
``trace`` (a dict that receives ``count``, the number of passes stamped, and their ``names``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

# KDE_LIBRARY may name another build of the same library (same ABI), e.g. for a tuning sweep.
_LIB_PATH = os.environ.get("KDE_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkde.so")

KDE_F32, KDE_F64 = 1, 2
_PREC = {"f32": KDE_F32, "f64": KDE_F64, KDE_F32: KDE_F32, KDE_F64: KDE_F64, None: KDE_F32}
_TDTYPE = {KDE_F32: torch.float32, KDE_F64: torch.float64}


class KdeError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {kde_strerror(code)} (status {code})")
        self.code = code


MAX_D = 4   # KDE_MAX_D


class KdeGrid(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("reserved", ctypes.c_int32), ("M", ctypes.c_int64 * MAX_D),
                ("lo", ctypes.c_double * MAX_D), ("hi", ctypes.c_double * MAX_D)]


class KdeParams(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("L", ctypes.c_int32 * MAX_D), ("Q", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("tile", ctypes.c_int32 * MAX_D), ("extent", ctypes.c_int32), ("reuse_spectrum", ctypes.c_int32),
                ("store_spectrum", ctypes.c_int32), ("lengths", ctypes.c_int32),
                ("trace_capacity", ctypes.c_int32),
                ("trace_events", ctypes.POINTER(ctypes.c_void_p)), ("trace_count", ctypes.POINTER(ctypes.c_int32)),
                ("trace_names", ctypes.POINTER(ctypes.c_char_p))]


class KdePlan(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("Q", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("L", ctypes.c_int32 * MAX_D), ("P", ctypes.c_int32 * MAX_D), ("reserved", ctypes.c_int32),
                ("delta", ctypes.c_double * MAX_D), ("lambda_max", ctypes.c_double), ("det_H", ctypes.c_double),
                ("norm", ctypes.c_double), ("lag_count", ctypes.c_int64), ("lag_bytes", ctypes.c_size_t),
                ("conv_ws_bytes", ctypes.c_size_t), ("eval_ws_bytes", ctypes.c_size_t),
                ("density_bytes", ctypes.c_size_t), ("bin_ws_bytes", ctypes.c_size_t),
                ("lscv_ws_bytes", ctypes.c_size_t)]


class KdeBatchItem(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("n", ctypes.c_int64), ("H", ctypes.c_double * (MAX_D * MAX_D)), ("grid", KdeGrid),
                ("density", ctypes.c_void_p), ("n_dropped", ctypes.c_void_p), ("counts", ctypes.c_void_p),
                ("dot", ctypes.c_void_p)]


class KdeLscvItem(ctypes.Structure):
    _fields_ = [("counts", ctypes.c_void_p), ("n", ctypes.c_int64), ("H", ctypes.c_double * (MAX_D * MAX_D)), ("grid", KdeGrid),
                ("out", ctypes.c_void_p)]


class KdeBatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("launches", ctypes.c_int32), ("ws_bytes", ctypes.c_size_t),
                ("tile", ctypes.c_int32 * MAX_D), ("narrow_mask", ctypes.c_int32)]


class KdeMlpInfo(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("rows_per_group", ctypes.c_int32), ("n_params", ctypes.c_int64), ("state_bytes", ctypes.c_size_t),
                ("ws_bytes", ctypes.c_size_t)]


_lib = None
EXPORTS = ("kde_grid_from_data", "kde_plan_query", "kde_bin", "kde_kernel_grid", "kde_conv", "kde_eval",
           "kde_eval_noalloc", "kde_lscv", "kde_mlp_query", "kde_mlp_load", "kde_mlp_forward",
           "kde_mlp_grad", "kde_mlp_train_step", "kde_batch_create",
           "kde_batch_query", "kde_batch_bind", "kde_batch_eval", "kde_batch_tune", "kde_batch_destroy",
           "kde_lscv_batch_create",
           "kde_strerror")


def library_path() -> str:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_1508_02766_amd.build` "
                              "(there is no CPU fallback for the estimator)")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
        G, Pp = ctypes.POINTER(KdeGrid), ctypes.POINTER(KdeParams)
        L.kde_grid_from_data.argtypes = [vp, i64, ctypes.c_int32, vp, ctypes.c_double, i64, G]
        L.kde_plan_query.argtypes = [vp, i64, G, Pp, ctypes.POINTER(KdePlan)]
        L.kde_bin.argtypes = [vp, i64, G, Pp, vp, vp, vp, sz, vp]
        L.kde_kernel_grid.argtypes = [vp, i64, G, Pp, vp, sz, vp]
        L.kde_conv.argtypes = [vp, i64, vp, G, Pp, vp, vp, sz, vp]
        L.kde_eval.argtypes = [vp, i64, vp, G, Pp, vp, vp, sz, vp, vp]
        L.kde_eval_noalloc.argtypes = [vp, i64, vp, G, Pp, vp, vp, vp]
        L.kde_lscv.argtypes = [vp, i64, vp, G, Pp, vp, vp, sz, vp]
        L.kde_mlp_query.argtypes = [i64, ctypes.POINTER(KdeMlpInfo)]
        L.kde_mlp_load.argtypes = [vp, vp, vp]
        L.kde_mlp_forward.argtypes = [vp, vp, i64, vp, vp, sz, vp]
        L.kde_mlp_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]
        L.kde_mlp_train_step.argtypes = [vp, vp, vp, i64, ctypes.c_float, ctypes.c_int32, vp, vp, sz, vp]
        L.kde_batch_create.argtypes = [ctypes.POINTER(KdeBatchItem), ctypes.c_int32, Pp, ctypes.POINTER(vp)]
        L.kde_lscv_batch_create.argtypes = [ctypes.POINTER(KdeLscvItem), ctypes.c_int32, Pp, ctypes.POINTER(vp)]
        L.kde_batch_query.argtypes = [vp, ctypes.POINTER(KdeBatchInfo)]
        L.kde_batch_bind.argtypes = [vp, vp, sz, vp]
        L.kde_batch_eval.argtypes = [vp, vp]
        L.kde_batch_tune.argtypes = [vp, ctypes.c_int32, vp]
        L.kde_batch_destroy.argtypes = [vp]
        L.kde_batch_destroy.restype = None
        L.kde_strerror.argtypes = [ctypes.c_int]
        L.kde_strerror.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("kde_strerror", "kde_batch_destroy"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def kde_strerror(code: int) -> str:
    return lib().kde_strerror(int(code)).decode()


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def make_grid(lo, hi, M) -> KdeGrid:
    lo = np.atleast_1d(np.asarray(lo, dtype=np.float64))
    hi = np.atleast_1d(np.asarray(hi, dtype=np.float64))
    M = np.atleast_1d(np.asarray(M, dtype=np.int64))
    d = int(M.size)
    if lo.size != d or hi.size != d or not 1 <= d <= MAX_D:
        raise ValueError(f"lo, hi and M need one entry per axis, 1 <= d <= {MAX_D}")
    g = KdeGrid()
    g.d = d
    for k in range(d):
        g.M[k], g.lo[k], g.hi[k] = int(M[k]), float(lo[k]), float(hi[k])
    return g


def _grid(grid) -> KdeGrid:
    return grid if isinstance(grid, KdeGrid) else make_grid(*grid)


def _grid_shape(g: KdeGrid):
    return tuple(int(g.M[k]) for k in range(g.d))


def _params(prec=None, tau=None, L=None, Q=None, tile=None, extent=None, reuse_spectrum=None, store_spectrum=None,
            lengths=None, trace_events=None,
            trace=None):
    p = KdeParams()
    if reuse_spectrum:
        p.reuse_spectrum = 1
    if store_spectrum:
        p.store_spectrum = 1
    if lengths is not None:
        p.lengths = {"auto": 0, "composite": 1, "pow2": 2}.get(lengths, lengths)
    if extent is not None:
        p.extent = {"eigen": 0, "marginal": 1}.get(extent, extent)
    if tile is not None:
        for k, v in enumerate(tile):
            p.tile[k] = int(v)
    p.prec = _PREC.get(prec, prec)
    if tau is not None:
        p.tau = float(tau)
    if L is not None:
        for k, v in enumerate(L):
            p.L[k] = int(v)
    if Q is not None:
        p.Q = int(Q)
    keep = []
    if trace_events:
        arr = (ctypes.c_void_p * len(trace_events))(*[int(e) for e in trace_events])
        cnt = ctypes.c_int32(0)
        names = (ctypes.c_char_p * max(len(trace_events) // 2, 1))()
        p.trace_capacity = len(trace_events)
        p.trace_events = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        p.trace_count = ctypes.pointer(cnt)
        p.trace_names = ctypes.cast(names, ctypes.POINTER(ctypes.c_char_p))
        keep = [arr, cnt, names, trace]
    return p, keep


def _finish_trace(keep):
    if keep and keep[3] is not None:
        arr, cnt, names, trace = keep
        n = cnt.value
        trace["count"] = n
        trace["names"] = [names[i].decode() for i in range(n)]


def _H(H, d: int):
    Hn = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(d, d))
    return Hn, Hn.ctypes.data_as(ctypes.c_void_p)


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check(code: int, where: str):
    if code != 0:
        raise KdeError(code, where)


def _need_cuda(t: torch.Tensor, dtype, name: str):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor")


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------

def kde_grid_from_data(X, H, M: int, nsd: float = 3.0) -> KdeGrid:
    """Grid box around host samples X (n, d): data range widened by nsd sqrt(H_kk) per side."""
    Xn = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
    if Xn.ndim != 2:
        raise ValueError("X must be (n, d)")
    n, d = Xn.shape
    Hn, Hp = _H(H, d)
    g = KdeGrid()
    _check(lib().kde_grid_from_data(Xn.ctypes.data_as(ctypes.c_void_p), n, d, Hp, float(nsd), int(M),
                                    ctypes.byref(g)), "kde_grid_from_data")
    return g


def grid_tuple(g: KdeGrid):
    """(lo, hi, M) of a KdeGrid as NumPy arrays and a tuple."""
    return (np.array([g.lo[k] for k in range(g.d)]), np.array([g.hi[k] for k in range(g.d)]),
            tuple(int(g.M[k]) for k in range(g.d)))


def kde_plan_query(H, n: int, grid, **opts) -> dict:
    """Host plan; with H None only the binning quantities are filled (n >= 0)."""
    g = _grid(grid)
    p, _ = _params(**opts)
    if H is None:
        Hn, Hp = None, ctypes.c_void_p(0)
    else:
        Hn, Hp = _H(H, g.d)
    out = KdePlan()
    _check(lib().kde_plan_query(Hp, int(n), ctypes.byref(g), ctypes.byref(p), ctypes.byref(out)), "kde_plan_query")
    d = out.d
    return {
        "d": d, "Q": out.Q, "prec": out.prec, "L": tuple(out.L[:d]), "P": tuple(out.P[:d]),
        "delta": tuple(out.delta[:d]), "lambda_max": out.lambda_max, "det_H": out.det_H, "norm": out.norm,
        "lag_count": out.lag_count, "lag_bytes": out.lag_bytes, "conv_ws_bytes": out.conv_ws_bytes,
        "eval_ws_bytes": out.eval_ws_bytes, "density_bytes": out.density_bytes,
        "bin_ws_bytes": out.bin_ws_bytes, "lscv_ws_bytes": out.lscv_ws_bytes,
    }


_PLAN_OPTS = ("prec", "tau", "L", "Q", "tile", "extent", "store_spectrum", "lengths")


def _workspace(nbytes: int, device, ws=None) -> torch.Tensor:
    if ws is None:
        ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if ws.numel() < nbytes or ws.data_ptr() % 256:
        raise ValueError("workspace too small or not 256-byte aligned")
    return ws


def kde_bin(X: torch.Tensor, grid, counts=None, n_dropped=None, ws=None, **opts):
    """Fixed-point counts (uint64 in units 2^-dQ, returned as a torch.uint64 tensor) and n_dropped."""
    g = _grid(grid)
    _need_cuda(X, torch.float64, "X")
    if X.dim() != 2 or X.shape[1] != g.d:
        raise ValueError("X must be (n, d)")
    dev = X.device
    if counts is None:
        counts = torch.empty(_grid_shape(g), dtype=torch.uint64, device=dev)
    if n_dropped is None:
        n_dropped = torch.empty(1, dtype=torch.uint64, device=dev)
    need = kde_plan_query(None, X.shape[0], g, **{k: v for k, v in opts.items() if k in ("Q", "tile")})["bin_ws_bytes"]
    ws = _workspace(need, dev, ws) if need else ws
    p, keep = _params(**opts)
    _check(lib().kde_bin(_ptr(X), X.shape[0], ctypes.byref(g), ctypes.byref(p), _ptr(counts), _ptr(n_dropped),
                         _ptr(ws), ws.numel() if ws is not None else 0, _stream(dev)), "kde_bin")
    _finish_trace(keep)
    return counts, n_dropped


def kde_kernel_grid(H, n: int, grid, out=None, device="cuda", **opts) -> torch.Tensor:
    g = _grid(grid)
    plan = kde_plan_query(H, n, g, **{k: v for k, v in opts.items() if k in _PLAN_OPTS})
    shape = tuple(2 * L + 1 for L in plan["L"])
    dt = _TDTYPE[plan["prec"]]
    if out is None:
        out = torch.empty(shape, dtype=dt, device=device)
    _need_cuda(out, dt, "out")
    p, keep = _params(**opts)
    Hn, Hp = _H(H, g.d)
    _check(lib().kde_kernel_grid(Hp, int(n), ctypes.byref(g), ctypes.byref(p), _ptr(out),
                                 out.numel() * out.element_size(), _stream(out.device)), "kde_kernel_grid")
    _finish_trace(keep)
    return out


def kde_conv(counts: torch.Tensor, n: int, H, grid, out=None, ws=None, **opts) -> torch.Tensor:
    g = _grid(grid)
    if not (counts.is_cuda and counts.dtype in (torch.uint64, torch.int64) and counts.is_contiguous()):
        raise TypeError("counts must be a contiguous uint64 CUDA tensor")
    plan = kde_plan_query(H, n, g, **{k: v for k, v in opts.items() if k in _PLAN_OPTS})
    dt = _TDTYPE[plan["prec"]]
    dev = counts.device
    if out is None:
        out = torch.empty(_grid_shape(g), dtype=dt, device=dev)
    _need_cuda(out, dt, "out")
    ws = _workspace(plan["conv_ws_bytes"], dev, ws)
    p, keep = _params(**opts)
    Hn, Hp = _H(H, g.d)
    _check(lib().kde_conv(_ptr(counts), int(n), Hp, ctypes.byref(g), ctypes.byref(p), _ptr(out), _ptr(ws),
                          ws.numel(), _stream(dev)), "kde_conv")
    _finish_trace(keep)
    return out


def kde_eval(X: torch.Tensor, H, grid, out=None, ws=None, n_dropped=None, **opts):
    """The binned estimate on the grid (Eq. 7) and the number of samples outside the grid box."""
    g = _grid(grid)
    _need_cuda(X, torch.float64, "X")
    if X.dim() != 2 or X.shape[1] != g.d:
        raise ValueError("X must be (n, d)")
    n = X.shape[0]
    plan = kde_plan_query(H, n, g, **{k: v for k, v in opts.items() if k in _PLAN_OPTS})
    dt = _TDTYPE[plan["prec"]]
    dev = X.device
    if out is None:
        out = torch.empty(_grid_shape(g), dtype=dt, device=dev)
    _need_cuda(out, dt, "out")
    ws = _workspace(plan["eval_ws_bytes"], dev, ws)
    if n_dropped is None:
        n_dropped = torch.empty(1, dtype=torch.uint64, device=dev)
    p, keep = _params(**opts)
    Hn, Hp = _H(H, g.d)
    _check(lib().kde_eval(_ptr(X), n, Hp, ctypes.byref(g), ctypes.byref(p), _ptr(out), _ptr(ws), ws.numel(),
                          _ptr(n_dropped), _stream(dev)), "kde_eval")
    _finish_trace(keep)
    return out, n_dropped


NOALLOC_SCRATCH_BYTES = 256 << 20     # KDE_NOALLOC_SCRATCH_BYTES


def kde_eval_noalloc(X: torch.Tensor, H, grid, out: torch.Tensor, n_dropped=None, **opts):
    """kde_eval with the library's fixed device scratch as workspace (no device
    allocation in the library; out and n_dropped are the caller's)."""
    g = _grid(grid)
    _need_cuda(X, torch.float64, "X")
    if X.dim() != 2 or X.shape[1] != g.d:
        raise ValueError("X must be (n, d)")
    p, keep = _params(**opts)
    Hn, Hp = _H(H, g.d)
    _check(lib().kde_eval_noalloc(_ptr(X), X.shape[0], Hp, ctypes.byref(g), ctypes.byref(p), _ptr(out),
                                  _ptr(n_dropped), _stream(X.device)), "kde_eval_noalloc")
    _finish_trace(keep)
    return out, n_dropped


def kde_lscv(counts: torch.Tensor, n: int, H, grid, out=None, ws=None, **opts) -> torch.Tensor:
    """LSCV(H) from fixed-point counts: a float64 CUDA tensor {LSCV, first term, second term}."""
    g = _grid(grid)
    if not (counts.is_cuda and counts.dtype in (torch.uint64, torch.int64) and counts.is_contiguous()):
        raise TypeError("counts must be a contiguous uint64 CUDA tensor")
    plan = kde_plan_query(H, n, g, **{k: v for k, v in opts.items() if k in _PLAN_OPTS})
    if plan["lscv_ws_bytes"] == 0:
        raise ValueError("LSCV needs n >= 2 and padded lengths <= 4096 for 2H")
    dev = counts.device
    if out is None:
        out = torch.empty(3, dtype=torch.float64, device=dev)
    _need_cuda(out, torch.float64, "out")
    ws = _workspace(plan["lscv_ws_bytes"], dev, ws)
    p, keep = _params(**opts)
    Hn, Hp = _H(H, g.d)
    _check(lib().kde_lscv(_ptr(counts), int(n), Hp, ctypes.byref(g), ctypes.byref(p), _ptr(out), _ptr(ws),
                          ws.numel(), _stream(dev)), "kde_lscv")
    _finish_trace(keep)
    return out


class PreparedCall:
    """A library call with every argument marshalled once, for repeated launches
    (benchmarks, serving loops): ``call()`` enqueues the work on the stream that
    was current when it was prepared and raises on a non-zero status."""

    def __init__(self, fn, args, keep, name):
        self._fn, self._args, self._keep, self._name = fn, args, keep, name

    def __call__(self):
        _check(self._fn(*self._args), self._name)

    def trace(self) -> dict:
        out = {}
        if self._keep:
            arr, cnt, names, _ = self._keep
            _finish_trace([arr, cnt, names, out])
        return out


def prepare_eval(X: torch.Tensor, H, grid, out: torch.Tensor, ws: torch.Tensor, n_dropped=None,
                 **opts) -> PreparedCall:
    g = _grid(grid)
    _need_cuda(X, torch.float64, "X")
    p, keep = _params(**opts)
    Hn, Hp = _H(H, g.d)
    args = (_ptr(X), X.shape[0], Hp, ctypes.byref(g), ctypes.byref(p), _ptr(out), _ptr(ws), ws.numel(),
            _ptr(n_dropped), _stream(X.device))
    return _Prepared(lib().kde_eval, args, keep, (g, p, Hn), "kde_eval")


def prepare_conv(counts: torch.Tensor, n: int, H, grid, out: torch.Tensor, ws: torch.Tensor, **opts) -> PreparedCall:
    g = _grid(grid)
    p, keep = _params(**opts)
    Hn, Hp = _H(H, g.d)
    args = (_ptr(counts), int(n), Hp, ctypes.byref(g), ctypes.byref(p), _ptr(out), _ptr(ws), ws.numel(),
            _stream(counts.device))
    return _Prepared(lib().kde_conv, args, keep, (g, p, Hn), "kde_conv")


def prepare_bin(X: torch.Tensor, grid, counts: torch.Tensor, n_dropped=None, ws=None, **opts) -> PreparedCall:
    g = _grid(grid)
    _need_cuda(X, torch.float64, "X")
    p, keep = _params(**opts)
    args = (_ptr(X), X.shape[0], ctypes.byref(g), ctypes.byref(p), _ptr(counts), _ptr(n_dropped),
            _ptr(ws), ws.numel() if ws is not None else 0, _stream(X.device))
    return _Prepared(lib().kde_bin, args, keep, (g, p), "kde_bin")


class _Prepared(PreparedCall):
    def __init__(self, fn, args, keep, owned, name):
        super().__init__(fn, args, keep, name)
        self._owned = owned          # keeps the ctypes structs and H alive


class KdeBatch:
    """Many independent estimates in one batched pipeline (kde_batch_*).

    ``items`` is a sequence of ``(X, H, grid)`` with X a contiguous (n, d)
    float64 CUDA tensor, or ``(counts, n, H, grid)`` with fixed-point counts
    (uint64 CUDA tensor, as kde_bin writes them). The densities
    (``self.densities``, one tensor per item) and the workspace are allocated
    here with torch; the batch is bound on the current stream. ``eval()``
    enqueues the whole batch (capturable in a CUDA/HIP graph), ``tune(reps)``
    runs the library's autotuner. With ``dots=True``, ``self.dots`` (float64,
    one entry per item) receives sum_j c_j f_j at every eval.
    """

    def __init__(self, items, n_dropped: bool = False, dots: bool = False, **opts):
        self._X = []
        arr = (KdeBatchItem * len(items))()
        p, keep = _params(**opts)
        prec = _PREC.get(opts.get("prec"), opts.get("prec"))
        dt = _TDTYPE[prec]
        first = items[0][0]
        dev = first.device
        self.dots = torch.zeros(len(items), dtype=torch.float64, device=dev) if dots else None
        # one allocation for all densities (and dropped-sample counters): item i's density
        # starts on a 256-byte boundary at element self._offs[i]; `densities` are views
        grids = [_grid(item[-1]) for item in items]
        self._shapes = [_grid_shape(g) for g in grids]
        esize = torch.empty(0, dtype=dt).element_size()
        align = 256 // esize
        offs, total = [], 0
        for shp in self._shapes:
            offs.append(total)
            cells = 1
            for m in shp:
                cells *= m
            total += -(-cells // align) * align
        self._offs = offs
        self._dens_buf = torch.empty(max(total, 1), dtype=dt, device=dev)
        self._nd_buf = torch.empty(len(items), dtype=torch.uint64, device=dev) if n_dropped else None
        dbase = self._dens_buf.data_ptr()
        ndbase = self._nd_buf.data_ptr() if n_dropped else 0
        dotbase = self.dots.data_ptr() if dots else 0
        for i, item in enumerate(items):
            it = arr[i]
            g = grids[i]
            if len(item) == 4:
                C, n, H, _ = item
                if not (C.is_cuda and C.dtype in (torch.uint64, torch.int64) and C.is_contiguous()):
                    raise TypeError("counts must be a contiguous uint64 CUDA tensor")
                it.counts = C.data_ptr()
                it.n = int(n)
                X = C
            else:
                X, H, _ = item
                _need_cuda(X, torch.float64, "X")
                if X.dim() != 2 or X.shape[1] != g.d:
                    raise ValueError("X must be (n, d)")
                it.X = X.data_ptr()
                it.n = X.shape[0]
            if X.device != dev:
                raise ValueError("all items of a batch must be on one device")
            Hn = np.asarray(H, dtype=np.float64)
            if Hn.size != g.d * g.d:
                raise ValueError("H must be d x d")
            it.H[:g.d * g.d] = Hn.ravel().tolist()
            it.grid = g
            it.density = dbase + esize * offs[i]
            if dots:
                it.dot = dotbase + 8 * i
            if n_dropped:
                it.n_dropped = ndbase + 8 * i
            self._X.append(X)
        self.device = dev
        self._params, self._keep = p, keep
        self._items = arr
        h = ctypes.c_void_p(0)
        _check(lib().kde_batch_create(arr, len(items), ctypes.byref(p), ctypes.byref(h)), "kde_batch_create")
        self._h = h
        self.ws = torch.empty(max(self.info()["ws_bytes"], 1), dtype=torch.uint8, device=dev)
        if self.ws.data_ptr() % 256:
            raise RuntimeError("workspace not 256-byte aligned")
        _check(lib().kde_batch_bind(self._h, _ptr(self.ws), self.ws.numel(), _stream(dev)), "kde_batch_bind")
        self._stream = _stream(dev)

    @property
    def densities(self) -> list:
        """One tensor per item (views of the batch's density buffer)."""
        if getattr(self, "_dens_views", None) is None:
            self._dens_views = [self._dens_buf[o:o + int(np.prod(shp))].view(shp)
                                for o, shp in zip(self._offs, self._shapes)]
        return self._dens_views

    @property
    def n_dropped(self) -> list:
        """One single-element uint64 tensor per item (with ``n_dropped=True``)."""
        if self._nd_buf is None:
            return []
        return [self._nd_buf[i:i + 1] for i in range(self._nd_buf.numel())]

    def info(self) -> dict:
        inf = KdeBatchInfo()
        _check(lib().kde_batch_query(self._h, ctypes.byref(inf)), "kde_batch_query")
        return {"count": inf.count, "launches": inf.launches, "ws_bytes": inf.ws_bytes, "tile": tuple(inf.tile),
                "narrow_mask": inf.narrow_mask}

    def eval(self):
        _check(lib().kde_batch_eval(self._h, _stream(self.device)), "kde_batch_eval")

    def tune(self, reps: int = 3) -> dict:
        _check(lib().kde_batch_tune(self._h, int(reps), _stream(self.device)), "kde_batch_tune")
        return self.info()

    def trace(self) -> dict:
        out = {}
        if self._keep:
            arr, cnt, names, _ = self._keep
            _finish_trace([arr, cnt, names, out])
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().kde_batch_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class KdeLscvBatch:
    """LSCV objectives of many problems in one batched pipeline (kde_lscv_batch_create).

    ``problems`` is a sequence of ``(counts, n, H, grid)`` with fixed-point
    counts (uint64 CUDA tensor, as kde_bin writes them). ``self.out`` (float64,
    problems x 3) receives {LSCV, first term, second term} of every problem at
    each ``eval()``, bit-identical to kde_lscv of the same problem.
    """

    def __init__(self, problems, **opts):
        arr = (KdeLscvItem * len(problems))()
        p, keep = _params(**opts)
        dev = problems[0][0].device
        self.out = torch.empty((len(problems), 3), dtype=torch.float64, device=dev)
        self._counts = []
        base = self.out.data_ptr()
        for i, (C, n, H, grid) in enumerate(problems):
            if not (C.is_cuda and C.dtype in (torch.uint64, torch.int64) and C.is_contiguous()):
                raise TypeError("counts must be a contiguous uint64 CUDA tensor")
            if C.device != dev:
                raise ValueError("all problems of a batch must be on one device")
            g = _grid(grid)
            Hn = np.asarray(H, dtype=np.float64)
            if Hn.size != g.d * g.d:
                raise ValueError("H must be d x d")
            it = arr[i]
            it.counts = C.data_ptr()
            it.n = int(n)
            it.H[:g.d * g.d] = Hn.ravel().tolist()
            it.grid = g
            it.out = base + 24 * i
            self._counts.append(C)
        self.device = dev
        self._params, self._keep, self._items = p, keep, arr
        h = ctypes.c_void_p(0)
        _check(lib().kde_lscv_batch_create(arr, len(problems), ctypes.byref(p), ctypes.byref(h)),
               "kde_lscv_batch_create")
        self._h = h
        self.ws = torch.empty(max(self.info()["ws_bytes"], 1), dtype=torch.uint8, device=dev)
        _check(lib().kde_batch_bind(self._h, _ptr(self.ws), self.ws.numel(), _stream(dev)), "kde_batch_bind")

    info = KdeBatch.info
    eval = KdeBatch.eval
    tune = KdeBatch.tune
    trace = KdeBatch.trace
    close = KdeBatch.close
    __del__ = KdeBatch.__del__


def mlp_query(batch: int = 0) -> dict:
    inf = KdeMlpInfo()
    _check(lib().kde_mlp_query(int(batch), ctypes.byref(inf)), "kde_mlp_query")
    return {"n_in": inf.n_in, "n_hidden": inf.n_hidden, "n_out": inf.n_out, "rows_per_group": inf.rows_per_group,
            "n_params": inf.n_params, "state_bytes": inf.state_bytes, "ws_bytes": inf.ws_bytes}


class MlpNet:
    """The learned-bandwidth network (kde_mlp_*): device state allocated with torch."""

    def __init__(self, params, device="cuda:0"):
        info = mlp_query()
        self.n_params = info["n_params"]
        self.device = device
        self.state = torch.empty(info["state_bytes"], dtype=torch.uint8, device=device)
        self._ws = torch.empty(1, dtype=torch.uint8, device=device)
        self.load(params)

    def load(self, params):
        p = torch.as_tensor(np.asarray(params, dtype=np.float32), device=self.device).contiguous()
        if p.numel() != self.n_params:
            raise ValueError(f"need {self.n_params} parameters")
        _check(lib().kde_mlp_load(_ptr(self.state), _ptr(p), _stream(self.device)), "kde_mlp_load")
        torch.cuda.current_stream(self.device).synchronize()

    def params(self) -> np.ndarray:
        return self.state[: self.n_params * 4].view(torch.float32).cpu().numpy().astype(np.float64)

    def _ws_for(self, B):
        need = mlp_query(B)["ws_bytes"]
        if self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def forward(self, X: torch.Tensor, Y=None) -> torch.Tensor:
        _need_cuda(X, torch.float32, "X")
        B = X.shape[0]
        if Y is None:
            Y = torch.empty(B, 3, dtype=torch.float32, device=self.device)
        _check(lib().kde_mlp_forward(_ptr(self.state), _ptr(X), B, _ptr(Y), None, 0, _stream(self.device)),
               "kde_mlp_forward")
        return Y

    def grad(self, X: torch.Tensor, T: torch.Tensor):
        _need_cuda(X, torch.float32, "X")
        _need_cuda(T, torch.float32, "T")
        B = X.shape[0]
        ws = self._ws_for(B)
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        Y = torch.empty(B, 3, dtype=torch.float32, device=self.device)
        _check(lib().kde_mlp_grad(_ptr(self.state), _ptr(X), _ptr(T), B, _ptr(Y), _ptr(g), _ptr(loss), _ptr(ws),
                                  ws.numel(), _stream(self.device)), "kde_mlp_grad")
        return g, loss, Y

    def train_step(self, X: torch.Tensor, T: torch.Tensor, lr: float, step: int, loss=None):
        B = X.shape[0]
        ws = self._ws_for(B)
        _check(lib().kde_mlp_train_step(_ptr(self.state), _ptr(X), _ptr(T), B, float(lr), int(step), _ptr(loss),
                                        _ptr(ws), ws.numel(), _stream(self.device)), "kde_mlp_train_step")
        return loss
