"""MI355X-native binned FFT kernel density estimation with an unconstrained
bandwidth matrix (Gramacki & Gramacki, arXiv 1508.02766).

The estimator runs in gfx950 HIP kernels behind the C ABI of include/kde.h
(libkde.so); this package is its ctypes binding.
"""
from .kde import (  # noqa: F401
    EXPORTS, KDE_F32, KDE_F64, KdeBatch, KdeLscvBatch, KdeError, KdeGrid, MlpNet, mlp_query, PreparedCall, kde_bin, kde_conv, kde_eval, kde_eval_noalloc, NOALLOC_SCRATCH_BYTES, kde_grid_from_data, kde_kernel_grid, kde_lscv,
    grid_tuple,
    kde_plan_query, kde_strerror, lib, library_path, make_grid, prepare_bin, prepare_conv, prepare_eval,
)
from . import lscv  # noqa: F401,E402
