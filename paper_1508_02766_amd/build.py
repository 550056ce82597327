"""Build step of the gfx950 library: compiles csrc/ with hipcc into libkde.so.

Run as ``python -m paper_1508_02766_amd.build`` or through ``build()``.
Every call recompiles (sources are few); objects go to ``_build/`` beside the
package and the shared library into the package directory.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libkde.so")

ARCH = "gfx950"
COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]
# per-source extra flags: binning must not fuse or approximate its FP64 arithmetic
SOURCES = {
    "kde_bin.hip": ["-ffp-contract=off", "-fno-fast-math"],
    "kde_fused.hip": ["-ffp-contract=off", "-fno-fast-math"],
    # FFT kernels: explicit fused multiply-adds only, so that every kernel built
    # from the same device code rounds identically
    "kde_fft.hip": ["-ffp-contract=off"],
    "kde_fft_batch.hip": ["-ffp-contract=off"],
    "kde_lscv.hip": ["-ffp-contract=off"],
    "kde_mlp.hip": ["-ffp-contract=off"],
    "kde_static.hip": [],
    "kde_api.cpp": [],
}


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = []
    for src, extra in SOURCES.items():
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(([hipcc, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for r in ex.map(lambda j: _run(j[0]), jobs):
            if verbose and r.stderr:
                print(r.stderr, file=sys.stderr)
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *[o for _, o in jobs], "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
