"""ctypes access to libtkgen.so, the C/HIP build of the input recipes.

Holds no Top-K arithmetic.  ``build()`` compiles ``gen.hip`` in place.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import KIND_DTYPE

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gen.hip")
LIB = os.path.join(HERE, "libtkgen.so")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["/opt/rocm/bin/hipcc", *HIP_FLAGS, SRC, "-o", LIB + ".tmp", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building libtkgen.so failed:\n" + r.stderr)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print(" ".join(cmd))
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        u64, vp = ctypes.c_uint64, ctypes.c_void_p
        L.tkgen_host.argtypes = [ctypes.c_int, u64, u64, u64, u64, vp, u64, vp, ctypes.c_int]
        L.tkgen_host.restype = ctypes.c_int
        L.tkgen_device.argtypes = [ctypes.c_int, u64, u64, u64, u64, vp, u64, vp, vp]
        L.tkgen_device.restype = ctypes.c_int
        _lib = L
    return _lib


def host_fill(kind: int, seed: int, n: int, start: int = 0, n_total: int | None = None,
              cdf: np.ndarray | None = None, nthreads: int | None = None) -> np.ndarray:
    """Host array of elements start..start+n-1 (multi-threaded C)."""
    if n_total is None:
        n_total = start + n
    out = np.empty(n, dtype=KIND_DTYPE[kind])
    if nthreads is None:
        nthreads = min(16, len(os.sched_getaffinity(0)))
    cptr = cdf.ctypes.data if cdf is not None else None
    m = 0 if cdf is None else len(cdf)
    rc = lib().tkgen_host(kind, seed % (1 << 64), start, n, n_total, cptr, m,
                          out.ctypes.data if n else None, nthreads)
    if rc != 0:
        raise ValueError(f"tkgen_host failed ({rc})")
    return out


def device_fill(kind: int, seed: int, n: int, dst_ptr: int, start: int = 0,
                n_total: int | None = None, cdf_dev_ptr: int | None = None, m: int = 0,
                stream: int = 0) -> None:
    """Fills a device buffer (raw pointer) on ``stream``."""
    if n_total is None:
        n_total = start + n
    rc = lib().tkgen_device(kind, seed % (1 << 64), start, n, n_total, cdf_dev_ptr, m, dst_ptr,
                            stream)
    if rc != 0:
        raise RuntimeError(f"tkgen_device failed ({rc})")
