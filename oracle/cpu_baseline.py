"""Timed CPU baseline of the PageRank workload -- BENCHMARK INFRASTRUCTURE ONLY.

Only the benchmark's CPU-baseline leg calls this module (the product never
does; the parity tests use the oracle's checker functions).  It wraps
``cpu_baseline.c``: the power method of Sec. 5.5.1 on the same CSR as the
oracle's ``pagerank``, with plain double sums, on one thread or row-parallel
with OpenMP.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpu_baseline.c")
_LIB = os.path.join(_HERE, "libcpubaseline.so")
_lib = None


def build() -> str:
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-fopenmp", "-o", tmp,
                    _SRC], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i32 = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64 = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        lib.cb_pagerank.restype = ctypes.c_int
        lib.cb_pagerank.argtypes = [ctypes.c_int64, i32, i32, f64, ctypes.c_double, ctypes.c_int,
                                    f64, ctypes.c_int]
        _lib = lib
    return _lib


def pagerank(row_ptr, col, values, alpha: float, iters: int, x0, threads: int):
    """`iters` power-method steps from x0 with `threads` OpenMP threads
    (<= 0: OpenMP's default).  Returns (x, threads actually used)."""
    row_ptr = np.ascontiguousarray(row_ptr, np.int32)
    x = np.array(x0, np.float64, copy=True)
    used = _load().cb_pagerank(len(row_ptr) - 1, row_ptr, np.ascontiguousarray(col, np.int32),
                               np.ascontiguousarray(values, np.float64), float(alpha), int(iters),
                               x, int(threads))
    if used < 0:
        raise MemoryError("cb_pagerank failed")
    return x, used


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"
