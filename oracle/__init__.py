"""CPU FP64 oracle for partitioned local depths -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never calls it and shares no code
with it.

`pald_oracle.c` evaluates, for each requested row x,

* u_xy = #{z : d_xz <= d_xy or d_yz <= d_xy}       (local focus, Section 2)
* c_xz = 1/(n-1) sum_{y != x} s(d_xz, d_yz) [d_xz <= d_xy] / u_xy
                                                   (Section 3, Eq. (fxz))

with s(p, q) = [p < q] + 1/2 [p == q] (ties split, Section 5), in double
precision after promoting the FP32 distances exactly to double.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pald_oracle.c")
_LIB = os.path.join(_HERE, "libpald_oracle.so")

# Plain -O2: no -ffast-math / -Ofast, which would enable flush-to-zero and
# change the outcome of comparisons between denormal distances.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libpald_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        lib.pald_oracle_rows.argtypes = [vp, i64, i64, vp, i64, vp, vp, ctypes.c_int]
        lib.pald_oracle_rows.restype = ctypes.c_int
        lib.pald_oracle_full.argtypes = [vp, i64, i64, vp, vp, ctypes.c_int]
        lib.pald_oracle_full.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def _as_input(D) -> np.ndarray:
    D = np.ascontiguousarray(np.asarray(D, dtype=np.float32))
    if D.ndim != 2 or D.shape[0] != D.shape[1]:
        raise ValueError("D must be a square 2-D array")
    if D.shape[0] < 2:
        raise ValueError("PaLD needs at least two points")
    return D


def pald_rows(D, rows, threads: int | None = None):
    """Rows `rows` of (U, C): U int32 [len(rows), n], C float64 [len(rows), n]."""
    D = _as_input(D)
    n = D.shape[0]
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1))
    U = np.empty((rows.size, n), dtype=np.int32)
    C = np.empty((rows.size, n), dtype=np.float64)
    if rows.size == 0:
        return U, C
    t = default_threads() if threads is None else int(threads)
    rc = _load().pald_oracle_rows(D.ctypes.data, n, n, rows.ctypes.data, rows.size,
                                  U.ctypes.data, C.ctypes.data, t)
    if rc != 0:
        raise RuntimeError("pald_oracle_rows failed (bad arguments)")
    return U, C


def pald(D, threads: int | None = None):
    """Full (U, C) of a distance matrix: U int32 [n, n], C float64 [n, n]."""
    D = _as_input(D)
    n = D.shape[0]
    U = np.empty((n, n), dtype=np.int32)
    C = np.empty((n, n), dtype=np.float64)
    t = default_threads() if threads is None else int(threads)
    rc = _load().pald_oracle_full(D.ctypes.data, n, n, U.ctypes.data, C.ctypes.data, t)
    if rc != 0:
        raise RuntimeError("pald_oracle_full failed (bad arguments)")
    return U, C
