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

The steps around the two passes:

* `local_depths` -- l_x = sum_z c_xz (Section 2: cohesion partitions the
  local depth of Eq. (LD));
* `strong_ties` -- the directed graph of the entries of C above a threshold,
  in CSR form (Section 2 and Section 6 read community structure off the
  cohesion matrix by thresholding it);
* `distances` (`distance_oracle.c`) -- Euclidean or squared Euclidean
  distances between points, the input Section 6 feeds to PaLD;
* `graph_distances` (`distance_oracle.c`) -- all-pairs shortest-path hop
  counts of an unweighted graph, the input of the appendix's collaboration-
  network runs (unreachable pairs at distance n).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "pald_oracle.c"), os.path.join(_HERE, "distance_oracle.c")]
_LIB = os.path.join(_HERE, "libpald_oracle.so")

# Plain -O2: no -ffast-math / -Ofast, which would enable flush-to-zero and
# change the outcome of comparisons between denormal distances; no implicit
# contraction of a multiply and an add into one fused operation either.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra", "-ffp-contract=off"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libpald_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, *_SRCS, "-lm"])
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
        lib.pald_oracle_distances.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.c_int, vp, i64, vp, i64]
        lib.pald_oracle_distances.restype = ctypes.c_int
        lib.pald_oracle_graph_distances.argtypes = [vp, vp, i64, vp, i64, vp, i64]
        lib.pald_oracle_graph_distances.restype = ctypes.c_int
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


def local_depths(C) -> np.ndarray:
    """l_x = sum_z c_xz for every row x of C, in float64 (Section 2: cohesion
    is partitioned local depth)."""
    return np.asarray(C, dtype=np.float64).sum(axis=1)


def strong_ties(C, threshold):
    """The entries of a float32 cohesion matrix above `threshold`, as CSR.

    Row x lists, in increasing order, every z != x with C[x][z] > threshold,
    the comparison made in float32 (threshold rounded to float32 first).
    Returns (row_ptr int64 [n+1], col int32 [nnz], val float32 [nnz]).
    """
    C = np.asarray(C)
    if C.dtype != np.float32 or C.ndim != 2 or C.shape[0] != C.shape[1]:
        raise ValueError("C must be a square float32 matrix")
    t = np.float32(threshold)
    n = C.shape[0]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for x in range(n):
        z = np.nonzero(C[x] > t)[0]
        z = z[z != x]
        cols.append(z.astype(np.int32))
        vals.append(C[x, z])
        row_ptr[x + 1] = row_ptr[x] + z.size
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    val = np.concatenate(vals) if vals else np.zeros(0, np.float32)
    return row_ptr, col.astype(np.int32), val.astype(np.float32)


METRICS = {"euclidean": 0, "sqeuclidean": 1}


def distances(P, metric: str = "euclidean", rows=None) -> np.ndarray:
    """Distance matrix (or rows `rows` of it) of the points P [n, dim]
    (float32 or float64) as float32, by the definition in distance_oracle.c."""
    P = np.asarray(P)
    if P.dtype not in (np.float32, np.float64):
        P = P.astype(np.float64)
    P = np.ascontiguousarray(P)
    if P.ndim != 2:
        raise ValueError("P must be [n, dim]")
    n, dim = P.shape
    dtype = 1 if P.dtype == np.float64 else 0
    if rows is None:
        out = np.empty((n, n), dtype=np.float32)
        rp, nr = None, n
    else:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1))
        out = np.empty((rows.size, n), dtype=np.float32)
        rp, nr = rows.ctypes.data, rows.size
    rc = _load().pald_oracle_distances(P.ctypes.data, dtype, n, dim, dim, METRICS[metric], rp, nr,
                                       out.ctypes.data, n)
    if rc != 0:
        raise RuntimeError("pald_oracle_distances failed (bad arguments)")
    return out


def graph_distances(row_ptr, col, n: int, rows=None) -> np.ndarray:
    """Hop-distance matrix (or rows `rows`) of the unweighted graph in CSR form,
    float32, unreachable pairs = n, by one breadth-first search per row."""
    row_ptr = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    col = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
    if row_ptr.shape != (n + 1,) or row_ptr[0] != 0 or row_ptr[-1] > col.size or (np.diff(row_ptr) < 0).any():
        raise ValueError("row_ptr must be a CSR offset array of length n + 1")
    if rows is None:
        out = np.empty((n, n), dtype=np.float32)
        rp, nr = None, n
    else:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1))
        out = np.empty((rows.size, n), dtype=np.float32)
        rp, nr = rows.ctypes.data, rows.size
    rc = _load().pald_oracle_graph_distances(row_ptr.ctypes.data, col.ctypes.data if col.size else None, n,
                                             rp, nr, out.ctypes.data, n)
    if rc != 0:
        raise RuntimeError("pald_oracle_graph_distances failed (bad arguments)")
    return out
