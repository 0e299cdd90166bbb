"""Python binding of libpald (ctypes over the C ABI in include/pald.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libpald.so.  PyTorch supplies device memory (tensors) and the
stream (`torch.cuda.current_stream()`); nothing here computes PaLD.

If libpald.so is missing or cannot be loaded, every call raises -- there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpald.so")

OK, ERR_ARG, ERR_INPUT, ERR_DEVICE, ERR_NOMEM, ERR_UNSUPPORTED = range(6)
VARIANTS = {"auto": 0, "pairwise": 1, "triplet": 2, "hybrid": 3, "hybrid2": 4}
ACCUMS = {"compensated": 0, "f64": 1}
FLAG_TIMING = 1
TIMING_KINDS = ("pass1_focus", "weights", "pass2_cohesion", "finalize", "batched",
                "triplet_pass1", "triplet_pass2", "triplet_finalize", "distances", "local_depths",
                "strong_ties_count", "strong_ties_fill", "graph_distances", "rows_pass1", "rows_pass2",
                "ooc_copies")
DTYPES = {"float32": 0, "float64": 1}
METRICS = {"euclidean": 0, "sqeuclidean": 1}
INPUT_FLAGS = {1: "nan", 2: "inf", 4: "negative", 8: "asymmetric", 16: "nonzero_diagonal"}

#: every symbol include/pald.h declares
EXPORTED = (
    "pald_status_string", "pald_version", "pald_workspace_bytes", "pald_focus_sizes",
    "pald_cohesion", "pald_check_input", "pald_batch_plan_create", "pald_batch_workspace_bytes",
    "pald_batch_total_elements", "pald_batch_offset", "pald_batch_grid", "pald_cohesion_batched",
    "pald_batch_timestamps", "pald_batch_queue", "pald_batch_plan_destroy",
    "pald_batch_graph_create", "pald_batch_graph_launch", "pald_batch_graph_destroy",
    "pald_timings_collect", "pald_distances", "pald_local_depths", "pald_strong_ties",
    "pald_graph_distances_workspace_bytes", "pald_graph_distances", "pald_cohesion_noalloc",
    "pald_rows_workspace_bytes", "pald_cohesion_rows", "pald_ooc_workspace_bytes", "pald_cohesion_ooc",
    "pald_resolved_variant",
)
BATCH_MAX_BUCKETS = 8
BATCH_TIMESTAMPS = 1
BATCH_SPLIT_PASS1 = 2
BATCH_ONE_LAUNCH = 4


class PaldError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


class Options(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("accum", ctypes.c_int32),
        ("y_chunks", ctypes.c_int32),
        ("z_chunks", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class BatchBucket(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("y_chunks", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("nbuckets", ctypes.c_int32), ("workgroups_per_cu", ctypes.c_int32),
                ("queue_lag", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("bucket", BatchBucket * BATCH_MAX_BUCKETS)]


def make_batch_config(buckets=None, workgroups_per_cu: int = 0, queue_lag: int = 0,
                      timestamps: bool = False, split_pass1: bool | None = False) -> BatchConfig:
    """buckets: list of (n_max, y_chunks) or (n_max, y_chunks, tile) tuples, or dicts with keys
    n_max / y_chunks / tile (tile = pass-2 tile side, 64 or 32; default 64); empty = the
    library's built-in tuned buckets.  split_pass1: True = pass 1 of every matrix as a launch
    of its own before the persistent kernel, False = the one-launch form, None = the
    library's built-in tuned choice."""
    c = BatchConfig()
    buckets = list(buckets or [])
    if len(buckets) > BATCH_MAX_BUCKETS:
        raise ValueError(f"at most {BATCH_MAX_BUCKETS} buckets")
    for i, b in enumerate(buckets):
        if isinstance(b, dict):
            c.bucket[i].n_max = int(b["n_max"])
            c.bucket[i].tile = int(b.get("tile", 0))
            c.bucket[i].y_chunks = int(b.get("y_chunks", 1))
        else:
            c.bucket[i].n_max, c.bucket[i].y_chunks = int(b[0]), int(b[1])
            if len(b) > 2:
                c.bucket[i].tile = int(b[2])
    c.nbuckets = len(buckets)
    c.workgroups_per_cu = int(workgroups_per_cu)
    c.queue_lag = int(queue_lag)
    form = 0 if split_pass1 is None else (BATCH_SPLIT_PASS1 if split_pass1 else BATCH_ONE_LAUNCH)
    c.flags = (BATCH_TIMESTAMPS if timestamps else 0) | form
    return c


#: batched-mode settings written by paper_2307_16652_amd.tune for this GPU
TUNING_PATH = os.path.join(PKG, "tuning", "batch_gfx950.json")


#: per-size variant choice written by paper_2307_16652_amd.tune --variants; build.py
#: compiles it into the library, whose PALD_VARIANT_AUTO follows it
VARIANT_TUNING_PATH = os.path.join(PKG, "tuning", "variants_gfx950.json")


def load_tuning(path: str | None = None, timestamps: bool = False) -> BatchConfig | None:
    """The autotuned batched configuration, or None (library defaults) if none was written."""
    import json

    p = path or TUNING_PATH
    if not os.path.exists(p):
        return make_batch_config(timestamps=True) if timestamps else None
    with open(p) as f:
        data = json.load(f)
    return make_batch_config(data.get("buckets"), data.get("workgroups_per_cu", 0), data.get("queue_lag", 0),
                             timestamps, bool(data.get("split_pass1", False)))


_lib = None


def load_library(path: str | None = None):
    """Load libpald.so (built by paper_2307_16652_amd.build); raises if it is absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2307_16652_amd.build`")
    lib = ctypes.CDLL(p)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    opt = ctypes.POINTER(Options)
    lib.pald_status_string.argtypes = [i32]
    lib.pald_status_string.restype = ctypes.c_char_p
    lib.pald_version.argtypes = []
    lib.pald_version.restype = i32
    lib.pald_workspace_bytes.argtypes = [i64, opt]
    lib.pald_workspace_bytes.restype = sz
    lib.pald_resolved_variant.argtypes = [i64, opt]
    lib.pald_resolved_variant.restype = i32
    lib.pald_focus_sizes.argtypes = [vp, i64, i64, vp, i64, vp, opt]
    lib.pald_focus_sizes.restype = i32
    lib.pald_cohesion.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp, sz, vp, opt]
    lib.pald_cohesion.restype = i32
    lib.pald_cohesion_noalloc.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp, opt]
    lib.pald_cohesion_noalloc.restype = i32
    lib.pald_rows_workspace_bytes.argtypes = [i64, i64, opt]
    lib.pald_rows_workspace_bytes.restype = sz
    lib.pald_cohesion_rows.argtypes = [vp, i64, i64, i64, i64, vp, i64, vp, i64, vp, sz, vp, opt]
    lib.pald_cohesion_rows.restype = i32
    lib.pald_ooc_workspace_bytes.argtypes = [i64, i64]
    lib.pald_ooc_workspace_bytes.restype = sz
    lib.pald_cohesion_ooc.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp, sz, vp, opt]
    lib.pald_cohesion_ooc.restype = i32
    lib.pald_check_input.argtypes = [vp, i64, i64, vp, sz, vp, ctypes.POINTER(ctypes.c_uint32)]
    lib.pald_check_input.restype = i32
    cfgp = ctypes.POINTER(BatchConfig)
    lib.pald_batch_plan_create.argtypes = [i32, ctypes.POINTER(i64), cfgp, ctypes.POINTER(vp)]
    lib.pald_batch_plan_create.restype = i32
    lib.pald_batch_workspace_bytes.argtypes = [vp]
    lib.pald_batch_workspace_bytes.restype = sz
    lib.pald_batch_total_elements.argtypes = [vp]
    lib.pald_batch_total_elements.restype = i64
    lib.pald_batch_offset.argtypes = [vp, i32]
    lib.pald_batch_offset.restype = i64
    lib.pald_batch_grid.argtypes = [vp]
    lib.pald_batch_grid.restype = i32
    lib.pald_cohesion_batched.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.pald_cohesion_batched.restype = i32
    lib.pald_batch_timestamps.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]
    lib.pald_batch_timestamps.restype = i32
    lib.pald_batch_queue.argtypes = [i32, ctypes.POINTER(i64), cfgp, i32, ctypes.POINTER(i32), i64,
                                     ctypes.POINTER(i32)]
    lib.pald_batch_queue.restype = i64
    lib.pald_batch_plan_destroy.argtypes = [vp]
    lib.pald_batch_plan_destroy.restype = None
    lib.pald_batch_graph_create.argtypes = [vp, vp, vp, vp, vp, sz, ctypes.POINTER(vp)]
    lib.pald_batch_graph_create.restype = i32
    lib.pald_batch_graph_launch.argtypes = [vp, vp]
    lib.pald_batch_graph_launch.restype = i32
    lib.pald_batch_graph_destroy.argtypes = [vp]
    lib.pald_batch_graph_destroy.restype = None
    lib.pald_timings_collect.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32]
    lib.pald_timings_collect.restype = i32
    u32 = ctypes.c_uint32
    lib.pald_distances.argtypes = [vp, i32, i64, i64, i64, i32, vp, i64, vp, u32]
    lib.pald_distances.restype = i32
    lib.pald_local_depths.argtypes = [vp, i64, i64, vp, vp, u32]
    lib.pald_local_depths.restype = i32
    lib.pald_strong_ties.argtypes = [vp, i64, i64, ctypes.c_float, vp, vp, vp, i64, vp, u32]
    lib.pald_strong_ties.restype = i32
    lib.pald_graph_distances_workspace_bytes.argtypes = [i64]
    lib.pald_graph_distances_workspace_bytes.restype = sz
    lib.pald_graph_distances.argtypes = [vp, vp, i64, i64, vp, i64, vp, sz, vp, u32]
    lib.pald_graph_distances.restype = i32
    if path is None:
        _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load_library().pald_status_string(int(status)).decode()
    except Exception:  # pragma: no cover - library missing
        return f"status {status}"


def _check(status: int, where: str):
    if status != OK:
        raise PaldError(status, where)


def make_options(variant: str = "auto", accum: str = "compensated", y_chunks: int = 0,
                 z_chunks: int = 0, timing: bool = False) -> Options:
    o = Options()
    o.variant = VARIANTS[variant]
    o.accum = ACCUMS[accum]
    o.y_chunks = int(y_chunks)
    o.z_chunks = int(z_chunks)
    o.flags = FLAG_TIMING if timing else 0
    return o


# ----------------------------------------------------------------------------
# torch-facing helpers (torch is imported lazily: only memory and streams)


def _torch():
    import torch

    return torch


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_matrix(D):
    torch = _torch()
    if not isinstance(D, torch.Tensor) or not D.is_cuda:
        raise TypeError("D must be a torch tensor on a HIP (cuda) device")
    if D.dtype != torch.float32 or D.dim() != 2 or D.shape[0] != D.shape[1]:
        raise ValueError("D must be a square float32 matrix")
    if D.stride(1) != 1 or D.stride(0) < D.shape[0]:
        raise ValueError("D must be row-major with unit column stride")
    return D.shape[0], D.stride(0)


def workspace_bytes(n: int, **opts) -> int:
    o = make_options(**opts)
    return int(load_library().pald_workspace_bytes(int(n), ctypes.byref(o)))


def resolved_variant(n: int, **opts) -> str:
    """The variant pald_cohesion runs for size n with these options ("auto" resolved)."""
    v = int(load_library().pald_resolved_variant(int(n), ctypes.byref(make_options(**opts))))
    names = {i: k for k, i in VARIANTS.items()}
    if v not in names or v == 0:
        raise PaldError(ERR_UNSUPPORTED, "pald_resolved_variant")
    return names[v]


def workspace(n: int, device, **opts):
    torch = _torch()
    nbytes = workspace_bytes(n, **opts)
    if nbytes == 0:
        raise PaldError(ERR_ARG, "pald_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def focus_sizes(D, *, variant: str = "auto", z_chunks: int = 0, timing: bool = False, out=None):
    """U (int32, n x n): local focus sizes of distance matrix D."""
    torch = _torch()
    n, ldd = _check_matrix(D)
    U = out if out is not None else torch.empty((n, n), dtype=torch.int32, device=D.device)
    o = make_options(variant=variant, z_chunks=z_chunks, timing=timing)
    st = load_library().pald_focus_sizes(D.data_ptr(), n, ldd, U.data_ptr(), U.stride(0),
                                         _stream_ptr(D.device), ctypes.byref(o))
    _check(st, "pald_focus_sizes")
    return U


def cohesion(D, *, variant: str = "auto", accum: str = "compensated", y_chunks: int = 0,
             z_chunks: int = 0, want_u: bool = True, timing: bool = False, ws=None,
             out_u=None, out_c=None):
    """(U, C): focus sizes (int32, or None if want_u is False) and cohesion (float32)."""
    torch = _torch()
    n, ldd = _check_matrix(D)
    opts = dict(variant=variant, accum=accum, y_chunks=y_chunks, z_chunks=z_chunks, timing=timing)
    o = make_options(**opts)
    if ws is None:
        ws = workspace(n, D.device, **opts)
    U = None
    if want_u:
        U = out_u if out_u is not None else torch.empty((n, n), dtype=torch.int32, device=D.device)
    C = out_c if out_c is not None else torch.empty((n, n), dtype=torch.float32, device=D.device)
    st = load_library().pald_cohesion(
        D.data_ptr(), n, ldd,
        U.data_ptr() if U is not None else None, U.stride(0) if U is not None else 0,
        C.data_ptr(), C.stride(0), ws.data_ptr(), ws.numel(),
        _stream_ptr(D.device), ctypes.byref(o))
    _check(st, "pald_cohesion")
    return U, C


#: bytes of the library's fixed per-GPU workspace used by cohesion_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20


def cohesion_noalloc(D, *, accum: str = "compensated", y_chunks: int = 0, z_chunks: int = 0,
                     timing: bool = False, out_u=None, out_c=None):
    """(U, C) like cohesion(), through pald_cohesion_noalloc: no workspace is allocated
    (the library's fixed per-GPU array serves as one).  out_u / out_c given: nothing
    is allocated here either.  Pairwise variant only; calls on one GPU must not overlap."""
    torch = _torch()
    n, ldd = _check_matrix(D)
    o = make_options(variant="pairwise", accum=accum, y_chunks=y_chunks, z_chunks=z_chunks,
                     timing=timing)
    U = out_u
    C = out_c if out_c is not None else torch.empty((n, n), dtype=torch.float32, device=D.device)
    st = load_library().pald_cohesion_noalloc(
        D.data_ptr(), n, ldd,
        U.data_ptr() if U is not None else None, U.stride(0) if U is not None else 0,
        C.data_ptr(), C.stride(0), _stream_ptr(D.device), ctypes.byref(o))
    _check(st, "pald_cohesion_noalloc")
    return U, C


def rows_workspace_bytes(n: int, rows: int) -> int:
    return int(load_library().pald_rows_workspace_bytes(int(n), int(rows), None))


def cohesion_rows(D, x0: int, x1: int, *, want_u: bool = True, timing: bool = False, ws=None,
                  out_u=None, out_c=None):
    """(U rows, C rows) for rows x0 <= x < x1 of D's focus sizes and cohesion: int32 and
    float32 (x1 - x0) x n tensors (U None if want_u is False)."""
    torch = _torch()
    n, ldd = _check_matrix(D)
    rows = int(x1) - int(x0)
    if ws is None:
        nbytes = rows_workspace_bytes(n, rows)
        if nbytes == 0:
            raise PaldError(ERR_ARG, "pald_rows_workspace_bytes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=D.device)
    U = None
    if want_u:
        U = out_u if out_u is not None else torch.empty((rows, n), dtype=torch.int32, device=D.device)
    C = out_c if out_c is not None else torch.empty((rows, n), dtype=torch.float32, device=D.device)
    o = make_options(timing=timing)
    st = load_library().pald_cohesion_rows(
        D.data_ptr(), n, ldd, int(x0), int(x1),
        U.data_ptr() if U is not None else None, U.stride(0) if U is not None else 0,
        C.data_ptr(), C.stride(0), ws.data_ptr(), ws.numel(), _stream_ptr(D.device), ctypes.byref(o))
    _check(st, "pald_cohesion_rows")
    return U, C


def ooc_workspace_bytes(n: int, panel_rows: int) -> int:
    return int(load_library().pald_ooc_workspace_bytes(int(n), int(panel_rows)))


def cohesion_ooc(D_host, ws_bytes: int, *, device="cuda:0", want_u: bool = True, timing: bool = False):
    """(U, C) as host numpy arrays for a float32 distance matrix held in host memory
    (numpy array or CPU torch tensor, C-contiguous), computed out of core in panels of
    rows sized to a device workspace of ws_bytes (which this call allocates)."""
    import numpy as np

    torch = _torch()
    if isinstance(D_host, torch.Tensor):
        if D_host.is_cuda:
            raise TypeError("D_host must be in host memory")
        D_host = D_host.numpy()
    D_host = np.ascontiguousarray(D_host, dtype=np.float32)
    n = D_host.shape[0]
    if D_host.shape != (n, n):
        raise ValueError("D_host must be square")
    U = np.empty((n, n), dtype=np.int32) if want_u else None
    C = np.empty((n, n), dtype=np.float32)
    ws = torch.empty(int(ws_bytes), dtype=torch.uint8, device=device)
    o = make_options(timing=timing)
    st = load_library().pald_cohesion_ooc(
        D_host.ctypes.data, n, n, U.ctypes.data if U is not None else None, n, C.ctypes.data, n,
        ws.data_ptr(), ws.numel(), _stream_ptr(ws.device), ctypes.byref(o))
    _check(st, "pald_cohesion_ooc")
    return U, C


def check_input(D) -> list[str]:
    """Names of the input-contract violations found in D (empty list if valid)."""
    torch = _torch()
    n, ldd = _check_matrix(D)
    ws = torch.empty(256, dtype=torch.uint8, device=D.device)
    flags = ctypes.c_uint32(0)
    st = load_library().pald_check_input(D.data_ptr(), n, ldd, ws.data_ptr(), ws.numel(),
                                         _stream_ptr(D.device), ctypes.byref(flags))
    if st not in (OK, ERR_INPUT):
        _check(st, "pald_check_input")
    return [name for bit, name in INPUT_FLAGS.items() if flags.value & bit]


def distances(P, metric: str = "euclidean", *, timing: bool = False, out=None):
    """D (float32, n x n) from points P [n, dim] (float32 or float64 torch tensor on the GPU)."""
    torch = _torch()
    if not isinstance(P, torch.Tensor) or not P.is_cuda or P.dim() != 2:
        raise TypeError("P must be a 2-D torch tensor on a HIP (cuda) device")
    if P.dtype not in (torch.float32, torch.float64):
        raise ValueError("P must be float32 or float64")
    if P.stride(1) != 1:
        raise ValueError("P must be row-major with unit column stride")
    n, dim = P.shape
    D = out if out is not None else torch.empty((n, n), dtype=torch.float32, device=P.device)
    st = load_library().pald_distances(
        P.data_ptr(), DTYPES["float64" if P.dtype == torch.float64 else "float32"], n, dim,
        max(P.stride(0), dim), METRICS[metric], D.data_ptr(), D.stride(0), _stream_ptr(P.device),
        FLAG_TIMING if timing else 0)
    _check(st, "pald_distances")
    return D


def graph_distances(row_ptr, col, n: int, *, timing: bool = False, out=None, ws=None):
    """Hop-distance matrix D (float32, n x n; unreachable pairs = n) of the
    undirected graph with CSR arrays row_ptr (int64 [n+1]) and col (int32),
    torch tensors on the GPU."""
    torch = _torch()
    for a, dt, name in ((row_ptr, torch.int64, "row_ptr"), (col, torch.int32, "col")):
        if not isinstance(a, torch.Tensor) or not a.is_cuda or a.dtype != dt or a.dim() != 1 or \
                not a.is_contiguous():
            raise TypeError(f"{name} must be a contiguous 1-D {dt} tensor on a HIP (cuda) device")
    if row_ptr.numel() != n + 1:
        raise ValueError("row_ptr must have n + 1 entries")
    lib = load_library()
    D = out if out is not None else torch.empty((n, n), dtype=torch.float32, device=row_ptr.device)
    if ws is None:
        ws = torch.empty(int(lib.pald_graph_distances_workspace_bytes(n)), dtype=torch.uint8,
                         device=row_ptr.device)
    st = lib.pald_graph_distances(row_ptr.data_ptr(), col.data_ptr() if col.numel() else None, col.numel(), n,
                                  D.data_ptr(), D.stride(0), ws.data_ptr(), ws.numel(), _stream_ptr(row_ptr.device),
                                  FLAG_TIMING if timing else 0)
    _check(st, "pald_graph_distances")
    return D


def local_depths(C, *, timing: bool = False, out=None):
    """Local depths l_x = sum_z C[x][z] (float32 [n]) of a cohesion matrix on the GPU."""
    torch = _torch()
    n, ldc = _check_matrix(C)
    depth = out if out is not None else torch.empty(n, dtype=torch.float32, device=C.device)
    st = load_library().pald_local_depths(C.data_ptr(), n, ldc, depth.data_ptr(), _stream_ptr(C.device),
                                          FLAG_TIMING if timing else 0)
    _check(st, "pald_local_depths")
    return depth


def strong_ties(C, threshold: float, *, with_values: bool = True, timing: bool = False):
    """CSR (row_ptr int64 [n+1], col int32 [nnz], val float32 [nnz] or None) of the
    entries C[x][z] > threshold, z != x.  Two library calls: count, then fill."""
    torch = _torch()
    n, ldc = _check_matrix(C)
    lib = load_library()
    flags = FLAG_TIMING if timing else 0
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=C.device)
    st = lib.pald_strong_ties(C.data_ptr(), n, ldc, float(threshold), row_ptr.data_ptr(), None, None, 0,
                              _stream_ptr(C.device), flags)
    _check(st, "pald_strong_ties")
    nnz = int(row_ptr[n].item())
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=C.device)
    val = torch.empty(max(nnz, 1), dtype=torch.float32, device=C.device) if with_values else None
    st = lib.pald_strong_ties(C.data_ptr(), n, ldc, float(threshold), row_ptr.data_ptr(), col.data_ptr(),
                              val.data_ptr() if val is not None else None, nnz, _stream_ptr(C.device), flags)
    _check(st, "pald_strong_ties")
    return row_ptr, col[:nnz], (val[:nnz] if val is not None else None)


def timings_collect() -> dict:
    """{kernel kind: (total ms, launches)} recorded by calls made with timing=True."""
    k = len(TIMING_KINDS)
    tot = (ctypes.c_double * k)()
    cnt = (ctypes.c_int64 * k)()
    load_library().pald_timings_collect(tot, cnt, k)
    return {name: (tot[i], cnt[i]) for i, name in enumerate(TIMING_KINDS) if cnt[i]}


# ----------------------------------------------------------------------------
# batched mode


def batch_queue(sizes: Sequence[int], grid: int, config: BatchConfig | None = None):
    """Host-only: the queue a batched plan would run, as (items [k, 4] int32, tiles1 [count])."""
    import numpy as np

    lib = load_library()
    arr = (ctypes.c_int64 * len(sizes))(*[int(x) for x in sizes])
    cfg = ctypes.byref(config) if config is not None else None
    total = lib.pald_batch_queue(len(sizes), arr, cfg, int(grid), None, 0, None)
    if total < 0:
        raise PaldError(ERR_ARG, "pald_batch_queue")
    items = np.empty((total, 4), dtype=np.int32)
    tiles1 = np.empty(len(sizes), dtype=np.int32)
    lib.pald_batch_queue(len(sizes), arr, cfg, int(grid),
                         items.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), total,
                         tiles1.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return items, tiles1


class BatchPlan:
    """Plan for one packed batch of matrices of sizes `sizes` (see pald.h)."""

    def __init__(self, sizes: Sequence[int], config: BatchConfig | None = None):
        lib = load_library()
        self.sizes = [int(s) for s in sizes]
        arr = (ctypes.c_int64 * len(self.sizes))(*self.sizes)
        self.config = config
        h = ctypes.c_void_p()
        st = lib.pald_batch_plan_create(len(self.sizes), arr,
                                        ctypes.byref(config) if config is not None else None,
                                        ctypes.byref(h))
        _check(st, "pald_batch_plan_create")
        self._h = h
        self._lib = lib
        self.total = int(lib.pald_batch_total_elements(h))
        self.offsets = [int(lib.pald_batch_offset(h, i)) for i in range(len(self.sizes))]
        self.ws_bytes = int(lib.pald_batch_workspace_bytes(h))
        self.grid = int(lib.pald_batch_grid(h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pald_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, device):
        torch = _torch()
        return torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)

    def _outputs(self, D_packed, U_packed, C_packed, ws, want_u):
        torch = _torch()
        if D_packed.dtype != torch.float32 or D_packed.numel() != self.total or not D_packed.is_cuda:
            raise ValueError("D_packed must be a flat float32 cuda tensor of sum(n_i^2) elements")
        dev = D_packed.device
        if want_u and U_packed is None:
            U_packed = torch.empty(self.total, dtype=torch.int32, device=dev)
        if C_packed is None:
            C_packed = torch.empty(self.total, dtype=torch.float32, device=dev)
        if ws is None:
            ws = self.workspace(dev)
        return U_packed, C_packed, ws

    def run(self, D_packed, U_packed=None, C_packed=None, ws=None, want_u: bool = True):
        U_packed, C_packed, ws = self._outputs(D_packed, U_packed, C_packed, ws, want_u)
        st = self._lib.pald_cohesion_batched(
            self._h, D_packed.data_ptr(), U_packed.data_ptr() if U_packed is not None else None,
            C_packed.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(D_packed.device))
        _check(st, "pald_cohesion_batched")
        return U_packed, C_packed

    def graph(self, D_packed, U_packed=None, C_packed=None, ws=None, want_u: bool = True):
        """A captured hipGraph of one run with these buffers (see BatchGraph)."""
        U_packed, C_packed, ws = self._outputs(D_packed, U_packed, C_packed, ws, want_u)
        return BatchGraph(self, D_packed, U_packed, C_packed, ws)

    def timestamps(self, ws):
        """Per-matrix (start_us, end_us) of the last run, if the plan records them."""
        import numpy as np

        k = len(self.sizes)
        a = (ctypes.c_double * k)()
        b = (ctypes.c_double * k)()
        st = self._lib.pald_batch_timestamps(self._h, ws.data_ptr(), _stream_ptr(ws.device), a, b)
        _check(st, "pald_batch_timestamps")
        return np.frombuffer(a, dtype=np.float64).copy(), np.frombuffer(b, dtype=np.float64).copy()

    def pack(self, mats):
        torch = _torch()
        return torch.cat([m.reshape(-1) for m in mats])

    def unpack(self, flat):
        return [flat[o:o + s * s].view(s, s) for o, s in zip(self.offsets, self.sizes)]


class BatchGraph:
    """One batched run captured as a hipGraph; keeps its buffers alive."""

    def __init__(self, plan: BatchPlan, D_packed, U_packed, C_packed, ws):
        self.plan, self.D, self.U, self.C, self.ws = plan, D_packed, U_packed, C_packed, ws
        h = ctypes.c_void_p()
        st = plan._lib.pald_batch_graph_create(
            plan._h, D_packed.data_ptr(), U_packed.data_ptr() if U_packed is not None else None,
            C_packed.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.byref(h))
        _check(st, "pald_batch_graph_create")
        self._h = h

    def launch(self):
        st = self.plan._lib.pald_batch_graph_launch(self._h, _stream_ptr(self.D.device))
        _check(st, "pald_batch_graph_launch")
        return self.U, self.C

    def close(self):
        if getattr(self, "_h", None):
            self.plan._lib.pald_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def cohesion_batched(mats, config: BatchConfig | None | str = "tuned"):
    """[(U_i, C_i)] for a list of square float32 cuda matrices, in one batched run.

    config: a BatchConfig, None for the library's built-in configuration (the
    autotuned table compiled into it), or "tuned" (default) for the autotuner's
    record tuning/batch_gfx950.json read at run time (the same table unless the
    record changed after the build)."""
    if isinstance(config, str):
        if config != "tuned":
            raise ValueError('config must be a BatchConfig, None or "tuned"')
        config = load_tuning()
    plan = BatchPlan([m.shape[0] for m in mats], config=config)
    try:
        Dp = plan.pack(mats)
        Up, Cp = plan.run(Dp)
        return list(zip(plan.unpack(Up), plan.unpack(Cp)))
    finally:
        plan.close()
