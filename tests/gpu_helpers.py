"""Shared helpers of the GPU parity tests: run libpald, compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np

#: relative tolerance on every cohesion entry (entries that are exactly 0 in the
#: oracle must be exactly 0)
C_RTOL = 1e-6


_ORACLE_CACHE = {}


def oracle_full_cached(name: str, D: np.ndarray):
    """Full oracle (U, C) of a named workload matrix, computed once per test session."""
    import oracle

    if name not in _ORACLE_CACHE:
        _ORACLE_CACHE[name] = oracle.pald(D)
    return _ORACLE_CACHE[name]


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def device():
    import torch

    return torch.device("cuda:0")


def to_gpu(D: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(D)).to(device())


def gpu_cohesion(D: np.ndarray, **opts):
    """(U int32 numpy, C float32 numpy) from libpald for a host matrix."""
    import torch

    from paper_2307_16652_amd import pald

    U, C = pald.cohesion(to_gpu(D), **opts)
    torch.cuda.synchronize()
    return (U.cpu().numpy() if U is not None else None), C.cpu().numpy()


def assert_c_close(C, Cref, rtol=C_RTOL, what=""):
    C = np.asarray(C, dtype=np.float64)
    Cref = np.asarray(Cref, dtype=np.float64)
    assert C.shape == Cref.shape, f"{what}: shape {C.shape} vs {Cref.shape}"
    zero = Cref == 0
    nz_bad = np.argwhere(zero & (C != 0))
    assert nz_bad.size == 0, f"{what}: {nz_bad.shape[0]} entries nonzero where the oracle is exactly 0, e.g. " \
                             f"{nz_bad[0].tolist()} = {C[tuple(nz_bad[0])]!r}"
    rel = np.zeros_like(C)
    rel[~zero] = np.abs(C[~zero] - Cref[~zero]) / np.abs(Cref[~zero])
    worst = np.unravel_index(np.argmax(rel), rel.shape)
    assert rel.max() <= rtol, f"{what}: max relative error {rel.max():.3e} at {list(worst)} " \
                              f"(got {C[worst]!r}, oracle {Cref[worst]!r})"
    return float(rel.max())


def assert_u_equal(U, Uref, what=""):
    U = np.asarray(U)
    Uref = np.asarray(Uref)
    assert U.shape == Uref.shape, f"{what}: U shape {U.shape} vs {Uref.shape}"
    bad = np.argwhere(U != Uref)
    assert bad.size == 0, f"{what}: {bad.shape[0]} U mismatches, first at {bad[0].tolist()}: " \
                          f"{U[tuple(bad[0])]} vs {Uref[tuple(bad[0])]}"


def check_invariants(U, C, what=""):
    """Properties that hold at any size: U symmetric in [2, n] off the diagonal,
    C >= 0, local depths in [0, 1], sum(C) = n/2."""
    n = U.shape[0]
    assert np.array_equal(U, U.T), f"{what}: U not symmetric"
    off = ~np.eye(n, dtype=bool)
    assert U[off].min() >= 2 and U[off].max() <= n, f"{what}: U off-diagonal outside [2, n]"
    assert (C >= 0).all(), f"{what}: negative cohesion"
    depth = C.astype(np.float64).sum(axis=1)
    assert depth.min() >= 0 and depth.max() <= 1 + 1e-5, f"{what}: local depth outside [0, 1]"
    total = float(C.astype(np.float64).sum())
    assert abs(total - n / 2) <= 1e-6 * n / 2, f"{what}: sum(C) = {total!r}, expected {n / 2}"
