"""Seeded synthetic inputs: point clouds -> exactly symmetric FP32 distance matrices.

This module holds no part of the PaLD computation itself.  It produces the
distance matrices that both the GPU library and the CPU oracle consume, so the
two see byte-identical inputs.

Every matrix is built the same way:

* points are drawn with numpy's PCG64 generator from a fixed seed;
* each distance is computed from coordinate differences in float64 and rounded
  once to float32 (Euclidean, or squared Euclidean for integer grids);
* only the upper triangle is computed; it is mirrored to the lower triangle, so
  D is exactly symmetric, and the diagonal is exactly zero.

The paper measures on "randomly generated distance matrices" of unstated
distribution (Section 5) plus text-embedding and SNAP shortest-path data that
are not available here; the workloads below stand in for them.

Workloads (name: points, distance):

* ``uniform2d``  -- n points uniform in [0,1]^2, Euclidean (default n = 256, seed 1)
* ``mixture8d``  -- 6 Gaussian clusters in R^8 with sizes in ratio 1:2:4:8:16:32
                    and standard deviations 0.05 ... 1.0 (default n = 4096, seed 2)
* ``grid3d``     -- coordinates uniform in {0..31}^3 with replacement, squared
                    Euclidean integer distances (many ties and duplicate points;
                    default n = 16384, seed 3)
* ``batch``      -- many independent 2-5 cluster mixtures in R^4 with
                    n_i uniform in [32, 1024] (default 2000 matrices, seed 4)
* ``aniso16d``   -- 50 anisotropic rotated Gaussians in R^16 (default n = 65536,
                    seed 5)
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "pairwise_distances",
    "uniform2d_points",
    "mixture8d_points",
    "grid3d_points",
    "aniso16d_points",
    "batch_sizes",
    "batch_points",
    "uniform2d",
    "mixture8d",
    "grid3d",
    "aniso16d",
    "batch",
    "workload",
    "random_tie_matrix",
    "WORKLOADS",
]


# ----------------------------------------------------------------------------
# distances


def pairwise_distances(P, squared: bool = False, block: int = 256) -> np.ndarray:
    """FP32 distance matrix of the rows of P (computed in float64, rounded once).

    Only pairs (i, j) with j >= i are evaluated; the lower triangle is the
    mirror image, so the result is exactly symmetric with a zero diagonal.
    """
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64))
    if P.ndim != 2:
        raise ValueError("P must be [n, dim]")
    n, dim = P.shape
    D = np.empty((n, n), dtype=np.float32)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        acc = np.zeros((r1 - r0, n - r0), dtype=np.float64)
        for k in range(dim):
            diff = P[r0:r1, k, None] - P[None, r0:, k]
            acc += diff * diff
        if not squared:
            np.sqrt(acc, out=acc)
        blk = acc.astype(np.float32)
        w = r1 - r0
        sq = np.triu(blk[:, :w], 1)
        blk[:, :w] = sq + sq.T
        D[r0:r1, r0:] = blk
        D[r0:, r0:r1] = blk.T
    np.fill_diagonal(D, 0.0)
    return D


def pairwise_distances_torch(P, squared: bool = False, device="cuda", block: int = 2048):
    """Same construction as :func:`pairwise_distances`, evaluated with torch.

    Used for the very large matrices (tens of GB) that would take minutes on
    the host.  Returns a float32 torch tensor on `device`.
    """
    import torch

    Pt = torch.as_tensor(np.asarray(P, dtype=np.float64), device=device)
    n, dim = Pt.shape
    D = torch.empty((n, n), dtype=torch.float32, device=device)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        acc = torch.zeros((r1 - r0, n - r0), dtype=torch.float64, device=device)
        for k in range(dim):
            diff = Pt[r0:r1, k, None] - Pt[None, r0:, k]
            acc += diff * diff
        if not squared:
            acc.sqrt_()
        blk = acc.to(torch.float32)
        del acc
        w = r1 - r0
        sq = torch.triu(blk[:, :w], 1)
        blk[:, :w] = sq + sq.T
        D[r0:r1, r0:] = blk
        D[r0:, r0:r1] = blk.T
        del blk, sq
    D.fill_diagonal_(0.0)
    return D


# ----------------------------------------------------------------------------
# point clouds


def uniform2d_points(n: int = 256, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((n, 2))


def _geometric_sizes(n: int, k: int) -> list[int]:
    """Cluster sizes in ratio 1:2:4:...:2^(k-1); the remainder goes to the largest."""
    total = 2**k - 1
    sizes = [(n * 2**i) // total for i in range(k)]
    sizes[-1] += n - sum(sizes)
    return sizes


def mixture8d_points(n: int = 4096, seed: int = 2) -> np.ndarray:
    """6 Gaussian clusters in R^8: sizes 1:2:4:8:16:32, std 0.05 * 20^(k/5)."""
    rng = np.random.default_rng(seed)
    k = 6
    sizes = _geometric_sizes(n, k)
    centres = rng.uniform(-5.0, 5.0, size=(k, 8))
    parts = []
    for i, m in enumerate(sizes):
        sigma = 0.05 * 20.0 ** (i / 5.0)
        parts.append(centres[i] + sigma * rng.standard_normal((m, 8)))
    P = np.concatenate(parts, axis=0)
    return P[rng.permutation(n)]


def grid3d_points(n: int = 16384, seed: int = 3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 32, size=(n, 3)).astype(np.float64)


def aniso16d_points(n: int = 65536, seed: int = 5, clusters: int = 50) -> np.ndarray:
    """50 anisotropic Gaussians in R^16 with log-uniform axis scales in [0.01, 1]."""
    rng = np.random.default_rng(seed)
    dim = 16
    sizes = rng.multinomial(n, np.full(clusters, 1.0 / clusters))
    parts = []
    for m in sizes:
        scales = np.exp(rng.uniform(np.log(0.01), np.log(1.0), size=dim))
        q, r = np.linalg.qr(rng.standard_normal((dim, dim)))
        q = q * np.sign(np.diag(r))
        centre = rng.uniform(-10.0, 10.0, size=dim)
        parts.append(centre + (rng.standard_normal((m, dim)) * scales) @ q.T)
    P = np.concatenate(parts, axis=0)
    return P[rng.permutation(n)]


def batch_sizes(count: int = 2000, seed: int = 4, lo: int = 32, hi: int = 1024) -> np.ndarray:
    """Matrix sizes n_i, uniform integers in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count).astype(np.int64)


def batch_points(i: int, n: int, seed: int = 4) -> np.ndarray:
    """Points of matrix i of the batch: a 2-5 cluster Gaussian mixture in R^4."""
    rng = np.random.default_rng([seed, i])
    k = int(rng.integers(2, 6))
    centres = rng.uniform(-5.0, 5.0, size=(k, 4))
    sigmas = np.exp(rng.uniform(np.log(0.05), np.log(1.0), size=k))
    sizes = rng.multinomial(n, np.full(k, 1.0 / k))
    parts = [centres[c] + sigmas[c] * rng.standard_normal((m, 4)) for c, m in enumerate(sizes)]
    P = np.concatenate(parts, axis=0)
    return P[rng.permutation(n)]


def collab_graph(n: int = 16384, papers: int | None = None, seed: int = 6):
    """A seeded stand-in for a collaboration network: `papers` (default 2n)
    papers each join 2-6 authors drawn with heavy-tailed activity weights
    (Pareto, shape 1.5), and every paper links its authors pairwise.  Returns
    the undirected simple graph as CSR (row_ptr int64 [n+1], col int32, both
    directions stored, neighbours sorted, no self-loops).  Authors on no paper
    are isolated vertices."""
    rng = np.random.default_rng(seed)
    papers = 2 * n if papers is None else int(papers)
    act = rng.pareto(1.5, size=n) + 1.0
    A = rng.choice(n, size=(papers, 6), p=act / act.sum())
    K = rng.integers(2, 7, size=papers)
    us, vs = [], []
    for j in range(6):
        for l in range(j + 1, 6):
            m = l < K
            us.append(A[m, j])
            vs.append(A[m, l])
    u = np.concatenate(us).astype(np.int64)
    v = np.concatenate(vs).astype(np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    key = np.unique(np.concatenate([u * n + v, v * n + u]))
    src, dst = key // n, key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    return np.cumsum(row_ptr), dst.astype(np.int32)


# ----------------------------------------------------------------------------
# distance matrices of the named workloads


def uniform2d(n: int = 256, seed: int = 1) -> np.ndarray:
    return pairwise_distances(uniform2d_points(n, seed))


def mixture8d(n: int = 4096, seed: int = 2) -> np.ndarray:
    return pairwise_distances(mixture8d_points(n, seed))


def grid3d(n: int = 16384, seed: int = 3) -> np.ndarray:
    return pairwise_distances(grid3d_points(n, seed), squared=True)


def aniso16d(n: int = 65536, seed: int = 5) -> np.ndarray:
    return pairwise_distances(aniso16d_points(n, seed))


def batch(count: int = 2000, seed: int = 4, lo: int = 32, hi: int = 1024) -> list[np.ndarray]:
    ns = batch_sizes(count, seed, lo, hi)
    return [pairwise_distances(batch_points(i, int(m), seed)) for i, m in enumerate(ns)]


WORKLOADS = {
    "uniform2d": uniform2d,
    "mixture8d": mixture8d,
    "grid3d": grid3d,
    "aniso16d": aniso16d,
}


def workload(name: str, n: int | None = None, seed: int | None = None) -> np.ndarray:
    fn = WORKLOADS[name]
    kw = {}
    if n is not None:
        kw["n"] = n
    if seed is not None:
        kw["seed"] = seed
    return fn(**kw)


def random_tie_matrix(n: int, values, seed: int) -> np.ndarray:
    """Symmetric zero-diagonal matrix whose off-diagonal entries are drawn from `values`.

    Not a metric in general (PaLD does not need the triangle inequality);
    used to saturate the tie cases.
    """
    rng = np.random.default_rng(seed)
    vals = np.asarray(values, dtype=np.float32)
    D = np.zeros((n, n), dtype=np.float32)
    iu = np.triu_indices(n, 1)
    D[iu] = rng.choice(vals, size=iu[0].size)
    D = D + D.T
    return D
