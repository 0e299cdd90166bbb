"""Seeded input generators: exact symmetry, zero diagonal, workload shapes (CPU only)."""
import numpy as np
import pytest

from paper_2307_16652_amd import synth


@pytest.mark.parametrize("name,n", [("uniform2d", 256), ("mixture8d", 300), ("grid3d", 700), ("aniso16d", 257)])
def test_exactly_symmetric_zero_diagonal(name, n):
    D = synth.workload(name, n=n)
    assert D.dtype == np.float32 and D.shape == (n, n)
    assert np.array_equal(D, D.T)
    assert (np.diag(D) == 0).all()
    assert np.isfinite(D).all() and (D >= 0).all()


def test_deterministic():
    assert np.array_equal(synth.mixture8d(n=200), synth.mixture8d(n=200))
    assert not np.array_equal(synth.mixture8d(n=200, seed=2), synth.mixture8d(n=200, seed=9))


def test_grid3d_is_integer_with_ties_and_duplicates():
    D = synth.grid3d(n=2048)
    assert (D == np.round(D)).all() and D.max() <= 3 * 31**2
    off = ~np.eye(2048, dtype=bool)
    assert (D[off] == 0).sum() > 0  # duplicate points occur
    assert np.unique(D).size < 3 * 31**2 + 1  # heavy ties


def test_mixture_cluster_sizes():
    assert synth._geometric_sizes(4096, 6) == [65, 130, 260, 520, 1040, 2081]


def test_batch_sizes_range():
    ns = synth.batch_sizes(2000)
    assert ns.min() >= 32 and ns.max() <= 1024 and ns.size == 2000
    D = synth.pairwise_distances(synth.batch_points(3, int(ns[3])))
    assert D.shape == (ns[3], ns[3]) and np.array_equal(D, D.T)
