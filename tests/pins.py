"""Checks that pin an FP64 PaLD oracle to facts fixed by the paper and by mathematics.

Each check takes `oracle(D) -> (U int[n,n], C float64[n,n])` and raises
AssertionError on a mismatch.  `test_oracle_pins.py` runs them against the real
oracle; `test_oracle_mutants.py` runs them against copies of the oracle with a
planted mistake and requires every mutant to fail at least one of them.

What pins what:

* golden worked examples (tests/golden/): normalisation, diagonal, ordering,
  the one-half tie split, focus sizes, duplicate points;
* exact rational brute force from the probability definition and the
  tie-exact triplet enumeration (tests/exact_pald.py) on random and
  exhaustive tie patterns;
* closed forms: the regular simplex and K equidistant separated clusters;
* invariants: U = U^T, 2 <= U_xy <= n, sum(C) = n/2, row sums in [0, 1],
  C >= 0, the C_xx identity, permutation equivariance, invariance under
  strictly increasing value maps, exact scaling into the denormal range.
"""
from __future__ import annotations

import glob
import os
from fractions import Fraction
from itertools import product

import numpy as np

import exact_pald

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RTOL = 1e-13  # an FP64 evaluation of n <= 64 terms lands far inside this


# ----------------------------------------------------------------------------
# helpers


def load_golden(path):
    """Parse a worked-example fixture: returns (D float32, U int, C Fraction)."""
    lines = [ln.strip() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    n = int(lines[0].split()[1])
    i = lines.index("D")
    D = np.array([[float(v) for v in lines[i + 1 + r].split()] for r in range(n)], dtype=np.float32)
    i = lines.index("U")
    U = np.array([[int(v) for v in lines[i + 1 + r].split()] for r in range(n)], dtype=np.int64)
    i = lines.index("C")
    C = [[Fraction(v) for v in lines[i + 1 + r].split()] for r in range(n)]
    return D, U, C


def golden_files():
    return sorted(glob.glob(os.path.join(GOLDEN, "example_*.txt")))


def close_to_exact(C, Cx, rtol=RTOL, what=""):
    """Every entry within rtol of the exact value; exact zeros must be exact."""
    n = len(Cx)
    for x in range(n):
        for z in range(n):
            ref = Cx[x][z]
            got = C[x][z]
            if ref == 0:
                assert got == 0.0, f"{what} C[{x},{z}] = {got!r}, expected exactly 0"
            else:
                refv = float(ref)
                assert abs(got - refv) <= rtol * abs(refv), (
                    f"{what} C[{x},{z}] = {got!r}, expected {ref} = {refv!r}")


def same_U(U, Ux, what=""):
    U = np.asarray(U, dtype=np.int64)
    Ux = np.asarray(Ux, dtype=np.int64)
    assert U.shape == Ux.shape, f"{what} U shape {U.shape} vs {Ux.shape}"
    bad = np.argwhere(U != Ux)
    assert bad.size == 0, f"{what} U differs at {bad[:5].tolist()}: {U[tuple(bad[0])]} vs {Ux[tuple(bad[0])]}"


def check_invariants(D, U, C, what=""):
    n = D.shape[0]
    U = np.asarray(U, dtype=np.int64)
    assert (U == U.T).all(), f"{what} U not symmetric"
    off = ~np.eye(n, dtype=bool)
    assert U[off].min() >= 2 and U[off].max() <= n, f"{what} U off-diagonal outside [2, n]"
    assert (C >= 0).all(), f"{what} negative cohesion"
    total = float(np.sum(C, dtype=np.float64))
    assert abs(total - n / 2) <= 1e-12 * n, f"{what} sum(C) = {total!r}, expected n/2 = {n / 2}"
    depth = C.sum(axis=1)
    assert (depth >= -1e-15).all() and (depth <= 1 + 1e-12).all(), f"{what} local depth outside [0, 1]"
    # diagonal identity when no two distinct points coincide
    if (D[off] > 0).all():
        Ud = np.where(off, U, 1).astype(np.float64)
        cxx = (np.where(off, 1.0 / Ud, 0.0)).sum(axis=1) / (n - 1)
        assert np.allclose(np.diag(C), cxx, rtol=1e-13, atol=0), f"{what} C_xx identity"


# ----------------------------------------------------------------------------
# pins


def pin_golden(oracle):
    files = golden_files()
    assert files, "no golden fixtures found"
    for f in files:
        D, Ux, Cx = load_golden(f)
        U, C = oracle(D)
        name = os.path.basename(f)
        same_U(U, Ux, name)
        close_to_exact(C, Cx, what=name)


def _random_small_cases():
    rng = np.random.default_rng(12345)
    cases = []
    for n in (2, 3, 4, 5, 6, 7, 8):
        cases.append(rng.random((n, 3)))  # continuous Euclidean
    mats = []
    for P in cases:
        diff = P[:, None, :] - P[None, :, :]
        D = np.sqrt((diff * diff).sum(-1)).astype(np.float32)
        D = np.triu(D, 1)
        mats.append(D + D.T)
    for n in (3, 4, 5, 6, 7, 8):
        for vals in ((1, 2), (1, 2, 3), (0, 1, 2), (0, 1, 1, 2, 3), (5,)):
            for s in range(2):
                v = rng.choice(np.asarray(vals, dtype=np.float32), size=(n, n))
                v = np.triu(v, 1)
                mats.append((v + v.T).astype(np.float32))
    return mats


def pin_bruteforce_random(oracle):
    """Exact-rational brute force from the probability definition, n <= 8."""
    for k, D in enumerate(_random_small_cases()):
        Ux, Cx = exact_pald.by_probability(D)
        U, C = oracle(D)
        same_U(U, Ux, f"case {k} (n={D.shape[0]})")
        close_to_exact(C, Cx, what=f"case {k} (n={D.shape[0]})")


def exhaustive_n4(values):
    """All symmetric zero-diagonal 4x4 matrices with entries from `values`."""
    iu = np.triu_indices(4, 1)
    for combo in product(values, repeat=6):
        D = np.zeros((4, 4), dtype=np.float32)
        D[iu] = combo
        yield D + D.T


def pin_exhaustive_ties(oracle, values=(1.0, 2.0)):
    """Every tie pattern of a 4-point matrix against the exact brute force."""
    for D in exhaustive_n4(values):
        Ux, Cx = exact_pald.by_probability(D)
        U, C = oracle(D)
        same_U(U, Ux, f"D={D.tolist()}")
        close_to_exact(C, Cx, what=f"D={D.tolist()}")


def pin_simplex(oracle):
    """All off-diagonal distances equal: U_xy = n, C_xx = 1/n, C_xz = (n-2)/(2n(n-1))."""
    for n in (2, 3, 5, 9, 16):
        D = np.ones((n, n), dtype=np.float32) * 3.5
        np.fill_diagonal(D, 0)
        U, C = oracle(D)
        Ux = np.full((n, n), n)
        np.fill_diagonal(Ux, 1)
        same_U(U, Ux, f"simplex n={n}")
        Cx = [[Fraction(1, n) if x == z else Fraction(n - 2, 2 * n * (n - 1)) for z in range(n)]
              for x in range(n)]
        close_to_exact(C, Cx, what=f"simplex n={n}")


def separated_clusters(sizes, intra, inter):
    """K clusters; all pairs inside cluster k at distance intra[k]; all cross pairs at inter."""
    n = sum(sizes)
    lab = np.repeat(np.arange(len(sizes)), sizes)
    D = np.full((n, n), inter, dtype=np.float32)
    for k in range(len(sizes)):
        idx = np.where(lab == k)[0]
        D[np.ix_(idx, idx)] = intra[k]
    np.fill_diagonal(D, 0)
    return D, lab


def pin_clusters(oracle):
    """Closed form for K equidistant separated clusters of different sizes and densities.

    x in a cluster of size a: same-cluster foci hold the cluster (u = a), cross
    foci hold everything (u = n).  Then
      C_xx = [(a-1)/a + (n-a)/n] / (n-1)
      C_xz = [(a-2)/(2a) + (n-a)/n] / (n-1)          z != x in x's cluster
      C_xz = (n-a-c) / (2n(n-1))                     z in another cluster of size c
    """
    for sizes, intra in (((2, 3, 4), (1.0, 2.0, 0.5)), ((1, 1, 1, 1), (1.0, 1.0, 1.0, 1.0)),
                         ((3, 3), (1.0, 4.0)), ((2, 5, 1, 3), (0.25, 3.0, 1.0, 2.5))):
        D, lab = separated_clusters(sizes, intra, 10.0)
        n = D.shape[0]
        U, C = oracle(D)
        Ux = np.where(lab[:, None] == lab[None, :], np.asarray(sizes)[lab][:, None], n)
        np.fill_diagonal(Ux, 1)
        same_U(U, Ux, f"clusters {sizes}")
        Cx = [[None] * n for _ in range(n)]
        for x in range(n):
            a = sizes[lab[x]]
            for z in range(n):
                if z == x:
                    v = Fraction(a - 1, a) + Fraction(n - a, n)
                    v /= n - 1
                elif lab[z] == lab[x]:
                    v = (Fraction(a - 2, 2 * a) + Fraction(n - a, n)) / (n - 1)
                else:
                    c = sizes[lab[z]]
                    v = Fraction(n - a - c, 2 * n * (n - 1))
                Cx[x][z] = v
        close_to_exact(C, Cx, what=f"clusters {sizes}")
    # two clusters, arbitrary cross distances above every intra distance: no cross cohesion
    rng = np.random.default_rng(7)
    D, lab = separated_clusters((4, 6), (1.0, 2.0), 10.0)
    cross = lab[:, None] != lab[None, :]
    R = rng.uniform(5.0, 50.0, size=D.shape).astype(np.float32)
    R = np.triu(R, 1)
    R = R + R.T
    D = np.where(cross, R, D).astype(np.float32)
    U, C = oracle(D)
    assert (C[cross] == 0).all(), "cross-cluster cohesion must vanish for two separated clusters"


def pin_triplet_formulation(oracle):
    """The oracle equals the tie-exact triplet enumeration (a second formulation)."""
    for k, D in enumerate(_random_small_cases()[::2]):
        Ux, Cx = exact_pald.by_triplets(D)
        U, C = oracle(D)
        same_U(U, Ux, f"triplet case {k}")
        close_to_exact(C, Cx, what=f"triplet case {k}")


def pin_invariants(oracle):
    rng = np.random.default_rng(99)
    for n, vals in ((40, None), (33, (0, 1, 2, 3)), (50, None)):
        if vals is None:
            P = rng.random((n, 4))
            diff = P[:, None, :] - P[None, :, :]
            D = np.sqrt((diff * diff).sum(-1)).astype(np.float32)
            D = np.triu(D, 1)
            D = D + D.T
        else:
            v = rng.choice(np.asarray(vals, dtype=np.float32), size=(n, n))
            v = np.triu(v, 1)
            D = (v + v.T).astype(np.float32)
        U, C = oracle(D)
        check_invariants(D, U, C, f"n={n}")


def pin_permutation(oracle):
    """Relabelling the points permutes U and C the same way."""
    rng = np.random.default_rng(5)
    n = 37
    v = rng.choice(np.asarray((1, 2, 3, 4, 5, 6), dtype=np.float32), size=(n, n))
    v = np.triu(v, 1)
    D = (v + v.T).astype(np.float32)
    p = rng.permutation(n)
    U, C = oracle(D)
    Up, Cp = oracle(D[np.ix_(p, p)])
    same_U(Up, np.asarray(U)[np.ix_(p, p)], "permutation")
    assert np.allclose(Cp, C[np.ix_(p, p)], rtol=1e-13, atol=0), "permutation C"


def pin_monotone_maps(oracle):
    """Strictly increasing maps of the distances that are exact in FP32 change nothing.

    Uses x -> 2x, x -> rank(x), and squared <-> Euclidean distances on an
    integer grid (PaLD only compares distances, Section 2).
    """
    rng = np.random.default_rng(11)
    n = 48
    P = rng.integers(0, 5, size=(n, 3)).astype(np.float64)
    diff = P[:, None, :] - P[None, :, :]
    sq = (diff * diff).sum(-1)
    Dsq = sq.astype(np.float32)
    Deu = np.sqrt(sq).astype(np.float32)
    U, C = oracle(Dsq)
    for what, D2 in (("euclidean", Deu), ("doubled", (2 * Dsq).astype(np.float32)),
                     ("rank", np.unique(Dsq, return_inverse=True)[1].reshape(n, n).astype(np.float32))):
        U2, C2 = oracle(D2)
        same_U(U2, U, what)
        assert np.array_equal(C2, C), f"{what}: C changed under an order-preserving map"


def pin_denormals(oracle):
    """Integer distances scaled into the denormal range compare exactly the same."""
    rng = np.random.default_rng(3)
    n = 30
    v = rng.integers(0, 7, size=(n, n)).astype(np.float32)
    v = np.triu(v, 1)
    D = (v + v.T).astype(np.float32)
    Dd = (D.astype(np.float64) * 2.0**-149).astype(np.float32)
    assert (Dd[D > 0] > 0).all() and (Dd[D > 0] < np.finfo(np.float32).tiny).all()
    U, C = oracle(D)
    Ud, Cd = oracle(Dd)
    same_U(Ud, U, "denormal")
    assert np.array_equal(Cd, C), "denormal distances changed C"


ALL_PINS = [
    pin_golden,
    pin_bruteforce_random,
    pin_exhaustive_ties,
    pin_simplex,
    pin_clusters,
    pin_triplet_formulation,
    pin_invariants,
    pin_permutation,
    pin_monotone_maps,
    pin_denormals,
]
