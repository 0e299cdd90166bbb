"""Exact-rational PaLD for tiny inputs (tests only).

Two formulations that do not share code with the FP64 oracle in `oracle/`:

* :func:`by_probability` -- straight from the probabilistic definition of
  cohesion (Section 2, Eq. (LD) and Eq. (cohesion)): Y is uniform on S \\ {x},
  Z is uniform on the local focus U_xY, and c_xz is the probability of the
  event {Z = z and d_Zx < d_ZY}, a tie d_Zx = d_ZY counting one half
  (Section 5: support is split on ties).
* :func:`by_triplets` -- a tie-exact version of the triplet idea (Section 3,
  triplet algorithm): every unordered triple {x, y, z} is visited once, each of
  its three pairs is tested for being a focus that contains the third point,
  and the six possible cohesion contributions are shared out; the terms where
  the third point coincides with one of the pair (the diagonal of C, and the
  duplicate-point case) are added per pair.

Both use Python Fractions, so they are exact; they are only used for n <= 8.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations

HALF = Fraction(1, 2)


def _vals(D):
    return [[Fraction(float(v)) for v in row] for row in D]


def focus(d, x, y):
    """The local focus U_xy = {z : d_xz <= d_xy or d_yz <= d_xy} (Section 2)."""
    n = len(d)
    return [z for z in range(n) if d[x][z] <= d[x][y] or d[y][z] <= d[x][y]]


def support(p, q):
    """[p < q] + 1/2 [p == q]."""
    if p < q:
        return Fraction(1)
    if p == q:
        return HALF
    return Fraction(0)


def by_probability(D):
    """(U, C) with U[x][y] = |U_xy| and C[x][z] = Pr[Z = z and d_Zx < d_ZY]."""
    d = _vals(D)
    n = len(d)
    U = [[len(focus(d, x, y)) for y in range(n)] for x in range(n)]
    C = [[Fraction(0)] * n for _ in range(n)]
    for x in range(n):
        for Y in range(n):
            if Y == x:
                continue
            F = focus(d, x, Y)
            pY = Fraction(1, n - 1)
            pZ = Fraction(1, len(F))
            for Z in F:
                C[x][Z] += pY * pZ * support(d[Z][x], d[Z][Y])
    return U, C


def by_triplets(D):
    """(U, C) from one visit per unordered triple plus per-pair self terms."""
    d = _vals(D)
    n = len(d)
    U = [[0] * n for _ in range(n)]
    for x in range(n):
        U[x][x] = sum(1 for z in range(n) if d[x][z] <= 0)
    for x, y in combinations(range(n), 2):
        U[x][y] = U[y][x] = 2  # x and y always lie in their own focus
    for x, y, z in combinations(range(n), 3):
        a, b, c = d[x][y], d[x][z], d[y][z]
        if min(b, c) <= a:
            U[x][y] += 1
            U[y][x] += 1
        if min(a, c) <= b:
            U[x][z] += 1
            U[z][x] += 1
        if min(a, b) <= c:
            U[y][z] += 1
            U[z][y] += 1

    C = [[Fraction(0)] * n for _ in range(n)]
    for x, y, z in combinations(range(n), 3):
        a, b, c = d[x][y], d[x][z], d[y][z]
        if min(b, c) <= a:  # z in the focus of (x, y)
            w = Fraction(1, U[x][y])
            C[x][z] += support(b, c) * w
            C[y][z] += support(c, b) * w
        if min(a, c) <= b:  # y in the focus of (x, z)
            w = Fraction(1, U[x][z])
            C[x][y] += support(a, c) * w
            C[z][y] += support(c, a) * w
        if min(a, b) <= c:  # x in the focus of (y, z)
            w = Fraction(1, U[y][z])
            C[y][x] += support(a, b) * w
            C[z][x] += support(b, a) * w
    for x, y in combinations(range(n), 2):
        a = d[x][y]
        w = Fraction(1, U[x][y])
        C[x][x] += support(0, a) * w  # third point x in the focus of (x, y)
        C[y][y] += support(0, a) * w  # third point y in the focus of (y, x)
        C[x][y] += support(a, 0) * w  # third point y, second point y: nonzero only if a == 0
        C[y][x] += support(a, 0) * w
    s = Fraction(1, n - 1)
    C = [[v * s for v in row] for row in C]
    return U, C
