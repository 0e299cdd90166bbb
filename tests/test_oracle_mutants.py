"""Plant plausible mistakes in copies of the oracle and require a pin to catch each.

Each mutant is the oracle's C source with one textual change, compiled with gcc
into a temporary library.  The real oracle is untouched.  A mutant that passes
every pin would mean the pins cannot tell that mistake from the definition.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pald_oracle.c")

MUTANTS = {
    # Alg. 1 / Alg. 2 style strict focus test (ties ignored, Section 5)
    "strict_focus": ("dxz <= dxy || dyz <= dxy", "dxz < dxy || dyz < dxy"),
    "and_focus": ("dxz <= dxy || dyz <= dxy", "dxz <= dxy && dyz <= dxy"),
    "tie_to_y": ("s = 0.5;", "s = 0.0;"),
    "tie_double_counted": ("s = 0.5;", "s = 1.0;"),
    "y_includes_x": ("if (y == x)          /* Y is drawn from S \\ {x} */\n            continue;", ";"),
    "normalise_by_n": ("Crow[z] /= (double)(n - 1);", "Crow[z] /= (double)n;"),
    "support_flipped": ("if (dxz < dyz)", "if (dxz > dyz)"),
    "membership_wrong_distance": ("if (!(dxz <= dxy))", "if (!(dyz <= dxy))"),
    "focus_off_by_one": ("int64_t u = 0;", "int64_t u = 1;"),
    "no_focus_weight": ("Crow[z] += s / (double)u;", "Crow[z] += s;"),
    "no_normalisation": ("Crow[z] /= (double)(n - 1);", ";"),
    "focus_compares_wrong_pair": ("dxz <= dxy || dyz <= dxy", "dxz <= dyz || dyz <= dxy"),
}


def _build_mutant(name, tmp_path):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation anchor for {name} not found in the oracle source"
    mutated = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(mutated)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", str(so), str(c)])
    lib = ctypes.CDLL(str(so))
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    lib.pald_oracle_full.argtypes = [vp, i64, i64, vp, vp, ctypes.c_int]
    lib.pald_oracle_full.restype = ctypes.c_int

    def oracle(D):
        D = np.ascontiguousarray(np.asarray(D, dtype=np.float32))
        n = D.shape[0]
        U = np.empty((n, n), np.int32)
        C = np.empty((n, n), np.float64)
        assert lib.pald_oracle_full(D.ctypes.data, n, n, U.ctypes.data, C.ctypes.data, 1) == 0
        return U, C

    return oracle


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    oracle = _build_mutant(name, tmp_path)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(oracle)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"


# ---------------------------------------------------------------------------
# the distance front end and the steps after the two passes

DIST_SRC = os.path.join(ROOT, "oracle", "distance_oracle.c")
DIST_MUTANTS = {
    "dim_off_by_one": ("k < dim;", "k < dim - 1;"),
    "no_sqrt": ("sqrt(acc) : acc", "acc : acc"),
    "metric_swapped": ("metric == ORACLE_METRIC_EUCLIDEAN ?", "metric == ORACLE_METRIC_SQEUCLIDEAN ?"),
    "same_point_twice": ("- coord(P, dtype, ldp, y, k)", "- coord(P, dtype, ldp, x, k)"),
    "f64_read_as_f32": ("if (dtype == ORACLE_F64)", "if (0)"),
    "abs_not_square": ("acc = fma(delta, delta, acc);", "acc = acc + fabs(delta);"),
    "hops_not_counted": ("dist[w] = dist[u] + 1;", "dist[w] = dist[u];"),
    "source_at_one": ("dist[s] = 0;", "dist[s] = 1;"),
    "unreachable_at_n_minus_1": ("(float)(dist[v] >= 0 ? dist[v] : n)", "(float)(dist[v] >= 0 ? dist[v] : n - 1)"),
    "depth_first": ("const int64_t u = queue[head++];", "const int64_t u = queue[--tail];"),
}


@pytest.mark.parametrize("name", sorted(DIST_MUTANTS))
def test_distance_mutant_is_caught(name, tmp_path, monkeypatch):
    import oracle
    import test_oracle_analysis as ta

    src = open(DIST_SRC).read()
    old, new = DIST_MUTANTS[name]
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", str(so), str(c), "-lm"])
    lib = ctypes.CDLL(str(so))
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    lib.pald_oracle_distances.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.c_int, vp, i64, vp, i64]
    lib.pald_oracle_distances.restype = ctypes.c_int
    lib.pald_oracle_graph_distances.argtypes = [vp, vp, i64, vp, i64, vp, i64]
    lib.pald_oracle_graph_distances.restype = ctypes.c_int
    monkeypatch.setattr(oracle, "_lib", lib)
    caught = []
    for pin in (ta.test_distances_integer_coordinates_exact, ta.test_distances_pythagorean,
                ta.test_distances_match_scipy_and_are_symmetric, ta.test_graph_distances_closed_forms,
                ta.test_graph_distances_components_and_isolated_vertices,
                ta.test_graph_distances_match_scipy_on_collaboration_graphs,
                ta.test_graph_distances_ignore_out_of_range_neighbours):
        try:
            pin()
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"distance mutant {name} passed every pin"


PY_MUTANTS = {
    "ties_at_equality": ("strong_ties", "C[x] > t", "C[x] >= t"),
    "ties_keep_diagonal": ("strong_ties", "z = z[z != x]", "z = z"),
    "depth_column_sums": ("local_depths", ".sum(axis=1)", ".sum(axis=0)"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_python_step_mutant_is_caught(name, monkeypatch):
    import inspect
    import textwrap

    import oracle
    import test_oracle_analysis as ta

    fn, old, new = PY_MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(getattr(oracle, fn)))
    assert src.count(old) == 1, f"mutation anchor for {name} not found"
    scope = dict(vars(oracle))
    exec(src.replace(old, new), scope)
    monkeypatch.setattr(oracle, fn, scope[fn])
    caught = []
    for pin in (ta.test_depths_of_the_worked_examples, ta.test_depths_equal_the_probability_definition,
                ta.test_depths_closed_forms, ta.test_strong_ties_brute_force,
                ta.test_strong_ties_extremes_equality_and_diagonal, ta.test_strong_ties_of_two_clusters):
        try:
            pin()
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
