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
