"""Blocks of rows (pald_cohesion_rows) and the out-of-core mode (pald_cohesion_ooc):
U bit-exact against the oracle and the whole-matrix call, C within 1e-6 relative
of the oracle (exactly 0 where it is 0)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_c_close, assert_u_equal, log, to_gpu
from paper_2307_16652_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_16652_amd import pald

    pald.load_library()


def sample_rows(n, bounds, k=48, seed=7):
    """Seeded random rows plus the first, last and panel-edge rows."""
    rng = np.random.default_rng(seed)
    edges = [b for x in bounds for b in (x - 1, x) if 0 <= b < n]
    return np.unique(np.concatenate([[0, n - 1], edges, rng.choice(n, size=k, replace=False)]))


@pytest.mark.parametrize("n,bounds", [(300, [0, 37, 300]), (257, [0, 64, 65, 128, 257]), (2, [0, 1, 2])],
                         ids=["n300_ragged", "n257_one_row_panel", "n2"])
def test_rows_small_full_oracle(n, bounds):
    """Panels at unaligned starts (x0 % 4 != 0), a one-row panel, n = 2."""
    import torch

    from paper_2307_16652_amd import pald

    D = synth.grid3d(n=n, seed=60 + n) if n > 2 else np.array([[0, 3], [3, 0]], dtype=np.float32)
    Uo, Co = oracle.pald(D)
    Dg = to_gpu(D)
    for x0, x1 in zip(bounds[:-1], bounds[1:]):
        log(f"[rows] n={n} rows [{x0}, {x1})")
        U, C = pald.cohesion_rows(Dg, x0, x1)
        torch.cuda.synchronize()
        assert_u_equal(U.cpu().numpy(), Uo[x0:x1], f"rows [{x0},{x1}) U")
        assert_c_close(C.cpu().numpy(), Co[x0:x1], what=f"rows [{x0},{x1}) C")


def test_rows_eight_panels_n16384_reassemble():
    """The n = 16384 integer-grid workload in 8 panels of 2048 rows: the panels
    reassemble the whole-matrix call's U exactly, and C is within 1e-6 of the
    oracle on sampled rows and within 2e-6 of the whole-matrix C everywhere."""
    import torch

    from paper_2307_16652_amd import pald

    n = 16384
    D = synth.grid3d()
    Dg = to_gpu(D)
    Uw, Cw = pald.cohesion(Dg)
    Cw64 = Cw.double()
    bounds = list(range(0, n + 1, 2048))
    rows = sample_rows(n, bounds)
    Uo, Co = oracle.pald_rows(D, rows)
    Ur = torch.empty((n, n), dtype=torch.int32, device="cuda")
    Cr = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ws = torch.empty(pald.rows_workspace_bytes(n, 2048), dtype=torch.uint8, device="cuda")
    for x0, x1 in zip(bounds[:-1], bounds[1:]):
        log(f"[rows] n=16384 panel [{x0}, {x1})")
        pald.cohesion_rows(Dg, x0, x1, ws=ws, out_u=Ur[x0:x1], out_c=Cr[x0:x1])
    torch.cuda.synchronize()
    assert torch.equal(Ur, Uw), "panel U differs from the whole-matrix U"
    Ur_rows = Ur[torch.from_numpy(rows).cuda()].cpu().numpy()
    Cr_rows = Cr[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert_u_equal(Ur_rows, Uo, "panels U rows vs oracle")
    err = assert_c_close(Cr_rows, Co, what="panels C rows vs oracle")
    zero = Cw64 == 0
    assert bool(((Cr == 0) == zero).all()), "exact zeros differ between panels and the whole matrix"
    rel = ((Cr.double() - Cw64).abs() / Cw64.abs().clamp_min(1e-300)).masked_fill(zero, 0.0)
    worst = float(rel.max().item())
    log(f"  {rows.size} oracle rows: max rel err {err:.3e}; panels vs whole matrix {worst:.3e}")
    assert worst <= 2e-6


@pytest.mark.parametrize("n,budget_rows", [(1000, 16), (333, 48), (64, 64)], ids=["n1000_p16", "n333_p48", "n64_p64"])
def test_ooc_small_full_oracle(n, budget_rows):
    """Out of core with the workspace of a panel of `budget_rows` rows: many panels
    and blocks, ragged last ones; against the full oracle."""
    from paper_2307_16652_amd import pald

    D = synth.mixture8d(n=n, seed=70 + n)
    Uo, Co = oracle.pald(D)
    ws = pald.ooc_workspace_bytes(n, budget_rows)
    log(f"[ooc] n={n}, workspace {ws} bytes ({budget_rows}-row panels)")
    U, C = pald.cohesion_ooc(D, ws)
    assert_u_equal(U, Uo, f"ooc n={n} U")
    assert_c_close(C, Co, what=f"ooc n={n} C")
    _, C2 = pald.cohesion_ooc(D, ws, want_u=False)
    assert np.array_equal(C2.view(np.uint32), C.view(np.uint32)), "ooc C without U differs"


def test_ooc_n16384_small_budget():
    """The n = 16384 workload through a 256 MiB device workspace (D alone is 1 GiB):
    29 panels of 576 rows, D streamed in blocks; U equal to the whole-matrix call,
    C within 1e-6 of the oracle on sampled rows."""
    import time

    import torch

    from paper_2307_16652_amd import pald

    n = 16384
    D = synth.grid3d()
    Dg = to_gpu(D)
    Uw, Cw = pald.cohesion(Dg)
    torch.cuda.synchronize()
    Uw, Cw = Uw.cpu().numpy(), Cw.cpu().numpy()
    del Dg
    budget = 256 << 20
    t0 = time.time()
    U, C = pald.cohesion_ooc(D, budget)
    log(f"[ooc] n=16384 in {budget >> 20} MiB of device workspace: {time.time() - t0:.1f} s")
    assert np.array_equal(U, Uw), "out-of-core U differs from the whole-matrix U"
    rows = sample_rows(n, list(range(0, n, 576)) + [n], k=32)
    Uo, Co = oracle.pald_rows(D, rows)
    assert_u_equal(U[rows], Uo, "ooc U rows vs oracle")
    err = assert_c_close(C[rows], Co, what="ooc C rows vs oracle")
    zero = Cw == 0
    assert np.array_equal(C == 0, zero), "exact zeros differ between out-of-core and whole-matrix C"
    rel = np.abs(C.astype(np.float64) - Cw) / np.where(zero, 1.0, Cw.astype(np.float64))
    log(f"  max rel err {err:.3e} on {rows.size} oracle rows; vs whole matrix {rel.max():.3e}")
    assert rel.max() <= 2e-6
