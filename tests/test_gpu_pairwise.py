"""GPU parity of the pairwise path (libpald through the C ABI) against the FP64 oracle.

U must match the oracle bit for bit; every C entry must be within 1e-6
relative of the oracle, and exactly 0 where the oracle is exactly 0.
"""
import numpy as np
import pytest

import oracle
import pins
from gpu_helpers import assert_c_close, assert_u_equal, check_invariants, gpu_cohesion, log, to_gpu
from paper_2307_16652_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_16652_amd import pald

    pald.load_library()


def parity(D, what, rows=None, **opts):
    log(f"[parity] {what} n={D.shape[0]} opts={opts}")
    U, C = gpu_cohesion(D, **opts)
    if rows is None:
        Uo, Co = oracle.pald(D)
        assert_u_equal(U, Uo, what)
        err = assert_c_close(C, Co, what=what)
    else:
        Uo, Co = oracle.pald_rows(D, rows)
        assert_u_equal(U[rows], Uo, what)
        err = assert_c_close(C[rows], Co, what=what)
    return U, C, err


def test_golden_examples():
    from fractions import Fraction  # noqa: F401

    for f in pins.golden_files():
        D, Ux, Cx = pins.load_golden(f)
        U, C = gpu_cohesion(D)
        assert_u_equal(U, Ux, f)
        Cref = np.array([[float(v) for v in row] for row in Cx])
        assert_c_close(C, Cref, what=f)


@pytest.mark.parametrize("values", [(1.0, 2.0), (0.0, 1.0, 2.0)], ids=["ones_twos", "with_zero"])
def test_exhaustive_tie_patterns_n4(values):
    """Every symmetric zero-diagonal 4x4 matrix with entries from `values`."""
    from paper_2307_16652_amd import pald

    import torch

    mats = list(pins.exhaustive_n4(values))
    log(f"[parity] exhaustive n=4 over {values}: {len(mats)} matrices")
    ws = pald.workspace(4, torch.device("cuda:0"))
    outs = []
    for D in mats:
        outs.append(pald.cohesion(to_gpu(D), ws=ws))
    torch.cuda.synchronize()
    for D, (U, C) in zip(mats, outs):
        Uo, Co = oracle.pald(D, threads=1)
        assert_u_equal(U.cpu().numpy(), Uo, f"D={D.tolist()}")
        assert_c_close(C.cpu().numpy(), Co, what=f"D={D.tolist()}")


SIZES = [2, 3, 5, 17, 63, 64, 65, 127, 128, 129, 191, 255, 257, 300]


@pytest.mark.parametrize("n", SIZES)
def test_sizes_continuous(n):
    parity(synth.mixture8d(n=n, seed=100 + n), f"mixture8d n={n}")


@pytest.mark.parametrize("n", [3, 64, 129, 257, 300])
def test_sizes_grid_ties(n):
    # a 4x4x4 grid: heavy ties and many duplicate points
    P = np.random.default_rng(n).integers(0, 4, size=(n, 3))
    D = synth.pairwise_distances(P, squared=True)
    parity(D, f"grid4 n={n}")


@pytest.mark.parametrize("n", [6, 70, 200])
def test_random_tie_matrices(n):
    D = synth.random_tie_matrix(n, (0.0, 1.0, 2.0, 3.0), seed=n)
    parity(D, f"random ties n={n}")


def test_denormal_distances():
    """Integer distances scaled by 2^-149 are denormals; results must not change."""
    n = 150
    P = np.random.default_rng(5).integers(0, 6, size=(n, 3))
    D = synth.pairwise_distances(P, squared=True)
    Dd = (D.astype(np.float64) * 2.0**-149).astype(np.float32)
    assert (Dd[D > 0] < np.finfo(np.float32).tiny).all()
    U, C, _ = parity(D, "integer")
    Ud, Cd, _ = parity(Dd, "denormal")
    assert np.array_equal(U, Ud)
    assert np.array_equal(C, Cd)


@pytest.mark.parametrize("y_chunks,z_chunks", [(1, 1), (3, 1), (1, 3), (7, 5), (20, 19)])
def test_forced_splits(y_chunks, z_chunks):
    D = synth.uniform2d(n=300, seed=9)
    parity(D, f"splits y={y_chunks} z={z_chunks}", y_chunks=y_chunks, z_chunks=z_chunks)


@pytest.mark.parametrize("n", [5, 129, 300])
def test_f64_accumulation(n):
    parity(synth.grid3d(n=n, seed=n), f"f64 n={n}", accum="f64")


def test_leading_dimensions_and_unaligned_rows():
    """D, U, C embedded in wider buffers, including a row pitch that is not a multiple of 4."""
    import torch

    from paper_2307_16652_amd import pald

    n = 133
    D = synth.mixture8d(n=n, seed=3)
    Uo, Co = oracle.pald(D)
    for pitch in (n + 1, n + 4, 160):
        big = torch.zeros((n, pitch), dtype=torch.float32, device="cuda:0")
        big[:, :n] = to_gpu(D)
        Ubig = torch.full((n, pitch + 3), -7, dtype=torch.int32, device="cuda:0")
        Cbig = torch.full((n, pitch + 5), -7.0, dtype=torch.float32, device="cuda:0")
        U, C = pald.cohesion(big[:, :n], out_u=Ubig[:, :n], out_c=Cbig[:, :n])
        torch.cuda.synchronize()
        assert_u_equal(U.cpu().numpy(), Uo, f"pitch {pitch}")
        assert_c_close(C.cpu().numpy(), Co, what=f"pitch {pitch}")
        assert (Ubig[:, n:].cpu().numpy() == -7).all(), "wrote outside the U block"
        assert (Cbig[:, n:].cpu().numpy() == -7.0).all(), "wrote outside the C block"


def test_focus_sizes_only_and_optional_u():
    import torch

    from paper_2307_16652_amd import pald

    D = synth.grid3d(n=260, seed=4)
    Uo, Co = oracle.pald(D)
    Dg = to_gpu(D)
    for zc in (0, 1, 4):
        U = pald.focus_sizes(Dg, z_chunks=zc)
        torch.cuda.synchronize()
        assert_u_equal(U.cpu().numpy(), Uo, f"focus_sizes z_chunks={zc}")
    for zc in (1, 4):
        U, C = pald.cohesion(Dg, want_u=False, z_chunks=zc)
        torch.cuda.synchronize()
        assert U is None
        assert_c_close(C.cpu().numpy(), Co, what=f"no U z_chunks={zc}")


def test_deterministic():
    D = synth.grid3d(n=700, seed=12)
    U1, C1 = gpu_cohesion(D)
    U2, C2 = gpu_cohesion(D)
    assert np.array_equal(U1, U2) and np.array_equal(C1, C2)


def test_order_preserving_maps_give_identical_results():
    """Strictly increasing maps that are exact in float32 leave U and C bit-identical:
    squared vs Euclidean distances on an integer grid, D -> 2D, and D -> rank(D)."""
    P = np.random.default_rng(21).integers(0, 8, size=(400, 3))
    Dsq = synth.pairwise_distances(P, squared=True)
    Deu = synth.pairwise_distances(P, squared=False)
    U1, C1 = gpu_cohesion(Dsq)
    U2, C2 = gpu_cohesion(Deu)
    assert np.array_equal(U1, U2) and np.array_equal(C1, C2)
    D = synth.mixture8d(n=350, seed=23)
    vals, inv = np.unique(D, return_inverse=True)  # dense ranks, 0 for the zero diagonal
    Drank = inv.reshape(D.shape).astype(np.float32)
    assert vals[0] == 0 and len(vals) < 2**24
    U0, C0 = gpu_cohesion(D)
    for Dm, what in ((2.0 * D, "2D"), (Drank, "rank(D)")):
        Um, Cm = gpu_cohesion(np.ascontiguousarray(Dm, dtype=np.float32))
        assert np.array_equal(Um, U0), what
        assert np.array_equal(Cm.view(np.int32), C0.view(np.int32)), what


def test_permutation_equivariance():
    D = synth.mixture8d(n=311, seed=8)
    p = np.random.default_rng(1).permutation(311)
    U, C = gpu_cohesion(D)
    Up, Cp = gpu_cohesion(np.ascontiguousarray(D[np.ix_(p, p)]))
    assert np.array_equal(Up, U[np.ix_(p, p)])
    np.testing.assert_allclose(Cp, C[np.ix_(p, p)], rtol=2e-6, atol=0)


def test_check_input_flags():
    import torch

    from paper_2307_16652_amd import pald

    D = synth.uniform2d(n=64, seed=1)
    assert pald.check_input(to_gpu(D)) == []
    bad = D.copy()
    bad[3, 5] = np.nan
    bad[7, 7] = 1.0
    bad[10, 11] = -2.0
    bad[11, 10] = -2.0
    bad[20, 21] = np.inf
    bad[21, 20] = np.inf
    bad[30, 31] = 5.0
    flags = pald.check_input(to_gpu(bad))
    assert set(flags) == {"nan", "inf", "negative", "asymmetric", "nonzero_diagonal"}
    torch.cuda.synchronize()


def test_invalid_arguments_on_device():
    import torch

    from paper_2307_16652_amd import pald

    D = to_gpu(synth.uniform2d(n=64))
    with pytest.raises(pald.PaldError) as e:
        pald.cohesion(D, ws=torch.empty(64, dtype=torch.uint8, device="cuda:0"))
    assert e.value.status == pald.ERR_ARG


# ---------------------------------------------------------------------------
# the workload configurations


def test_config_uniform2d_n256_full():
    D = synth.uniform2d()
    U, C, err = parity(D, "uniform2d n=256 (full oracle)")
    check_invariants(U, C, "uniform2d")
    _, _, err64 = parity(D, "uniform2d n=256 (full oracle), FP64 form", accum="f64")
    log(f"  max rel err {err:.3e} (compensated), {err64:.3e} (FP64 form)")


def test_config_mixture8d_n4096_full():
    """The six-cluster mixture at n = 4096 against the full oracle (all 4096 rows)."""
    from gpu_helpers import oracle_full_cached

    D = synth.mixture8d()
    log("[parity] mixture8d n=4096 (full oracle)")
    Uo, Co = oracle_full_cached("mixture8d_4096", D)
    for variant in ("auto", "pairwise"):  # auto: the tuned choice at this size
        U, C = gpu_cohesion(D, variant=variant)
        assert_u_equal(U, Uo, f"mixture8d n=4096 {variant}")
        err = assert_c_close(C, Co, what=f"mixture8d n=4096 {variant}")
        check_invariants(U, C, "mixture8d")
    _, C64 = gpu_cohesion(D, accum="f64")
    err64 = assert_c_close(C64, Co, what="mixture8d n=4096, FP64 form")
    log(f"  max rel err {err:.3e} (compensated), {err64:.3e} (FP64 form)")


def grid3d_oracle_rows(n: int = 16384, k: int = 256):
    """The benchmark's seeded sample of oracle rows (the rows bench.py times the
    oracle on: default_rng(123), k distinct rows) plus rows 0 and n - 1."""
    rows = np.random.default_rng(123).choice(n, size=k, replace=False)
    return np.unique(np.concatenate([[0, n - 1], rows]))


_GRID3D_ROWS = {}


def grid3d_oracle_cached():
    """(D, rows, U rows, C rows) of the n = 16384 workload, the oracle run once."""
    if not _GRID3D_ROWS:
        D = synth.grid3d()
        rows = grid3d_oracle_rows()
        log(f"[parity] grid3d n=16384: oracle on {rows.size} rows")
        Uo, Co = oracle.pald_rows(D, rows)
        _GRID3D_ROWS.update(D=D, rows=rows, Uo=Uo, Co=Co)
    g = _GRID3D_ROWS
    return g["D"], g["rows"], g["Uo"], g["Co"]


@pytest.mark.parametrize("variant", ["pairwise", "hybrid2"])
def test_config_grid3d_n16384_sampled(variant):
    """The benchmark's workload against the oracle on the config's 256 seeded rows
    (plus the first and last): the pairwise variant in its compensated and
    FP64-accumulate forms, and the variant the tuned table runs at this size
    (pairwise pass 1 + triplet pass 2)."""
    D, rows, Uo, Co = grid3d_oracle_cached()
    log(f"[parity] grid3d n=16384 {variant}")
    U, C = gpu_cohesion(D, variant=variant)
    assert_u_equal(U[rows], Uo, f"grid3d n=16384 {variant} U rows")
    err = assert_c_close(C[rows], Co, what=f"grid3d n=16384 {variant} C rows")
    check_invariants(U, C, "grid3d")
    del U, C
    if variant != "pairwise":
        log(f"  {rows.size} rows: max rel err {err:.3e}")
        return
    U64, C64 = gpu_cohesion(D, accum="f64")
    assert_u_equal(U64[rows], Uo, "grid3d n=16384 U rows, FP64 form")
    err64 = assert_c_close(C64[rows], Co, what="grid3d n=16384 C rows, FP64 form")
    log(f"  {rows.size} rows: max rel err {err:.3e} (compensated), {err64:.3e} (FP64 form)")


def test_diagonal_identity_without_coincident_points():
    """With no zero off-diagonal distance, every focus of x contains x with full
    support, so C_xx = 1/(n-1) sum_{y != x} 1/U_xy (computed here from the GPU's U)."""
    D = synth.mixture8d(n=400, seed=31)
    assert (D[~np.eye(400, dtype=bool)] > 0).all()
    U, C = gpu_cohesion(D)
    Ud = U.astype(np.float64)
    np.fill_diagonal(Ud, np.inf)
    expect = (1.0 / Ud).sum(axis=1) / (400 - 1)
    np.testing.assert_allclose(np.diag(C).astype(np.float64), expect, rtol=1e-6, atol=0)


def test_cohesion_captured_in_a_graph_replays_exactly():
    """pald_cohesion enqueues kernels only (no allocation, no memset node), so it can
    be captured; every replay, with eager work in between, equals the eager result."""
    import torch

    from paper_2307_16652_amd import pald

    for n, opts in ((300, {}), (257, {"y_chunks": 3, "z_chunks": 2}), (300, {"variant": "hybrid2"}),
                    (260, {"variant": "triplet"})):
        D = to_gpu(synth.mixture8d(n=n, seed=40 + n))
        ws = pald.workspace(n, D.device, **opts)
        U = torch.empty((n, n), dtype=torch.int32, device="cuda")
        C = torch.empty((n, n), dtype=torch.float32, device="cuda")
        pald.cohesion(D, ws=ws, out_u=U, out_c=C, **opts)
        torch.cuda.synchronize()
        Ue, Ce = U.clone(), C.clone()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            pald.cohesion(D, ws=ws, out_u=U, out_c=C, **opts)
        torch.cuda.synchronize()
        for rep in range(3):
            U.fill_(-1)
            C.fill_(-1.0)
            _ = (D * 2.0).sum()  # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(U, Ue), f"n={n} replay {rep}: U differs"
            assert torch.equal(C, Ce), f"n={n} replay {rep}: C differs"
        del g


def test_cohesion_on_a_side_stream():
    import torch

    from paper_2307_16652_amd import pald

    D = synth.grid3d(n=260, seed=6)
    Uo, Co = oracle.pald(D)
    Dg = to_gpu(D)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        U, C = pald.cohesion(Dg)
    s.synchronize()
    assert_u_equal(U.cpu().numpy(), Uo, "side stream")
    assert_c_close(C.cpu().numpy(), Co, what="side stream")
