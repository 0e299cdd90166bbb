"""GPU parity of the triplet variant (one visit per unordered triple) against the oracle
and against the pairwise variant."""
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


def parity(D, what, rows=None):
    log(f"[triplet] {what} n={D.shape[0]}")
    U, C = gpu_cohesion(D, variant="triplet")
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
    for f in pins.golden_files():
        D, Ux, Cx = pins.load_golden(f)
        U, C = gpu_cohesion(D, variant="triplet")
        assert_u_equal(U, Ux, f)
        assert_c_close(C, np.array([[float(v) for v in row] for row in Cx]), what=f)


@pytest.mark.parametrize("values", [(1.0, 2.0), (0.0, 1.0, 2.0)], ids=["ones_twos", "with_zero"])
def test_exhaustive_tie_patterns_n4(values):
    import torch

    from paper_2307_16652_amd import pald

    mats = list(pins.exhaustive_n4(values))
    ws = pald.workspace(4, torch.device("cuda:0"), variant="triplet")
    outs = [pald.cohesion(to_gpu(D), variant="triplet", ws=ws) for D in mats]
    torch.cuda.synchronize()
    for D, (U, C) in zip(mats, outs):
        Uo, Co = oracle.pald(D, threads=1)
        assert_u_equal(U.cpu().numpy(), Uo, f"D={D.tolist()}")
        assert_c_close(C.cpu().numpy(), Co, what=f"D={D.tolist()}")


@pytest.mark.parametrize("n", [2, 3, 5, 17, 63, 64, 65, 127, 129, 200, 257])
def test_sizes(n):
    parity(synth.mixture8d(n=n, seed=200 + n), f"mixture8d n={n}")


@pytest.mark.parametrize("n", [7, 64, 130, 260])
def test_ties_and_duplicates(n):
    P = np.random.default_rng(n).integers(0, 4, size=(n, 3))
    parity(synth.pairwise_distances(P, squared=True), f"grid4 n={n}")


def test_random_tie_matrix():
    parity(synth.random_tie_matrix(150, (0.0, 1.0, 2.0, 3.0), seed=3), "random ties")


def test_focus_sizes_triplet_matches_pairwise():
    import torch

    from paper_2307_16652_amd import pald

    D = synth.grid3d(n=333, seed=5)
    Dg = to_gpu(D)
    Ut = pald.focus_sizes(Dg, variant="triplet")
    Up = pald.focus_sizes(Dg, variant="pairwise")
    torch.cuda.synchronize()
    assert torch.equal(Ut, Up)


def test_triplet_vs_pairwise_and_optional_u():
    import torch

    from paper_2307_16652_amd import pald

    D = synth.mixture8d(n=500, seed=6)
    Dg = to_gpu(D)
    Up, Cp = pald.cohesion(Dg, variant="pairwise")
    Ut, Ct = pald.cohesion(Dg, variant="triplet")
    _, Cn = pald.cohesion(Dg, variant="triplet", want_u=False)
    torch.cuda.synchronize()
    assert torch.equal(Up, Ut)
    np.testing.assert_allclose(Ct.cpu().numpy(), Cp.cpu().numpy(), rtol=2e-6, atol=0)
    np.testing.assert_allclose(Cn.cpu().numpy(), Cp.cpu().numpy(), rtol=2e-6, atol=0)


def test_unsupported_option_combinations():
    from paper_2307_16652_amd import pald

    D = to_gpu(synth.uniform2d(n=64))
    with pytest.raises(pald.PaldError) as e:
        pald.cohesion(D, variant="triplet", accum="f64")
    assert e.value.status == pald.ERR_UNSUPPORTED


def test_config_mixture8d_n4096_full():
    """The configuration the two variants are compared on, against the full oracle."""
    from gpu_helpers import assert_c_close, assert_u_equal, gpu_cohesion, oracle_full_cached

    D = synth.mixture8d()
    log("[triplet] mixture8d n=4096 (full oracle)")
    U, C = gpu_cohesion(D, variant="triplet")
    Uo, Co = oracle_full_cached("mixture8d_4096", D)
    assert_u_equal(U, Uo, "triplet mixture8d n=4096")
    err = assert_c_close(C, Co, what="triplet mixture8d n=4096")
    check_invariants(U, C, "triplet mixture8d")
    log(f"  max rel err {err:.3e}")


@pytest.mark.parametrize("variant", ["triplet", "hybrid", "hybrid2"])
def test_bitwise_reproducible(variant):
    """U and C of the triplet and hybrid variants are the same bits on every run:
    their owners' partial sums are combined with integer (fixed-point) atomics,
    which commute, so the arrival order of the atomics does not matter."""
    import torch

    from paper_2307_16652_amd import pald

    D = to_gpu(synth.mixture8d(n=1500, seed=81))
    ws = pald.workspace(1500, D.device, variant=variant)
    U0, C0 = pald.cohesion(D, variant=variant, ws=ws)
    U0, C0 = U0.clone(), C0.clone()
    for rep in range(4):
        _ = (D * 3.0).sum()  # unrelated work between the runs
        U, C = pald.cohesion(D, variant=variant, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(U, U0), f"{variant} run {rep}: U differs"
        assert torch.equal(C.view(torch.int32), C0.view(torch.int32)), f"{variant} run {rep}: C bits differ"
