"""GPU parity of the batched persistent mode (one launch for many matrices)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_c_close, assert_u_equal, check_invariants, log
from paper_2307_16652_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2307_16652_amd import pald

    pald.load_library()


def make_batch(sizes, seed=0, kind="mixture"):
    mats = []
    for i, n in enumerate(sizes):
        if kind == "grid":
            P = np.random.default_rng([seed, i]).integers(0, 4, size=(n, 3))
            mats.append(synth.pairwise_distances(P, squared=True))
        else:
            mats.append(synth.pairwise_distances(synth.batch_points(i, int(n), seed=seed)))
    return mats


def run_batch(mats, config=None, want_u=True):
    import torch

    from paper_2307_16652_amd import pald

    plan = pald.BatchPlan([m.shape[0] for m in mats], config=config)
    Dp = torch.from_numpy(np.concatenate([m.reshape(-1) for m in mats])).cuda()
    ws = plan.workspace(Dp.device)
    Up, Cp = plan.run(Dp, ws=ws, want_u=want_u)
    torch.cuda.synchronize()
    Us = [u.cpu().numpy() for u in plan.unpack(Up)] if Up is not None else None
    Cs = [c.cpu().numpy() for c in plan.unpack(Cp)]
    return plan, ws, Us, Cs


def check_all(mats, Us, Cs, every=1, what=""):
    """Oracle parity of every `every`-th matrix; returns the largest relative error of C."""
    worst = 0.0
    for i, D in enumerate(mats):
        if i % every:
            continue
        Uo, Co = oracle.pald(D)
        if Us is not None:
            assert_u_equal(Us[i], Uo, f"{what} matrix {i} (n={D.shape[0]})")
        worst = max(worst, assert_c_close(Cs[i], Co, what=f"{what} matrix {i} (n={D.shape[0]})"))
    return worst


RAGGED = [2, 3, 5, 17, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 200, 257, 300]


def form_config(form):
    """None (the library's built-in, tuned configuration) or an explicit launch form."""
    from paper_2307_16652_amd import pald

    return None if form == "builtin" else pald.make_batch_config(split_pass1=(form == "split"))


FORMS = ["builtin", "one_launch", "split"]


@pytest.mark.parametrize("form", FORMS)
def test_ragged_sizes(form):
    mats = make_batch(RAGGED, seed=1)
    log(f"[batched] ragged {RAGGED}, {form}")
    _, _, Us, Cs = run_batch(mats, config=form_config(form))
    check_all(mats, Us, Cs, what=f"ragged {form}")


@pytest.mark.parametrize("form", FORMS)
def test_tie_heavy_and_duplicates(form):
    sizes = [4, 9, 64, 70, 150]
    mats = make_batch(sizes, seed=2, kind="grid")
    _, _, Us, Cs = run_batch(mats, config=form_config(form))
    check_all(mats, Us, Cs, what=f"grid {form}")


@pytest.mark.parametrize("chunks", [2, 3, 7])
def test_y_split_tiles(chunks):
    from paper_2307_16652_amd import pald

    sizes = [40, 65, 130, 260, 33]
    mats = make_batch(sizes, seed=3)
    cfg = pald.make_batch_config([(50, 1), (1 << 30, chunks)])
    log(f"[batched] y split {chunks}")
    _, _, Us, Cs = run_batch(mats, config=cfg)
    check_all(mats, Us, Cs, what=f"y_chunks={chunks}")


@pytest.mark.parametrize("chunks", [1, 3])
def test_small_pass2_tiles(chunks):
    """The 32-wide pass-2 tile (chosen per size bucket): oracle parity on ragged and
    tie-heavy sizes, with and without a y split, and C bit-identical to the 64-wide
    tile of the general kernel (each C entry is summed over y in the same order by
    both shapes).  With 64-wide tiles everywhere and no y split the one-launch form
    runs the lean kernel (longer float32 runs): C then agrees to the error bound."""
    from paper_2307_16652_amd import pald

    mats = make_batch(RAGGED, seed=11) + make_batch([40, 96, 161], seed=12, kind="grid")
    small = pald.make_batch_config([(1 << 30, chunks, 32)])
    mixed = pald.make_batch_config([(100, chunks, 32), (1 << 30, chunks, 64)])
    wide = pald.make_batch_config([(1 << 30, chunks, 64)])
    log(f"[batched] 32-wide pass-2 tiles, y_chunks={chunks}")
    _, _, Us, Cs = run_batch(mats, config=small)
    check_all(mats, Us, Cs, what=f"tile 32 y_chunks={chunks}")
    _, _, Um, Cm = run_batch(mats, config=mixed)
    _, _, Uw, Cw = run_batch(mats, config=wide)
    for i in range(len(mats)):
        assert np.array_equal(Us[i], Uw[i]) and np.array_equal(Um[i], Uw[i])
        assert np.array_equal(Cm[i].view(np.int32), Cs[i].view(np.int32)), f"matrix {i}: mixed != tile 32"
        if chunks > 1:
            assert np.array_equal(Cs[i].view(np.int32), Cw[i].view(np.int32)), f"matrix {i}: tile 32 != tile 64"
        else:
            assert_c_close(Cw[i], Cs[i], rtol=2e-6, what=f"matrix {i}: lean tile 64 vs tile 32")


@pytest.mark.parametrize("wpc,lag", [(1, 1), (2, 5), (4, 1)])
def test_grid_and_lag_settings(wpc, lag):
    from paper_2307_16652_amd import pald

    mats = make_batch([90, 7, 200, 64, 150, 33], seed=4)
    cfg = pald.make_batch_config(workgroups_per_cu=wpc, queue_lag=lag)
    _, _, Us, Cs = run_batch(mats, config=cfg)
    check_all(mats, Us, Cs, what=f"wpc={wpc} lag={lag}")


def test_without_u():
    mats = make_batch([50, 120], seed=5)
    _, _, Us, Cs = run_batch(mats, want_u=False)
    assert Us is None
    check_all(mats, None, Cs, what="no U")


def test_matches_single_matrix_path():
    """Batched and single-matrix launches agree to the tolerance (different tilings)."""
    from gpu_helpers import gpu_cohesion

    mats = make_batch([100, 257], seed=6)
    _, _, Us, Cs = run_batch(mats)
    for D, U, C in zip(mats, Us, Cs):
        U1, C1 = gpu_cohesion(D)
        assert np.array_equal(U, U1)
        np.testing.assert_allclose(C, C1, rtol=2e-6, atol=0)


def test_deterministic_and_graph_replays():
    import torch

    from paper_2307_16652_amd import pald

    mats = make_batch([77, 150, 3, 64, 201], seed=7)
    cfg = pald.make_batch_config([(100, 1), (1 << 30, 2)])
    plan = pald.BatchPlan([m.shape[0] for m in mats], config=cfg)
    Dp = torch.from_numpy(np.concatenate([m.reshape(-1) for m in mats])).cuda()
    ws = plan.workspace(Dp.device)
    U1, C1 = plan.run(Dp, ws=ws)
    U1, C1 = U1.clone(), C1.clone()
    U2, C2 = plan.run(Dp, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2) and torch.equal(C1, C2), "two batched runs differ"
    g = plan.graph(Dp)
    for r in range(4):
        g.C.fill_(-1.0)  # eager work between the replays
        g.U.fill_(-1)
        torch.cuda.synchronize()
        Ug, Cg = g.launch()
        torch.cuda.synchronize()
        assert torch.equal(Ug, U1), f"graph replay {r}: U differs"
        assert torch.equal(Cg, C1), f"graph replay {r}: C differs"
        plan.run(Dp, ws=ws)  # eager batched run in between
        torch.cuda.synchronize()
    g.close()
    Us = [u.cpu().numpy() for u in plan.unpack(U1)]
    Cs = [c.cpu().numpy() for c in plan.unpack(C1)]
    check_all(mats, Us, Cs, what="graph")


def test_timestamps():
    import torch

    from paper_2307_16652_amd import pald

    mats = make_batch([60, 130, 90], seed=8)
    cfg = pald.make_batch_config(timestamps=True)
    plan, ws, Us, Cs = run_batch(mats, config=cfg)
    start, end = plan.timestamps(ws)
    assert (start >= 0).all() and (end > start).all() and start.min() == 0
    check_all(mats, Us, Cs, what="timestamps")
    torch.cuda.synchronize()


def test_unaligned_base_pointer():
    """The packed arrays start 4 bytes past an aligned address."""
    import torch

    from paper_2307_16652_amd import pald

    mats = make_batch([36, 64, 100], seed=9)
    plan = pald.BatchPlan([m.shape[0] for m in mats], config=pald.make_batch_config(split_pass1=False))
    flat = np.concatenate([m.reshape(-1) for m in mats])
    buf = torch.zeros(flat.size + 1, dtype=torch.float32, device="cuda")
    buf[1:] = torch.from_numpy(flat).cuda()
    Dp = buf[1:]
    Ub = torch.zeros(flat.size + 1, dtype=torch.int32, device="cuda")
    Cb = torch.zeros(flat.size + 1, dtype=torch.float32, device="cuda")
    Up, Cp = plan.run(Dp, U_packed=Ub[1:], C_packed=Cb[1:])
    torch.cuda.synchronize()
    check_all(mats, [u.cpu().numpy() for u in plan.unpack(Up)], [c.cpu().numpy() for c in plan.unpack(Cp)],
              what="unaligned")


@pytest.mark.parametrize("tile,chunks", [(64, 1), (32, 1), (64, 3)])
def test_split_pass1(tile, chunks):
    """Pass 1 as its own launch of 16 x 16 lanes-over-z tiles: oracle parity on
    ragged and tie-heavy sizes, and U and C bit-identical to the one-launch form
    (the same fl32(1/U) weights and the same pass-2 tile: the general persistent
    kernel in both forms with 32-wide tiles or a y split, the lean kernels --
    batched_pass2_lean_kernel and batched_lean_kernel -- with 64-wide tiles and
    no y split)."""
    from paper_2307_16652_amd import pald

    mats = make_batch(RAGGED, seed=13) + make_batch([4, 40, 96, 161], seed=14, kind="grid")
    buckets = [(100, 1, tile), (1 << 30, chunks, tile)]
    log(f"[batched] split pass 1, tile {tile}, y_chunks {chunks}")
    _, _, Us, Cs = run_batch(mats, config=pald.make_batch_config(buckets, split_pass1=True))
    check_all(mats, Us, Cs, what=f"split tile {tile} y_chunks={chunks}")
    _, _, Uf, Cf = run_batch(mats, config=pald.make_batch_config(buckets))
    for i in range(len(mats)):
        assert np.array_equal(Us[i], Uf[i]), f"matrix {i}: U differs between the modes"
        assert np.array_equal(Cs[i].view(np.int32), Cf[i].view(np.int32)), f"matrix {i}: C differs"


@pytest.mark.parametrize("buckets", [[(100, 1), (1 << 30, 2)], [(1 << 30, 1, 64)]], ids=["general", "lean"])
def test_split_pass1_graph_timestamps_unaligned_no_u(buckets):
    """Split mode: graph replays with eager work between them, timestamps, a packed
    base 4 bytes past an aligned address, and no U output; with a y split (the
    general persistent pass-2 kernel) and without (the lean one)."""
    import torch

    from paper_2307_16652_amd import pald

    mats = make_batch([77, 150, 3, 64, 201, 36], seed=15)
    cfg = pald.make_batch_config(buckets, timestamps=True, split_pass1=True)
    plan = pald.BatchPlan([m.shape[0] for m in mats], config=cfg)
    flat = np.concatenate([m.reshape(-1) for m in mats])
    buf = torch.zeros(flat.size + 1, dtype=torch.float32, device="cuda")
    buf[1:] = torch.from_numpy(flat).cuda()
    Dp = buf[1:]
    ws = plan.workspace(Dp.device)
    U1, C1 = plan.run(Dp, ws=ws)
    U1, C1 = U1.clone(), C1.clone()
    torch.cuda.synchronize()
    start, end = plan.timestamps(ws)
    assert (start >= 0).all() and (end > start).all() and start.min() == 0
    check_all(mats, [u.cpu().numpy() for u in plan.unpack(U1)], [c.cpu().numpy() for c in plan.unpack(C1)],
              what="split unaligned")
    g = plan.graph(Dp)
    for r in range(3):
        g.C.fill_(-1.0)
        g.U.fill_(-1)
        torch.cuda.synchronize()
        Ug, Cg = g.launch()
        torch.cuda.synchronize()
        assert torch.equal(Ug, U1) and torch.equal(Cg, C1), f"split graph replay {r} differs"
        plan.run(Dp, ws=ws)
        torch.cuda.synchronize()
    g.close()
    _, C0 = plan.run(Dp, ws=ws, want_u=False)
    torch.cuda.synchronize()
    assert torch.equal(C0, C1)


def test_cohesion_batched_convenience():
    """pald.cohesion_batched with the autotuner's record read at run time (default)
    and with a NULL config (the library's built-in table, compiled from the same
    record): oracle parity and bit-identical results."""
    import torch

    from paper_2307_16652_amd import pald

    mats = make_batch([70, 3, 129, 40, 1000, 513], seed=16)
    tuned = pald.cohesion_batched([torch.from_numpy(m).cuda() for m in mats])
    plain = pald.cohesion_batched([torch.from_numpy(m).cuda() for m in mats], config=None)
    torch.cuda.synchronize()
    Us = [u.cpu().numpy() for u, _ in tuned]
    Cs = [c.cpu().numpy() for _, c in tuned]
    check_all(mats, Us, Cs, what="cohesion_batched")
    for (u1, c1), (u2, c2) in zip(tuned, plain):
        assert torch.equal(u1, u2) and torch.equal(c1, c2)


def test_config_batch_2000_sampled():
    """The 2000-matrix workload (n uniform in [32, 1024], 2-5 clusters in R^4):
    oracle on every 20th matrix, invariants on all."""
    import time

    t0 = time.time()
    ns = synth.batch_sizes()
    mats = [synth.pairwise_distances(synth.batch_points(i, int(n))) for i, n in enumerate(ns)]
    log(f"[batched] generated 2000 matrices in {time.time() - t0:.1f}s")
    from paper_2307_16652_amd import pald

    _, _, Us, Cs = run_batch(mats, config=None)  # the benchmark's: the library's built-in configuration
    log("[batched] run done; checking")
    err = check_all(mats, Us, Cs, every=20, what="batch2000")
    log(f"[batched] max rel err {err:.3e} over the 100 oracle matrices")
    for i in range(len(mats)):
        check_invariants(Us[i], Cs[i], f"batch2000 matrix {i}")


def test_tuner_timing_helpers():
    """The autotuner's two timing helpers run on the GPU: one batched candidate
    (the 2000-matrix batch, results checked against the first candidate's) and
    one single-matrix evaluation."""
    import torch

    from paper_2307_16652_amd import pald, tune

    dev = torch.device("cuda:0")
    batch = tune.Batch(dev)
    cfg = tune.config_of(pald, [1] * len(tune.BUCKETS), 0, 0, [64] * len(tune.BUCKETS), True)
    ms = batch.time(cfg, 1)
    assert 0.0 < ms < 10_000.0
    assert batch.time(cfg, 1) > 0.0  # the second call compares its results with the first's
    n = 256
    Dg = torch.from_numpy(synth.mixture8d(n=n, seed=7)).to(dev)
    assert tune._time_cohesion(pald, torch, Dg, n, 1, variant="pairwise") > 0.0
