"""The large single matrix: n = 65536 points in R^16 (50 anisotropic Gaussians),
D = 17 GB in HBM, full U and C on one GPU.  Oracle on sampled rows; the global
invariants (U symmetric, 2 <= U_xy <= n, sum C = n/2) on everything."""
import time

import numpy as np
import pytest

import oracle
from gpu_helpers import assert_c_close, assert_u_equal
from paper_2307_16652_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 65536
ORACLE_ROWS = 64


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, _ = torch.cuda.mem_get_info()
    if free < 90e9:
        pytest.skip("needs ~90 GB of free device memory")
    from paper_2307_16652_amd import pald

    pald.load_library()


def test_config_aniso16d_n65536(capsys):
    import torch

    from paper_2307_16652_amd import pald

    def log(msg):  # progress on the terminal as it happens (the test runs for minutes)
        with capsys.disabled():
            print(msg, flush=True)

    t0 = time.time()
    P = synth.aniso16d_points(n=N)
    D = synth.pairwise_distances_torch(P, device="cuda")
    torch.cuda.synchronize()
    log(f"[large] generated D ({N}x{N}) on the GPU in {time.time() - t0:.1f}s")
    t0 = time.time()
    U, C = pald.cohesion(D)
    torch.cuda.synchronize()
    log(f"[large] pald_cohesion n={N}: {time.time() - t0:.1f}s")

    # global invariants, in row blocks
    total = 0.0
    blk = 2048
    for r0 in range(0, N, blk):
        r1 = min(N, r0 + blk)
        Ub = U[r0:r1]
        assert torch.equal(Ub, U[:, r0:r1].T), f"U not symmetric in rows {r0}:{r1}"
        off = torch.ones_like(Ub, dtype=torch.bool)
        off[:, r0:r1].fill_diagonal_(False)
        assert int(Ub[off].min()) >= 2 and int(Ub[off].max()) <= N
        Cb = C[r0:r1]
        assert bool((Cb >= 0).all())
        depth = Cb.double().sum(dim=1)
        assert float(depth.max()) <= 1 + 1e-5
        total += float(depth.sum())
    assert abs(total - N / 2) <= 1e-6 * N / 2, f"sum(C) = {total!r}, expected {N / 2}"
    log(f"[large] invariants ok, sum(C) = {total:.6f}")

    # At this size pass 1 runs split over z (4 chunks, atomic counts) by
    # default; the unsplit pass 1 and a 2-chunk split must give the same U.
    # Both tile grids (2^23 tiles of 512 threads) are launched in pieces: one
    # dispatch would overflow the 32-bit work-item count along x and silently
    # skip tiles.
    for zc in (1, 2):
        t0 = time.time()
        U2 = pald.focus_sizes(D, z_chunks=zc)
        torch.cuda.synchronize()
        assert torch.equal(U2, U), f"pass 1 with z_chunks={zc} differs from the default split"
        del U2
        torch.cuda.empty_cache()
        log(f"[large] pass 1 with z_chunks={zc} equal to the default ({time.time() - t0:.1f}s)")

    # oracle rows (the oracle needs all of D on the host)
    rows = np.sort(np.random.default_rng(5).choice(N, size=ORACLE_ROWS, replace=False))
    t0 = time.time()
    Dh = D.cpu().numpy()
    Ug = U[torch.from_numpy(rows).cuda()].cpu().numpy()
    Cg = C[torch.from_numpy(rows).cuda()].cpu().numpy()
    del U, C, D
    torch.cuda.empty_cache()
    parts = []
    for k in range(0, ORACLE_ROWS, 16):
        parts.append(oracle.pald_rows(Dh, rows[k:k + 16]))
        log(f"[large] oracle rows {k + len(rows[k:k + 16])}/{ORACLE_ROWS}: {time.time() - t0:.1f}s")
    Uo = np.concatenate([u for u, _ in parts])
    Co = np.concatenate([c for _, c in parts])
    assert_u_equal(Ug, Uo, "aniso16d n=65536")
    err = assert_c_close(Cg, Co, what="aniso16d n=65536")
    log(f"[large] max rel err {err:.3e}")
