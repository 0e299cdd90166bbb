"""pald_cohesion_noalloc (no workspace argument, nothing allocated) against
pald_cohesion on the same inputs: U bit-exact, C within 1e-6 relative and
exactly 0 where pald_cohesion's is 0.  Two calls in a row, the second with a
smaller matrix, since every call shares the library's fixed array."""
import ctypes

import numpy as np
import pytest

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


def _both(D, **opts):
    import torch

    from paper_2307_16652_amd import pald

    Dg = to_gpu(D)
    U1, C1 = pald.cohesion(Dg, variant="pairwise", **opts)
    n = D.shape[0]
    U2 = torch.full((n, n), -7, dtype=torch.int32, device=Dg.device)
    C2 = torch.full((n, n), -7.0, dtype=torch.float32, device=Dg.device)
    pald.cohesion_noalloc(Dg, out_u=U2, out_c=C2, **opts)
    torch.cuda.synchronize()
    return U1.cpu().numpy(), C1.cpu().numpy(), U2.cpu().numpy(), C2.cpu().numpy()


def test_noalloc_matches_cohesion_two_calls():
    # call 1: the n = 4096 six-cluster mixture (the largest n whose default plan fits)
    D = synth.mixture8d(n=4096, seed=2)
    log("[noalloc] call 1: mixture8d n=4096")
    U1, C1, U2, C2 = _both(D)
    assert_u_equal(U2, U1, "noalloc n=4096 U")
    assert_c_close(C2, C1, what="noalloc n=4096 C")
    # same plan (no y split at n = 4096): identical bits
    assert np.array_equal(C2.view(np.uint32), C1.view(np.uint32))
    # call 2: smaller and ragged (n not a multiple of the tile sides); its
    # default y split does not fit the array and is lowered
    D = synth.uniform2d(n=1000, seed=11)
    log("[noalloc] call 2: uniform2d n=1000")
    U1, C1, U2, C2 = _both(D)
    assert_u_equal(U2, U1, "noalloc n=1000 U")
    assert_c_close(C2, C1, what="noalloc n=1000 C")


def test_noalloc_f64_and_no_u():
    import torch

    from paper_2307_16652_amd import pald

    D = synth.mixture8d(n=777, seed=12)
    log("[noalloc] f64 accumulate, U not written, n=777")
    Dg = to_gpu(D)
    _, C1 = pald.cohesion(Dg, variant="pairwise", accum="f64", want_u=False)
    _, C2 = pald.cohesion_noalloc(Dg, accum="f64")
    torch.cuda.synchronize()
    assert_c_close(C2.cpu().numpy(), C1.cpu().numpy(), what="noalloc f64 C")


def test_noalloc_rejects_oversize_and_triplet():
    import torch

    from paper_2307_16652_amd import pald

    lib = pald.load_library()
    n = 4160  # W alone needs 4160 x 4160 x 4 bytes > 64 MiB
    D = torch.zeros((n, n), dtype=torch.float32, device="cuda:0")
    C = torch.empty_like(D)
    o = pald.make_options(variant="pairwise")
    st = lib.pald_cohesion_noalloc(D.data_ptr(), n, n, None, 0, C.data_ptr(), n,
                                   pald._stream_ptr(D.device), ctypes.byref(o))
    assert st == pald.ERR_ARG
    o = pald.make_options(variant="triplet")
    st = lib.pald_cohesion_noalloc(D.data_ptr(), 64, n, None, 0, C.data_ptr(), n,
                                   pald._stream_ptr(D.device), ctypes.byref(o))
    assert st == pald.ERR_UNSUPPORTED
    torch.cuda.synchronize()
