"""The FP64 oracle against facts fixed by the paper and by mathematics (CPU only)."""
import numpy as np
import pytest

import pins


def _oracle(D):
    import oracle

    return oracle.pald(D, threads=2)


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(_oracle)


def test_rows_mode_matches_full():
    """Row-sampled evaluation returns exactly the corresponding rows."""
    import oracle
    from paper_2307_16652_amd import synth

    D = synth.grid3d(n=150, seed=8)
    U, C = oracle.pald(D, threads=3)
    rows = np.array([0, 7, 149, 7, 64])
    Ur, Cr = oracle.pald_rows(D, rows, threads=2)
    assert np.array_equal(Ur, U[rows])
    assert np.array_equal(Cr, C[rows])


def test_thread_count_does_not_change_results():
    import oracle
    from paper_2307_16652_amd import synth

    D = synth.mixture8d(n=90, seed=4)
    U1, C1 = oracle.pald(D, threads=1)
    U5, C5 = oracle.pald(D, threads=5)
    assert np.array_equal(U1, U5) and np.array_equal(C1, C5)


def test_bad_arguments_raise():
    import oracle

    with pytest.raises(ValueError):
        oracle.pald(np.zeros((1, 1), np.float32))
    with pytest.raises(ValueError):
        oracle.pald(np.zeros((2, 3), np.float32))
    with pytest.raises(RuntimeError):
        oracle.pald_rows(np.zeros((3, 3), np.float32), [3])
