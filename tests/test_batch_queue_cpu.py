"""The batched work queue and its dependency protocol, modelled on the CPU.

The queue comes from the library's host-only builder (pald_batch_queue).  A
discrete-event model replays the persistent kernel's protocol -- workers take
items strictly in queue order; a pass-2 item waits until every pass-1 item of
its matrix has finished -- with random item durations and grid sizes, and
checks that every run terminates with every item done once, never running a
pass-2 item before its matrix's pass 1 completed.
"""
import heapq

import numpy as np
import pytest

from paper_2307_16652_amd import pald


def simulate(items, tiles1, workers, rng):
    """Returns (finish time, number of items run). Raises on deadlock or order violation."""
    nmat = len(tiles1)
    done1 = np.zeros(nmat, dtype=np.int64)
    # a matrix whose pass-2 items wait for no pass-1 item had its pass 1 done
    # before the persistent launch (split mode)
    p1_finished_at = [0.0 if tiles1[m] == 0 else None for m in range(nmat)]
    head = 0
    t = 0.0
    running = []  # (finish_time, worker, item index)
    waiting = {}  # worker -> item index (pass-2 item waiting for its matrix)
    idle = list(range(workers))
    ran = 0
    seen = set()
    while True:
        # idle workers take the next item
        while idle and head < len(items):
            w = idle.pop()
            k = head
            head += 1
            m, kind, tile, chunk = (int(v) for v in items[k])
            key = (m, kind, tile, chunk)
            assert key not in seen, f"item {key} queued twice"
            seen.add(key)
            if kind == 1 and done1[m] < tiles1[m]:
                waiting[w] = k
            else:
                heapq.heappush(running, (t + rng.exponential(1.0 + m % 3), w, k))
        if not running:
            if waiting:
                raise AssertionError(f"deadlock: {len(waiting)} workers wait with nothing running")
            break
        t, w, k = heapq.heappop(running)
        m, kind = int(items[k][0]), int(items[k][1])
        ran += 1
        if kind == 0:
            done1[m] += 1
            if done1[m] == tiles1[m]:
                p1_finished_at[m] = t
                for ww, kk in list(waiting.items()):
                    if int(items[kk][0]) == m:
                        del waiting[ww]
                        heapq.heappush(running, (t + rng.exponential(1.0), ww, kk))
        else:
            assert p1_finished_at[m] is not None and p1_finished_at[m] <= t, "pass-2 item ran before pass 1"
        idle.append(w)
    return t, ran


SIZE_MIXES = {
    "tiny": [2, 3, 5, 7],
    "ragged": [2, 33, 64, 65, 100, 129, 257, 31, 1000],
    "batch_like": list(np.random.default_rng(4).integers(32, 1025, size=300)),
}


@pytest.mark.parametrize("mix", sorted(SIZE_MIXES))
@pytest.mark.parametrize("grid", [1, 3, 64, 512])
def test_queue_structure(mix, grid):
    sizes = SIZE_MIXES[mix]
    items, tiles1 = pald.batch_queue(sizes, grid, config=pald.make_batch_config(split_pass1=False))
    for m, n in enumerate(sizes):
        nb1 = -(-n // 64)
        assert tiles1[m] == nb1 * (nb1 + 1) // 2
        mine = items[items[:, 0] == m]
        kinds = mine[:, 1]
        assert (kinds == 0).sum() == tiles1[m]
        pos = np.where(items[:, 0] == m)[0]
        last_p1 = pos[kinds == 0].max()
        first_p2 = pos[kinds == 1].min()
        assert last_p1 < first_p2, "a pass-2 item precedes a pass-1 item of the same matrix"
        nb2 = -(-n // 64)
        assert (kinds == 1).sum() == nb2 * (nb2 + 1) // 2  # default: no y split
    keys = {tuple(r) for r in items.tolist()}
    assert len(keys) == len(items)


@pytest.mark.parametrize("mix", sorted(SIZE_MIXES))
@pytest.mark.parametrize("workers", [1, 2, 7, 64])
def test_protocol_terminates(mix, workers):
    sizes = SIZE_MIXES[mix]
    rng = np.random.default_rng(workers)
    cfg = pald.make_batch_config([(128, 1), (1 << 30, 3)])
    items, tiles1 = pald.batch_queue(sizes, grid=max(workers, 1), config=cfg)
    for _ in range(3):
        _, ran = simulate(items, tiles1, workers, rng)
        assert ran == len(items)


def test_model_detects_a_bad_queue():
    """Control: moving a pass-2 item ahead of its matrix's pass 1 deadlocks one worker."""
    items, tiles1 = pald.batch_queue([70, 40], grid=1, config=pald.make_batch_config(split_pass1=False))
    bad = items.copy()
    k = int(np.where((bad[:, 1] == 1) & (bad[:, 0] == 0))[0][0])
    bad = np.concatenate([bad[k:k + 1], np.delete(bad, k, axis=0)])
    with pytest.raises(AssertionError, match="deadlock"):
        simulate(bad, tiles1, 1, np.random.default_rng(0))


@pytest.mark.parametrize("tile", [32, 64])
def test_pass2_tile_side_per_bucket(tile):
    sizes = [2, 31, 32, 33, 100, 300, 1000]
    cfg = pald.make_batch_config([(64, 1, 32), (1 << 30, 2, tile)])
    items, tiles1 = pald.batch_queue(sizes, grid=16, config=cfg)
    for m, n in enumerate(sizes):
        t2, ch = (32, 1) if n <= 64 else (tile, 2)
        nb1, nb2 = -(-n // 64), -(-n // t2)
        assert tiles1[m] == nb1 * (nb1 + 1) // 2  # pass-1 tiles stay 64 wide
        mine = items[(items[:, 0] == m) & (items[:, 1] == 1)]
        ch = min(ch, -(-n // 12))
        assert len(mine) == nb2 * (nb2 + 1) // 2 * len(set(mine[:, 3].tolist()))
        assert mine[:, 2].max() == nb2 * (nb2 + 1) // 2 - 1
    rng = np.random.default_rng(3)
    _, ran = simulate(items, tiles1, 5, rng)
    assert ran == len(items)


@pytest.mark.parametrize("mix", sorted(SIZE_MIXES))
def test_split_pass1_queue(mix):
    """With pass 1 split into its own launch the queue holds every pass-2 item once,
    largest matrices first, and no item waits (every pass-1 count is 0)."""
    sizes = SIZE_MIXES[mix]
    cfg = pald.make_batch_config([(128, 1), (1 << 30, 3)], split_pass1=True)
    items, tiles1 = pald.batch_queue(sizes, grid=64, config=cfg)
    fused, _ = pald.batch_queue(sizes, grid=64, config=pald.make_batch_config([(128, 1), (1 << 30, 3)]))
    assert (items[:, 1] == 1).all() and (tiles1 == 0).all()
    assert {tuple(r) for r in items.tolist()} == {tuple(r) for r in fused[fused[:, 1] == 1].tolist()}
    assert len({tuple(r) for r in items.tolist()}) == len(items)
    order = [sizes[m] for m in items[:, 0]]
    assert all(a >= b for a, b in zip(order, order[1:])), "not largest matrix first"
    _, ran = simulate(items, tiles1, 7, np.random.default_rng(5))
    assert ran == len(items)


def test_y_split_items():
    cfg = pald.make_batch_config([(100, 1), (1 << 30, 4)])
    items, _ = pald.batch_queue([90, 300], grid=8, config=cfg)
    m1 = items[(items[:, 0] == 1) & (items[:, 1] == 1)]
    nb2 = -(-300 // 64)
    assert len(m1) == nb2 * (nb2 + 1) // 2 * 4
    assert set(m1[:, 3].tolist()) == {0, 1, 2, 3}
    m0 = items[(items[:, 0] == 0) & (items[:, 1] == 1)]
    assert set(m0[:, 3].tolist()) == {0}


def test_bad_batch_arguments():
    with pytest.raises(pald.PaldError):
        pald.batch_queue([], grid=4)
    with pytest.raises(pald.PaldError):
        pald.batch_queue([1, 5], grid=4)
    bad = pald.make_batch_config([(100, 1), (50, 1)])  # not ascending
    with pytest.raises(pald.PaldError):
        pald.batch_queue([10], grid=4, config=bad)
    bad = pald.make_batch_config([(100, 0)])
    with pytest.raises(pald.PaldError):
        pald.batch_queue([10], grid=4, config=bad)
    bad = pald.make_batch_config([(100, 1, 48)])  # only 64- and 32-wide pass-2 tiles exist
    with pytest.raises(pald.PaldError):
        pald.batch_queue([10], grid=4, config=bad)


def test_tuning_table_loads_into_a_valid_config():
    """The autotuner's table (if present) parses and the host queue builder accepts it."""
    import os

    cfg = pald.load_tuning()
    if not os.path.exists(pald.TUNING_PATH):
        assert cfg is None
        return
    assert cfg is not None and 1 <= cfg.nbuckets <= pald.BATCH_MAX_BUCKETS
    items, tiles1 = pald.batch_queue([40, 300, 1000], grid=512, config=cfg)
    split = bool(cfg.flags & pald.BATCH_SPLIT_PASS1)
    assert len(items) > 0 and ((tiles1 == 0).all() if split else (tiles1 > 0).all())
    tcfg = pald.load_tuning(timestamps=True)
    assert tcfg.flags == pald.BATCH_TIMESTAMPS | (pald.BATCH_SPLIT_PASS1 if split else pald.BATCH_ONE_LAUNCH)


def test_builtin_config_is_the_tuned_table():
    """A NULL config (and a config with every field 0) gives the queue of the autotuner's
    record, compiled into the library: with the split form on gfx950, no matrix has
    pass-1 items in the persistent queue."""
    import json
    import os

    sizes = SIZE_MIXES["batch_like"]
    with open(pald.TUNING_PATH) as f:
        rec = json.load(f)
    tuned = pald.load_tuning()
    for grid in (64, 1024):
        items0, tiles0 = pald.batch_queue(sizes, grid)  # NULL config
        items1, tiles1 = pald.batch_queue(sizes, grid, config=tuned)
        items2, tiles2 = pald.batch_queue(sizes, grid, config=pald.make_batch_config(split_pass1=None))
        assert np.array_equal(items0, items1) and np.array_equal(tiles0, tiles1)
        assert np.array_equal(items0, items2) and np.array_equal(tiles0, tiles2)
        if rec.get("split_pass1"):
            assert (tiles0 == 0).all()
            assert (items0[:, 1] == 1).all()
    assert os.path.exists(pald.TUNING_PATH)


def test_launch_form_flags():
    sizes = [40, 300]
    one = pald.make_batch_config(split_pass1=False)
    split = pald.make_batch_config(split_pass1=True)
    _, t_one = pald.batch_queue(sizes, 8, config=one)
    _, t_split = pald.batch_queue(sizes, 8, config=split)
    assert (t_one > 0).all() and (t_split == 0).all()
    both = pald.make_batch_config()
    both.flags = pald.BATCH_SPLIT_PASS1 | pald.BATCH_ONE_LAUNCH
    with pytest.raises(pald.PaldError):
        pald.batch_queue(sizes, 8, config=both)


def test_generated_tuned_header_matches_the_records():
    """csrc/tuned_gfx950.h is what build.py writes from the tuning records."""
    from paper_2307_16652_amd import build

    with open(build.TUNED_HEADER) as f:
        assert f.read() == build.tuned_header_text()
