"""Autotuner of the batched mode.

    python -m paper_2307_16652_amd.tune [--out PATH] [--reps 3]
    python -m paper_2307_16652_amd.tune --variants [--out PATH]

Searches, on the 2000-matrix batch (n uniform in [32, 1024], 2-5 Gaussian
clusters in R^4), for

* the pass-2 tile side of each size bucket (64 or 32: the smaller tile pads
  less and repeats less work on diagonal tiles, the larger one reuses each
  staged row over more pairs),
* the pass-2 y-split depth of each size bucket (splitting a large matrix's
  pass-2 tiles over y shortens the items at the end of the queue),
* the persistent grid size (workgroups per CU),
* the queue lag (how far a matrix's pass-2 items trail its pass-1 items), and
* whether pass 1 runs inside the persistent kernel or as a launch of its own
  ahead of it (split mode: 16 x 16 lanes-over-z tiles at 8 waves per SIMD,
  and a queue of pass-2 items only),

by coordinate descent on the measured time of one whole batched launch
(median of `reps` graph replays), and writes the winner to
tuning/batch_gfx950.json.  The next build (paper_2307_16652_amd.build)
compiles that record into the library as its built-in batched configuration
(what a NULL config gets), and `pald.load_tuning()` reads it at run time.
Both tile shapes are compiled into the batched kernel; the search picks one
per bucket.

With --variants it instead times the pairwise, hybrid (triplet pass 1 +
pairwise pass 2), triplet and hybrid2 (pairwise pass 1 + triplet pass 2)
variants of the single-matrix path on Gaussian mixtures of several sizes,
then the pass-2 y split or pass-1 z split of the fastest one, and writes,
per size, the fastest variant and splits to
tuning/variants_gfx950.json, which the next build compiles into the library's
PALD_VARIANT_AUTO choice.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

BUCKETS = (128, 256, 512, 1 << 30)
Y_CHUNKS = (1, 2, 3, 4)
TILES = (64, 32)
LAGS = (1, 2, 4, 8)
WPC = (1, 2)


def log(msg):
    print(f"[tune] {msg}", file=sys.stderr, flush=True)


class Batch:
    def __init__(self, dev, seed: int = 4):
        import torch

        from . import pald, synth

        self.pald = pald
        self.torch = torch
        self.ns = [int(n) for n in synth.batch_sizes(seed=seed)]
        t0 = time.time()
        flat = np.concatenate([synth.pairwise_distances(synth.batch_points(i, n, seed=seed)).reshape(-1)
                               for i, n in enumerate(self.ns)])
        self.D = torch.from_numpy(flat).to(dev)
        log(f"generated {len(self.ns)} matrices in {time.time() - t0:.1f}s")
        self.ref = None

    def time(self, cfg, reps: int) -> float:
        torch, pald = self.torch, self.pald
        plan = pald.BatchPlan(self.ns, config=cfg)
        try:
            ws = plan.workspace(self.D.device)
            U = torch.empty(plan.total, dtype=torch.int32, device=self.D.device)
            C = torch.empty(plan.total, dtype=torch.float32, device=self.D.device)
            plan.run(self.D, U, C, ws)
            g = plan.graph(self.D, U, C, ws)
            g.launch()
            torch.cuda.synchronize()
            if self.ref is None:
                self.ref = (U.clone(), C.clone())
            elif not torch.equal(U, self.ref[0]) or not torch.allclose(C, self.ref[1], rtol=2e-6, atol=0):
                raise RuntimeError("a tuning candidate changed the results")
            times = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                g.launch()
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            g.close()
            return float(np.median(times))
        finally:
            plan.close()


def config_of(pald, chunks, wpc, lag, tiles=None, split=False):
    tiles = tiles or [64] * len(BUCKETS)
    return pald.make_batch_config([(b, c, t) for b, c, t in zip(BUCKETS, chunks, tiles)], workgroups_per_cu=wpc,
                                  queue_lag=lag, split_pass1=split)


def tune(reps: int = 3, out: str | None = None) -> dict:
    import torch

    from . import pald

    pald.load_library()
    dev = torch.device("cuda:0")
    batch = Batch(dev)
    chunks = [1] * len(BUCKETS)
    tiles = [64] * len(BUCKETS)
    wpc, lag, split = 0, 0, False
    best = batch.time(config_of(pald, chunks, wpc, lag, tiles, split), reps)
    log(f"defaults: {best:.3f} ms")
    trials = [{"chunks": list(chunks), "tiles": list(tiles), "wpc": wpc, "lag": lag, "split_pass1": split,
               "ms": best}]

    def consider(c, t, w, l, sp):
        nonlocal best, chunks, tiles, wpc, lag, split
        ms = batch.time(config_of(pald, c, w, l, t, sp), reps)
        trials.append({"chunks": list(c), "tiles": list(t), "wpc": w, "lag": l, "split_pass1": sp, "ms": ms})
        log(f"chunks={c} tiles={t} wpc={w} lag={l} split={sp}: {ms:.3f} ms")
        if ms < best * 0.995:
            best, chunks, tiles, wpc, lag, split = ms, list(c), list(t), w, l, sp

    consider(chunks, tiles, wpc, lag, True)
    for w in WPC:
        for l in (LAGS if not split else (0,)):  # the lag only matters with pass-1 items in the queue
            consider(chunks, tiles, w, l, split)
    for _ in range(2):  # two sweeps of coordinate descent over the buckets
        for b in reversed(range(len(BUCKETS))):
            for tl in TILES:
                if tl != tiles[b]:
                    cand = list(tiles)
                    cand[b] = tl
                    consider(chunks, cand, wpc, lag, split)
            for c in Y_CHUNKS:
                if c != chunks[b]:
                    cand = list(chunks)
                    cand[b] = c
                    consider(cand, tiles, wpc, lag, split)
    result = {
        "arch": "gfx950",
        "workload": "2000 matrices, n uniform in [32, 1024], 2-5 Gaussian clusters in R^4, seed 4",
        "buckets": [{"n_max": b, "y_chunks": c, "tile": t} for b, c, t in zip(BUCKETS, chunks, tiles)],
        "workgroups_per_cu": wpc,
        "queue_lag": lag,
        "split_pass1": split,
        "ms_per_batch": round(best, 3),
        "default_ms_per_batch": round(trials[0]["ms"], 3),
        "trials": trials,
    }
    path = out or pald.TUNING_PATH
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(result, f, indent=1)
    log(f"best {best:.3f} ms -> {path}")
    return result


VARIANT_SIZES = (256, 512, 1024, 2048, 4096, 8192, 16384, 32768)


def _time_cohesion(pald, torch, Dg, n, reps, **opts) -> float:
    """Median milliseconds of pald_cohesion with these options (one warm-up call)."""
    ws = pald.workspace(n, Dg.device, **opts)
    U, C = pald.cohesion(Dg, ws=ws, **opts)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps if n <= 16384 else 1):  # seconds per call above that
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        pald.cohesion(Dg, ws=ws, out_u=U, out_c=C, **opts)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del ws, U, C
    return round(float(np.median(times)), 3)


def tune_variants(reps: int = 3, out: str | None = None) -> dict:
    """Per size: the fastest variant with automatic splits, then the fastest
    pass-2 y split (pairwise, hybrid) or pass-1 z split (pairwise, hybrid2)
    of that variant (0 = the automatic split)."""
    import torch

    from . import pald, synth

    pald.load_library()
    dev = torch.device("cuda:0")
    rows = []
    for n in VARIANT_SIZES:
        Dg = torch.from_numpy(synth.mixture8d(n=n, seed=2)).to(dev)
        ms = {v: _time_cohesion(pald, torch, Dg, n, reps, variant=v)
              for v in ("pairwise", "hybrid", "triplet", "hybrid2")}
        best = min(ms, key=ms.get)
        splits = {"y0_z0": ms[best]}
        if best in ("pairwise", "hybrid"):
            for yc in (1, 2, 4, 8):
                splits[f"y{yc}_z0"] = _time_cohesion(pald, torch, Dg, n, reps, variant=best, y_chunks=yc)
        if best in ("pairwise", "hybrid2"):
            for zc in (1, 2, 4):
                splits[f"y0_z{zc}"] = _time_cohesion(pald, torch, Dg, n, reps, variant=best, z_chunks=zc)
        key = min(splits, key=splits.get)
        yc, zc = (int(t[1:]) for t in key.split("_"))
        log(f"n={n}: {ms} -> {best}; splits {splits} -> y_chunks {yc}, z_chunks {zc}")
        rows.append({"n": n, "ms": ms, "best": best, "split_ms": splits, "y_chunks": yc, "z_chunks": zc})
        del Dg
        torch.cuda.empty_cache()
    result = {"arch": "gfx950", "workload": "mixture8d (6 Gaussian clusters in R^8), seed 2",
              "sizes": rows}
    path = out or pald.VARIANT_TUNING_PATH
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(result, f, indent=1)
    log(f"-> {path}")
    return result


def main():
    ap = argparse.ArgumentParser(description="autotune the batched PaLD mode")
    ap.add_argument("--out", default=None)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--variants", action="store_true", help="choose the single-matrix variant per size instead")
    args = ap.parse_args()
    if args.variants:
        print(json.dumps(tune_variants(args.reps, args.out)))
        return
    r = tune(args.reps, args.out)
    print(json.dumps({k: v for k, v in r.items() if k != "trials"}))


if __name__ == "__main__":
    main()
