#!/usr/bin/env python3
"""Throughput of the PaLD hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one full evaluation (pass 1: focus sizes, pass 2: cohesion) of the
n = 16384 integer-grid workload (points uniform in {0..31}^3, squared
Euclidean distances as float32: heavy ties), with D already resident in HBM.

Prints ONE JSON line on stdout.  `value` is triplet comparisons per second in
G/s: 2 n^3 comparison terms per evaluation (one per ordered pair and third
point in each of the two defining sums) divided by the time per step.

`roofline` describes the dominant kernel (pass 2, cohesion: the pairwise
kernel, or the triplet one where the library's tuned choice of variant runs
the pairwise pass 1 with the triplet pass 2), whose launches are timed with
HIP events on the stream they run on.  Its algorithmic work is 4
lane-operations per cohesion term (x, y, z), y != x: the three comparisons
the tie-exact term needs ([t <= a], [t <= b], [t < b] with t = d_xz, a = d_xy,
b = d_zy) and one accumulate -- 4 n^2 (n-1) per step, whichever kernel runs
(the triplet kernel shares one min and three compares among the six terms of
a triple, so it issues fewer lane-ops per term than that count).  The peak is the vector
issue capacity of the chip: 256 CUs x 4 SIMDs x 64 lanes x 2 wave64
instructions per 4 cycles x 2.4 GHz = 78.64 T lane-ops/s (the published
157.3 TFLOP/s float32 vector rate, an FMA counting 2).  `bench.py
--valu-probe` measures what each instruction class actually sustains:
float32 add/mul/fma and simple integer ops issue at about 2.2 cycles per wave
instruction, compares, min/max and selects at about 4.2 (half rate, 39.32 T
lane-ops/s), with float32 additions issuing beside them.  `compare_pipe`
sets the method's comparisons (3 per term) against that half-rate class.
`traffic`, and the issued vector instructions per term, are from rocprofv3
(profiles/<kernel>__grid3d_n16384.json), reported only while the kernel
sources are the ones that were profiled.

`cpu_baseline` is the FP64 oracle on the host cores for a bounded sample of
rows of the same matrix (2 n^2 comparison terms per row).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 16384
SEED = 3
# vector issue capacity: 2 wave64 instructions per SIMD per 4 cycles
VALU_PEAK_TOPS = 256 * 4 * 64 * (2 / 4) * 2.4e9 / 1e12  # 78.64 T lane-ops/s
# compares, min/max, selects: one wave64 instruction per SIMD per 4 cycles
COMPARE_PEAK_TOPS = 256 * 4 * 64 * (1 / 4) * 2.4e9 / 1e12  # 39.32 T lane-ops/s
PASS2_OPS_PER_TERM = 4
PASS2_COMPARES_PER_TERM = 3
# lane-ops per cohesion term of each pass-2 kernel's own block: pairwise, 4
# compares and 4 masked adds per pair and y (2 terms); triplet, a min, 3
# compares, 3 selects and 6 multiply-adds per triple (6 terms)
BLOCK_OPS_PER_TERM = {"pass2_cohesion": 4.0, "triplet_pass2": round(13 / 6, 4)}
# Pass 1 counts 64 z per instruction pair: per (pair, 64 z) one vector min +
# one vector compare and one scalar popcount + one scalar add.  Each pipe
# issues one wave instruction per SIMD every 4 cycles (vector: 64 lanes on
# 16-lane SIMDs; scalar: one unit per CU serving its 4 SIMDs in turn).
PASS1_INSTR_PER_64 = 2
PASS1_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4  # wave instructions/s per pipe


PROFILE_SOURCES = ("paper_2307_16652_amd/csrc/pairwise.hpp", "paper_2307_16652_amd/csrc/pald_api.hip")


def sources_digest(files=PROFILE_SOURCES) -> str:
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_record(record: str):
    """A rocprofv3 counter record from profiles/, or None if absent or if the
    kernel sources changed since it was taken."""
    try:
        with open(os.path.join(ROOT, "profiles", record)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    return rec if rec.get("sources_sha256") == sources_digest(rec.get("sources", PROFILE_SOURCES)) else None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def valu_probe(waves=(8, 4), iters: int = 20000) -> dict:
    """SIMD cycles per wave64 vector instruction of each probe class (libpald_probe.so)."""
    import ctypes

    from paper_2307_16652_amd import build as pald_build

    if not os.path.exists(pald_build.PROBE_LIB):
        pald_build.build_probe()
    lib = ctypes.CDLL(pald_build.PROBE_LIB)
    lib.pald_probe_valu.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.pald_probe_valu.restype = ctypes.c_int32
    names = ["v_add_f32", "v_fma_f32", "v_add_u32", "v_and_b32", "v_min_u32", "v_min_f32", "v_cmp_lt_u32_e64",
             "v_cmp_le_f32_e64", "v_cndmask_b32_e64", "v_addc_co_u32_e64", "v_cmp_lt_u32_e64 + v_add_f32",
             "v_min_u32 + v_add_f32", "v_min_u32 + v_and_b32", "pass-2 block: 16 compares + 16 masked v_add_f32",
             "triplet pass-2 block: 4 triples, 28 min/compare/select + 24 masked v_fmac_f32",
             "v_pk_sub_i16", "v_pk_min_i16", "v_pk_lshrrev_b16", "v_pk_add_u16",
             "rank pass-1 block: 16 pairs, 2 v_pk_sub_i16 + v_pk_min_i16 + v_pk_lshrrev_b16 + v_pk_add_u16 per 2"]
    assert lib.pald_probe_classes() == len(names)
    out = {"unit": "SIMD cycles per wave64 vector instruction (at the measured shader clock)", "classes": {}}
    buf = (ctypes.c_double * 4)()
    for k, name in enumerate(names):
        row = {}
        for w in waves:
            rc = lib.pald_probe_valu(k, w, iters, buf)
            if rc != 0:
                raise RuntimeError(f"pald_probe_valu({k}, {w}) failed: {rc}")
            row[f"{w}_waves_per_simd"] = round(buf[0], 3)
            row[f"clock_ghz_{w}"] = round(buf[1], 3)
        out["classes"][name] = row
        progress(f"probe {name}: {row}")
    return out


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(D: np.ndarray, workload: str = "grid3d", rows_wanted: int = 256):
    """Oracle throughput on the host cores for a seeded sample of rows of D.

    Returns the cpu_baseline record and (rows, U_rows, C_rows) for error checks."""
    import oracle

    n = D.shape[0]
    threads = oracle.default_threads()
    rng = np.random.default_rng(123)
    k = min(n, rows_wanted)
    rows = np.sort(rng.choice(n, size=k, replace=False))
    t0 = time.perf_counter()
    Uo, Co = oracle.pald_rows(D, rows, threads=threads)
    t = time.perf_counter() - t0
    value = k * 2.0 * n * n / t / 1e9
    rec = {
        "value": round(value, 4),
        "unit": "G triplet comparisons/s",
        "cores": threads,
        "cpu": cpu_model(),
        "kind": "oracle",
        "sample": f"{k} seeded random rows of U and C of the n={n} {workload} matrix "
                  f"(2*n^2 terms per row), {t:.1f} s wall",
    }
    return rec, (rows, Uo, Co)


def error_stats(C_rows: np.ndarray, Co: np.ndarray) -> dict:
    """Max / mean relative error of GPU cohesion rows against the oracle's."""
    C_rows = C_rows.astype(np.float64)
    nz = Co != 0
    rel = np.abs(C_rows[nz] - Co[nz]) / np.abs(Co[nz])
    return {"max_rel": float(rel.max()) if rel.size else 0.0,
            "mean_rel": float(rel.mean()) if rel.size else 0.0,
            "exact_zeros_ok": bool((C_rows[~nz] == 0).all())}


def batched_bench(dev, reps: int = 3, one_launch_form: bool = True):
    """The 2000-matrix batch (n uniform in [32, 1024]): one persistent launch per
    batch, replayed from a captured hipGraph, against the same library's
    single-matrix path launched once per matrix on one stream."""
    import torch

    from paper_2307_16652_amd import pald, synth

    ns = synth.batch_sizes()
    progress(f"batched: generating {len(ns)} matrices")
    mats = [synth.pairwise_distances(synth.batch_points(i, int(n))) for i, n in enumerate(ns)]
    # the library's built-in configuration (the autotuner's table compiled into it)
    plan = pald.BatchPlan([int(n) for n in ns], config=None)
    plan_split = bool((pald.batch_queue([int(ns[0])], plan.grid)[1] == 0).all())
    Dp = torch.from_numpy(np.concatenate([m.reshape(-1) for m in mats])).to(dev)
    del mats
    ws = plan.workspace(dev)
    Up = torch.empty(plan.total, dtype=torch.int32, device=dev)
    Cp = torch.empty(plan.total, dtype=torch.float32, device=dev)
    plan.run(Dp, Up, Cp, ws)  # warm-up
    g = plan.graph(Dp, Up, Cp, ws)
    g.launch()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        g.launch()
    ev1.record()
    torch.cuda.synchronize()
    batch_ms = ev0.elapsed_time(ev1) / reps
    g.close()

    def timestamped(one_launch: bool = False):
        """Per-matrix (start, end) device times of one run of the built-in config
        (in the one-launch form if asked)."""
        tcfg = pald.make_batch_config(timestamps=True, split_pass1=False if one_launch else None)
        tplan = pald.BatchPlan([int(n) for n in ns], config=tcfg)
        tws = tplan.workspace(dev)
        tplan.run(Dp, Up, Cp, tws)
        torch.cuda.synchronize()
        st, en = tplan.timestamps(tws)
        tplan.close()
        return st, en

    # per-matrix latency from one run with device timestamps
    start, end = timestamped()
    lat = end - start

    # the one-launch form (pass-1 items in the persistent queue): its time per
    # batch and per-matrix latency, since the split form starts every
    # matrix's pass 1 in the first launch
    fused = None
    if plan_split and one_launch_form:
        fcfg = pald.make_batch_config(split_pass1=False)
        fplan = pald.BatchPlan([int(n) for n in ns], config=fcfg)
        fws = fplan.workspace(dev)
        fplan.run(Dp, Up, Cp, fws)
        fg = fplan.graph(Dp, Up, Cp, fws)
        fg.launch()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            fg.launch()
        ev1.record()
        torch.cuda.synchronize()
        fms = ev0.elapsed_time(ev1) / reps
        fg.close()
        fplan.close()
        del fws
        fst, fen = timestamped(one_launch=True)
        flat_ = fen - fst
        fused = {"ms_per_batch": round(fms, 3), "matrices_per_s": round(len(ns) / (fms / 1e3), 1),
                 "latency_us_p50": round(float(np.percentile(flat_, 50)), 1),
                 "latency_us_p99": round(float(np.percentile(flat_, 99)), 1)}

    # comparator: one single-matrix call per matrix, same stream, no graph
    views = plan.unpack(Dp)
    cviews = plan.unpack(Cp)
    uviews = plan.unpack(Up)
    wsb = max(pald.workspace_bytes(int(n)) for n in set(int(x) for x in ns))
    ws1 = torch.empty(wsb, dtype=torch.uint8, device=dev)
    for D, U, C in zip(views[:50], uviews[:50], cviews[:50]):
        pald.cohesion(D, ws=ws1, out_u=U, out_c=C)
    torch.cuda.synchronize()
    ev0.record()
    for D, U, C in zip(views, uviews, cviews):
        pald.cohesion(D, ws=ws1, out_u=U, out_c=C)
    ev1.record()
    torch.cuda.synchronize()
    loop_ms = ev0.elapsed_time(ev1)
    terms = float((2.0 * ns.astype(np.float64) ** 3).sum())
    plan.close()
    return {
        "workload": "batch: 2000 matrices, n uniform in [32,1024], 2-5 Gaussian clusters in R^4, seed 4",
        "matrices_per_s": round(len(ns) / (batch_ms / 1e3), 1),
        "ms_per_batch": round(batch_ms, 3),
        "triplet_comparisons_G_per_s": round(terms / (batch_ms / 1e3) / 1e9, 1),
        "launch": ("hipGraph replay of one reset kernel, " + ("the pass-1 launch, " if plan_split else "") + "one persistent kernel"),
        "grid_workgroups": plan.grid,
        "per_matrix_launch_ms": round(loop_ms, 3),
        "per_matrix_launch_matrices_per_s": round(len(ns) / (loop_ms / 1e3), 1),
        "speedup_vs_per_matrix_launches": round(loop_ms / batch_ms, 3),
        "latency_us_p50": round(float(np.percentile(lat, 50)), 1),
        "latency_us_p99": round(float(np.percentile(lat, 99)), 1),
        "completion_since_launch_us_p50": round(float(np.percentile(end, 50)), 1),
        "completion_since_launch_us_p99": round(float(np.percentile(end, 99)), 1),
        "one_launch_form": fused,
    }


def variants_bench(dev, reps: int = 3):
    """Pairwise vs hybrid (triplet pass 1 + pairwise pass 2) vs triplet variant on
    the n = 4096 six-cluster mixture in R^8."""
    import torch

    from paper_2307_16652_amd import pald, synth

    n = 4096
    Dg = torch.from_numpy(synth.mixture8d(n=n)).to(dev)
    out = {"workload": "mixture8d n=4096 seed 2"}
    ref = None
    for variant in ("pairwise", "hybrid", "triplet", "hybrid2"):
        ws = pald.workspace(n, dev, variant=variant)
        U, C = pald.cohesion(Dg, variant=variant, ws=ws)
        torch.cuda.synchronize()
        pald.timings_collect()
        t0 = time.perf_counter()
        for _ in range(reps):
            pald.cohesion(Dg, variant=variant, ws=ws, out_u=U, out_c=C, timing=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        kt = pald.timings_collect()
        out[variant] = {"ms_per_step": round(ms, 3),
                        "triplet_comparisons_G_per_s": round(2.0 * n**3 / (ms / 1e3) / 1e9, 1),
                        "kernels_ms": {k: round(v[0] / v[1], 3) for k, v in kt.items()}}
        if ref is None:
            ref = (U.clone(), C.clone())
        elif variant == "hybrid":
            out["hybrid_U_C_identical_to_pairwise"] = bool(torch.equal(U, ref[0]) and torch.equal(C, ref[1]))
        elif variant == "triplet":
            out["triplet_U_equal"] = bool(torch.equal(U, ref[0]))
            rel = ((C.double() - ref[1].double()).abs() / ref[1].double().abs().clamp_min(1e-300))
            rel = torch.where(ref[1] == 0, (C != 0).double(), rel)
            out["triplet_vs_pairwise_max_rel"] = float(rel.max().item())
            ref_t = C.clone()
        else:
            out["hybrid2_U_pairwise_C_triplet_identical"] = bool(torch.equal(U, ref[0]) and torch.equal(C, ref_t))
        del ws
    return out


HBM_PEAK_GBS = 8000.0


def pipeline_bench(dev, n: int, Dg, C, workload: str, reps: int = 3):
    """The steps around the two passes at the benchmark size, each against the HBM
    roofline (8 TB/s) with its algorithmic bytes: the distance front end (writes
    4 n^2 bytes, reads the points), the graph front end on the collaboration-
    network stand-in (writes 4 n^2; also traversed edges/s, n x directed edges
    per evaluation), local depths (reads 4 n^2), the strong-tie count and scan
    (reads 4 n^2) and fill (reads each row up to its last edge, writes 8 bytes
    per edge)."""
    import torch

    from paper_2307_16652_amd import pald, synth

    def timed(fn):
        fn(False)
        torch.cuda.synchronize()
        pald.timings_collect()
        for _ in range(reps):
            fn(True)
        torch.cuda.synchronize()
        return {k: v[0] / v[1] for k, v in pald.timings_collect().items()}

    def hbm(nbytes, ms):
        gbs = nbytes / (ms / 1e3) / 1e9
        return {"ms": round(ms, 4), "bytes": int(nbytes), "GB_per_s": round(gbs, 1),
                "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4)}

    out = {}
    fronts = [("aniso16d_points_dim16_euclidean", synth.aniso16d_points(n=n, seed=5), "euclidean")]
    if workload == "grid3d":
        fronts.insert(0, ("grid3d_points_dim3_sqeuclidean", synth.grid3d_points(n=n, seed=SEED), "sqeuclidean"))
    Dtmp = torch.empty((n, n), dtype=torch.float32, device=dev)
    for name, P, metric in fronts:
        Pg = torch.from_numpy(np.ascontiguousarray(P)).to(dev)
        t = timed(lambda on: pald.distances(Pg, metric, timing=on, out=Dtmp))
        rec = hbm(4.0 * n * n + 8.0 * P.size, t["distances"])
        rec["ops_per_pair_and_dim"] = 2
        if name.startswith("grid3d"):
            rec["equals_benchmark_D"] = bool(torch.equal(Dtmp, Dg))
        out[name] = rec
    rp, colg = synth.collab_graph(n=n)
    rpg = torch.from_numpy(rp).to(dev)
    colgg = torch.from_numpy(colg).to(dev)
    gws = torch.empty(int(pald.load_library().pald_graph_distances_workspace_bytes(n)), dtype=torch.uint8, device=dev)
    t = timed(lambda on: pald.graph_distances(rpg, colgg, n, timing=on, out=Dtmp, ws=gws))
    rec = hbm(4.0 * n * n, t["graph_distances"])
    rec["edges_directed"] = int(rp[-1])
    rec["G_traversed_edges_per_s"] = round(n * float(rp[-1]) / (t["graph_distances"] / 1e3) / 1e9, 1)
    rec["max_finite_hops"] = int(Dtmp[Dtmp < n].max().item())
    out["collab_graph_hop_distances"] = rec
    del Dtmp, gws
    depth = torch.empty(n, dtype=torch.float32, device=dev)
    t = timed(lambda on: pald.local_depths(C, timing=on, out=depth))
    rec = hbm(4.0 * n * n + 4.0 * n, t["local_depths"])
    rec["sum_minus_half_n"] = float(depth.double().sum().item() - n / 2)
    out["local_depths"] = rec
    thr = float(torch.diagonal(C).double().mean().item() / 2)
    t = timed(lambda on: pald.strong_ties(C, thr, timing=on))
    row_ptr, col, val = pald.strong_ties(C, thr)
    nnz = int(row_ptr[-1].item())
    out["strong_ties"] = {"threshold": round(thr, 9), "threshold_rule": "half the mean of diag(C) (an example)",
                          "edges": nnz,
                          "count_scan": hbm(4.0 * n * n + 8.0 * (n + 1), t["strong_ties_count"]),
                          "fill_ms": round(t["strong_ties_fill"], 4)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[1])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=N, help="matrix size (default 16384)")
    ap.add_argument("--workload", default="grid3d", choices=["grid3d", "aniso16d", "mixture8d", "uniform2d"],
                    help="synthetic point cloud (default: the 16384-point integer grid)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 2000-matrix batched measurement")
    ap.add_argument("--no-one-launch-form", action="store_true",
                    help="batched: skip timing the one-launch form beside the tuned split form")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the distance front end, local depths and strong-tie measurements")
    ap.add_argument("--variant", default="auto", choices=["auto", "pairwise", "triplet", "hybrid", "hybrid2"],
                    help="algorithm of the timed step (default: the library's tuned choice for n)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="instead of the benchmark, measure the vector issue rate of each instruction class "
                         "the kernels use and print it as one JSON line")
    ap.add_argument("--valu-probe-waves", default="8,4",
                    help="waves per SIMD the probe classes run at (comma-separated, 1..8)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain elementwise kernel that reads and writes 1 GiB, so a "
                         "counter profile can scale FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rerun with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2307_16652_amd import pald, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if not os.path.exists(pald.LIB_PATH):
        from paper_2307_16652_amd import build as pald_build

        pald_build.build()
    pald.load_library()
    if args.valu_probe:
        waves = tuple(int(w) for w in args.valu_probe_waves.split(","))
        print(json.dumps({"valu_probe": valu_probe(waves)}), flush=True)
        return

    n = args.n
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        progress("copy calibration: one elementwise kernel, 1 GiB read + 1 GiB written")
        del src, dst
    seed = {"grid3d": SEED, "aniso16d": 5, "mixture8d": 2, "uniform2d": 1}[args.workload]
    progress(f"generating {args.workload} n={n} seed={seed}")
    if args.workload == "aniso16d":
        Dg = synth.pairwise_distances_torch(synth.aniso16d_points(n=n, seed=seed), device=dev)
        D = None
    else:
        D = synth.workload(args.workload, n=n, seed=seed)
        Dg = torch.from_numpy(D).to(dev)
    run_variant = pald.resolved_variant(n, variant=args.variant)
    progress(f"variant: {run_variant}")
    ws = pald.workspace(n, dev, variant=args.variant)
    U = torch.empty((n, n), dtype=torch.int32, device=dev)
    C = torch.empty((n, n), dtype=torch.float32, device=dev)

    def step(timing: bool):
        pald.cohesion(Dg, ws=ws, out_u=U, out_c=C, timing=timing, variant=args.variant)

    progress(f"warmup x{args.warmup}")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    pald.timings_collect()  # discard

    progress(f"timing x{args.steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = pald.timings_collect()
    ms_per_step = elapsed / args.steps * 1e3
    terms = 2.0 * n**3
    value = terms / (ms_per_step / 1e3) / 1e9
    progress(f"{ms_per_step:.1f} ms/step, {value:.1f} G/s; kernels {kt}")

    # per-step kernel time (a large grid runs as several launches per step)
    roofline = None
    p2_kind = next((k for k in ("pass2_cohesion", "triplet_pass2") if k in kt), None)
    if p2_kind:
        p2_ms = kt[p2_kind][0] / args.steps
        p2_launches = kt[p2_kind][1] // args.steps
        terms = n * n * (n - 1)
        p2_achieved = PASS2_OPS_PER_TERM * terms / (p2_ms / 1e3) / 1e12
        cmp_achieved = PASS2_COMPARES_PER_TERM * terms / (p2_ms / 1e3) / 1e12
        rec = profile_record(f"{p2_kind}__grid3d_n16384.json") if (n, args.workload) == (N, "grid3d") else None
        # the record holds per-dispatch averages over one step's launches
        issued = rec["valu_insts"] * p2_launches * 64 / terms if rec else None
        roofline = {
            "bound": "alu",
            "achieved": round(p2_achieved, 3),
            "peak": round(VALU_PEAK_TOPS, 3),
            "unit": "T VALU lane-ops/s",
            "frac": round(p2_achieved / VALU_PEAK_TOPS, 4),
            "traffic": rec["traffic_bytes"] * p2_launches if rec else None,
            "traffic_unit": "bytes per step",
            "kernel": p2_kind,
            "kernel_ms": round(p2_ms, 3),
            "launches_per_step": p2_launches,
            "ops_per_term": PASS2_OPS_PER_TERM,
            "kernel_block_lane_ops_per_term": BLOCK_OPS_PER_TERM[p2_kind],
            "issued_lane_ops_per_term": round(issued, 3) if issued else None,
            "useful_fraction": round(PASS2_OPS_PER_TERM / issued, 4) if issued else None,
            "compare_pipe": {"achieved": round(cmp_achieved, 3), "peak": round(COMPARE_PEAK_TOPS, 3),
                             "unit": "T compare lane-ops/s", "frac": round(cmp_achieved / COMPARE_PEAK_TOPS, 4),
                             "compares_per_term": PASS2_COMPARES_PER_TERM},
        }
    p1_ms = kt["pass1_focus"][0] / args.steps if "pass1_focus" in kt else None
    p1_units = (n * (n + 1) / 2) * n  # (pair x <= y, z)
    kernels = {k: round(v[0] / args.steps, 3) for k, v in kt.items()}

    extra = {}
    Cf = None
    if not args.no_comparators:
        progress("comparator: float64-accumulate pass 2")
        Cf = torch.empty_like(C)
        pald.cohesion(Dg, ws=ws, out_u=U, out_c=Cf, accum="f64")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pald.cohesion(Dg, ws=ws, out_u=U, out_c=Cf, accum="f64", timing=True)
        torch.cuda.synchronize()
        t_f64 = time.perf_counter() - t0
        kf = pald.timings_collect()
        diff = (C.double() - Cf.double()).abs() / Cf.double().abs().clamp_min(1e-300)
        diff = torch.where(Cf == 0, (C != 0).double(), diff)
        extra["comparators"] = {
            "f64_accumulate_ms_per_step": round(t_f64 * 1e3, 2),
            "f64_accumulate_pass2_ms": round(kf["pass2_cohesion"][0], 3),
            "compensated_vs_f64_max_rel": float(diff.max().item()),
        }
    if not args.no_comparators:
        extra["variants_n4096"] = variants_bench(dev)
        progress(f"variants: {extra['variants_n4096']}")
    if p1_ms:
        p1_bound_ms = PASS1_INSTR_PER_64 * p1_units / 64 / PASS1_ISSUE_PEAK * 1e3
        extra["pass1_focus"] = {"ms": round(p1_ms, 3), "G_pair_z_per_s": round(p1_units / (p1_ms / 1e3) / 1e9, 1),
                                "issue_bound_ms": round(p1_bound_ms, 3), "issue_frac": round(p1_bound_ms / p1_ms, 4)}
    if not args.no_pipeline:
        progress("pipeline: distances, local depths, strong ties")
        extra["pipeline"] = pipeline_bench(dev, n, Dg, C, args.workload)
        progress(f"pipeline: {extra['pipeline']}")

    base = None
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle rows)")
        base, (rows, Uo, Co) = cpu_baseline(D if D is not None else Dg.cpu().numpy(), args.workload)
        ridx = torch.from_numpy(rows).to(dev)
        err = {"rows": int(rows.size),
               "U_rows_equal": bool(np.array_equal(U[ridx].cpu().numpy(), Uo)),
               "compensated": error_stats(C[ridx].cpu().numpy(), Co)}
        if Cf is not None:
            err["f64_accumulate"] = error_stats(Cf[ridx].cpu().numpy(), Co)
        extra["error_vs_oracle"] = err
        progress(f"error vs oracle: {err}")
    del Cf

    if not args.no_batched:
        del U, C, ws
        torch.cuda.empty_cache()
        extra["batched"] = batched_bench(dev, one_launch_form=not args.no_one_launch_form)
        progress(f"batched: {extra['batched']}")

    out = {
        "metric": f"triplet comparisons/sec (G/s) + % VALU peak, n={n} fp32; batched matrices/sec",
        "value": round(value, 2),
        "unit": "G triplet comparisons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "seed": seed,
                   "points": {"grid3d": "uniform in {0..31}^3",
                              "aniso16d": "50 anisotropic rotated Gaussians in R^16",
                              "mixture8d": "6 Gaussian clusters in R^8, sizes 1:2:...:32",
                              "uniform2d": "uniform in [0,1]^2"}[args.workload],
                   "distance": "squared euclidean (integer, fp32)" if args.workload == "grid3d"
                   else "euclidean (fp32)",
                   "variant": run_variant,
                   "accumulation": "fp32 runs + Kahan partials, "
                   + ("64-bit fixed-point cross-tile sums" if run_variant in ("triplet", "hybrid2")
                      else "fp64 final reduce")},
        "roofline": roofline,
        "cpu_baseline": base,
        "kernels_ms": kernels,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
