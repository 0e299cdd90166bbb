"""Builds libpald.so (the gfx950 HIP library behind include/pald.h) in-tree.

    python -m paper_2307_16652_amd.build          # or build() from Python

hipcc cross-compiles for gfx950 without a GPU present.  Every build first
regenerates csrc/tuned_gfx950.h, the built-in tuned tables, from the
autotuner's records in tuning/.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpald.so")
ARCH = os.environ.get("PALD_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # comparisons must see denormal distances exactly: never flush them
    "-fno-gpu-flush-denormals-to-zero",
    # no packed FP32 instructions in the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libpald)")


def sources():
    return [os.path.join(CSRC, f) for f in ("pald_api.hip", "frontend_api.hip")]


PROBE_LIB = os.path.join(PKG, "libpald_probe.so")


TUNING = os.path.join(PKG, "tuning")
TUNED_HEADER = os.path.join(CSRC, "tuned_gfx950.h")
_VARIANT_ENUM = {"pairwise": "PALD_VARIANT_PAIRWISE", "triplet": "PALD_VARIANT_TRIPLET",
                 "hybrid": "PALD_VARIANT_HYBRID", "hybrid2": "PALD_VARIANT_HYBRID2"}


def tuned_header_text() -> str:
    """C++ text of the library's built-in tuned tables, from the autotuner's JSON
    records in tuning/ (batch_gfx950.json: batched buckets, grid, queue lag and
    launch form; variants_gfx950.json: single-matrix variant per size).  A
    missing record gives the untuned defaults."""
    import json

    buckets, wpc, lag, split, src = [{"n_max": 1 << 30, "tile": 64, "y_chunks": 1}], 0, 0, False, []
    path = os.path.join(TUNING, "batch_gfx950.json")
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        buckets = rec["buckets"]
        wpc, lag, split = int(rec.get("workgroups_per_cu", 0)), int(rec.get("queue_lag", 0)), \
            bool(rec.get("split_pass1", False))
        src.append("tuning/batch_gfx950.json")
    variants = [(2, "pairwise", 0, 0)]
    path = os.path.join(TUNING, "variants_gfx950.json")
    if os.path.exists(path):
        with open(path) as f:
            variants = sorted((int(r["n"]), str(r["best"]), int(r.get("y_chunks", 0)), int(r.get("z_chunks", 0)))
                              for r in json.load(f)["sizes"])
        src.append("tuning/variants_gfx950.json")
    if not 1 <= len(buckets) <= 8:
        raise ValueError("the batched tuning record needs 1 to 8 buckets")
    bl = ",\n    ".join(f"{{{int(b['n_max'])}, {int(b.get('tile', 64))}, {int(b.get('y_chunks', 1))}, 0}}"
                         for b in buckets)
    vl = ",\n    ".join(f"{{{n}, {_VARIANT_ENUM[v]}, {yc}, {zc}}}" for n, v, yc, zc in variants)
    return f"""// tuned_gfx950.h -- the library's built-in tuned tables for MI355X (gfx950).
// Written by build.py on every build from the autotuner's records
// ({', '.join(src) or 'none found: untuned defaults'}); do not edit by hand:
// rerun paper_2307_16652_amd.tune, then the build.
#pragma once

#include <stdint.h>

#include "pald.h"

namespace pald_tuned {{

// batched mode: per-size buckets (n_max ascending), persistent grid per CU
// (0 = resident capacity), queue lag (0 = default) and launch form
constexpr pald_batch_bucket kBatchBuckets[] = {{
    {bl}}};
constexpr int32_t kBatchWorkgroupsPerCu = {wpc};
constexpr int32_t kBatchQueueLag = {lag};
constexpr bool kBatchSplitPass1 = {'true' if split else 'false'};

// single-matrix variant for PALD_VARIANT_AUTO, with the pass-2 y split and
// the pass-1 z split it was fastest with (0 = the automatic split): the entry
// with the largest n not above the problem's n (the first entry below that)
struct VariantPick {{
    int64_t n;
    int32_t variant;
    int32_t y_chunks;
    int32_t z_chunks;
}};
constexpr VariantPick kVariants[] = {{
    {vl}}};

}}  // namespace pald_tuned
"""


def write_tuned_header() -> str:
    text = tuned_header_text()
    old = None
    if os.path.exists(TUNED_HEADER):
        with open(TUNED_HEADER) as f:
            old = f.read()
    if old != text:
        with open(TUNED_HEADER, "w") as f:
            f.write(text)
    return TUNED_HEADER


def build(verbose: bool = False) -> str:
    """Compile libpald.so for gfx950; always recompiles."""
    write_tuned_header()
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(ln for ln in res.stdout.splitlines()
                    if "packed-fp32-ops" not in ln and "hip-link" not in ln)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{out}")
    if out.strip() and verbose:
        print(out)
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


def build_probe(verbose: bool = False) -> str:
    """libpald_probe.so: the vector-unit issue-rate probes behind the roofline's
    peak (bench.py --valu-probe); measurement support, not part of the method."""
    tmp = PROBE_LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-o", tmp, os.path.join(CSRC, "valu_probe.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stdout}")
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
