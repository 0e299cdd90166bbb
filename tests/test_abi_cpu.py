"""The C ABI without a GPU: the library loads, exports every declared symbol,
and rejects bad arguments synchronously before any device work (CPU only)."""
import ctypes
import os
import re

import pytest

from paper_2307_16652_amd import pald

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pald.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pald_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_what_the_binding_expects():
    assert declared_functions() == sorted(pald.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pald.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, f"missing exports: {missing}"


def test_status_strings_and_version():
    lib = pald.load_library()
    assert lib.pald_status_string(0) == b"ok"
    assert lib.pald_status_string(99) == b"unknown status"
    assert lib.pald_version() >= 100


def test_workspace_sizes():
    assert pald.workspace_bytes(1) == 0
    small = pald.workspace_bytes(100)
    big = pald.workspace_bytes(16384)
    assert small >= 100 * 100 * 4 and big >= 16384 * 16384 * 4
    assert big % 256 == 0
    # a forced y split needs float64 partials
    assert pald.workspace_bytes(1000, y_chunks=4) >= 4 * 1000 * 1000 * 8


def test_auto_variant_follows_the_tuned_table():
    """PALD_VARIANT_AUTO sizes its workspace for the variant the autotuner's record
    (compiled into the library) picks at each n."""
    import json

    with open(pald.VARIANT_TUNING_PATH) as f:
        table = sorted((int(r["n"]), r["best"], int(r.get("y_chunks", 0)), int(r.get("z_chunks", 0)))
                       for r in json.load(f)["sizes"])
    for n in (100, 256, 300, 1024, 3000, 5000, 20000, 40000):
        pick = table[0]
        for row in table:
            if row[0] <= n:
                pick = row
        _, v, yc, zc = pick
        # AUTO takes the tuned variant and, with both splits left automatic, its splits
        assert pald.workspace_bytes(n, variant="auto") == \
            pald.workspace_bytes(n, variant=v, y_chunks=yc, z_chunks=zc), n
        assert pald.resolved_variant(n) == v, n
        assert pald.resolved_variant(n, variant="triplet") == "triplet"
    assert pald.load_library().pald_resolved_variant(100, ctypes.byref(pald.make_options(accum="f64"))) in (1, 3)
    bad = pald.make_options()
    bad.variant = 9
    assert pald.load_library().pald_resolved_variant(100, ctypes.byref(bad)) == -1
    # the triplet variant takes no forced split: AUTO with one runs pairwise
    assert pald.workspace_bytes(3000, variant="auto", y_chunks=2) == \
        pald.workspace_bytes(3000, variant="pairwise", y_chunks=2)


def _opts(**kw):
    return ctypes.byref(pald.make_options(**kw))


@pytest.mark.parametrize("n,ldd,ldc", [(1, 1, 1), (0, 4, 4), (8, 7, 8), (8, 8, 7)])
def test_cohesion_bad_sizes(n, ldd, ldc):
    lib = pald.load_library()
    fake = ctypes.c_void_p(0x10000)
    st = lib.pald_cohesion(fake, n, ldd, None, 0, fake, ldc, fake, 1 << 20, None, _opts())
    assert st == pald.ERR_ARG


def test_cohesion_null_pointers_and_small_workspace():
    lib = pald.load_library()
    fake = ctypes.c_void_p(0x10000)
    assert lib.pald_cohesion(None, 8, 8, None, 0, fake, 8, fake, 1 << 20, None, _opts()) == pald.ERR_ARG
    assert lib.pald_cohesion(fake, 8, 8, None, 0, None, 8, fake, 1 << 20, None, _opts()) == pald.ERR_ARG
    assert lib.pald_cohesion(fake, 8, 8, None, 0, fake, 8, None, 1 << 20, None, _opts()) == pald.ERR_ARG
    assert lib.pald_cohesion(fake, 8, 8, None, 0, fake, 8, fake, 16, None, _opts()) == pald.ERR_ARG
    # misaligned workspace
    assert lib.pald_cohesion(fake, 8, 8, None, 0, fake, 8, ctypes.c_void_p(0x10004), 1 << 20, None,
                             _opts()) == pald.ERR_ARG
    # U given with a too-small leading dimension
    assert lib.pald_cohesion(fake, 8, 8, fake, 4, fake, 8, fake, 1 << 20, None, _opts()) == pald.ERR_ARG


def test_unknown_options_rejected():
    lib = pald.load_library()
    fake = ctypes.c_void_p(0x10000)
    o = pald.make_options()
    o.reserved[1] = 3
    assert lib.pald_cohesion(fake, 8, 8, None, 0, fake, 8, fake, 1 << 20, None, ctypes.byref(o)) == \
        pald.ERR_UNSUPPORTED
    o = pald.make_options()
    o.accum = 7
    assert lib.pald_cohesion(fake, 8, 8, None, 0, fake, 8, fake, 1 << 20, None, ctypes.byref(o)) == \
        pald.ERR_UNSUPPORTED
    o = pald.make_options()
    o.flags = 0x80
    assert lib.pald_focus_sizes(fake, 8, 8, fake, 8, None, ctypes.byref(o)) == pald.ERR_UNSUPPORTED
    # the triplet pass 2's fixed-point sums are exact up to n = 2^18 only
    big = (1 << 18) + 1
    for v in ("triplet", "hybrid2"):
        assert lib.pald_cohesion(fake, big, big, None, 0, fake, big, fake, 1 << 62, None,
                                 _opts(variant=v)) == pald.ERR_UNSUPPORTED
    # hybrid2: the triplet pass 2 takes no y split and no float64 form; the triplet
    # variant takes no z split either
    for kw in (dict(variant="hybrid2", y_chunks=2), dict(variant="hybrid2", accum="f64"),
               dict(variant="triplet", z_chunks=2)):
        assert lib.pald_cohesion(fake, 8, 8, None, 0, fake, 8, fake, 1 << 20, None, _opts(**kw)) == \
            pald.ERR_UNSUPPORTED, kw
    o = pald.make_options()
    o.variant = 5
    assert lib.pald_cohesion(fake, 8, 8, None, 0, fake, 8, fake, 1 << 20, None, ctypes.byref(o)) == \
        pald.ERR_UNSUPPORTED
    # hybrid2 needs the triplet workspace (A, B, W and U scratch)
    assert pald.workspace_bytes(1000, variant="hybrid2") == pald.workspace_bytes(1000, variant="triplet")
    o = pald.make_options()
    o.y_chunks = -1
    assert lib.pald_workspace_bytes(8, ctypes.byref(o)) == 0


def test_focus_sizes_and_check_input_bad_args():
    lib = pald.load_library()
    fake = ctypes.c_void_p(0x10000)
    assert lib.pald_focus_sizes(None, 8, 8, fake, 8, None, None) == pald.ERR_ARG
    assert lib.pald_focus_sizes(fake, 8, 8, None, 8, None, None) == pald.ERR_ARG
    assert lib.pald_focus_sizes(fake, 8, 8, fake, 7, None, None) == pald.ERR_ARG
    assert lib.pald_check_input(fake, 8, 8, fake, 8, None, None) == pald.ERR_ARG
    assert lib.pald_check_input(fake, 1, 1, fake, 256, None, None) == pald.ERR_ARG


def test_rows_and_ooc_argument_errors():
    lib = pald.load_library()
    fake = ctypes.c_void_p(0x10000)
    assert lib.pald_rows_workspace_bytes(100, 0, None) == 0
    assert lib.pald_rows_workspace_bytes(100, 101, None) == 0
    assert lib.pald_rows_workspace_bytes(100, 10, None) >= 100 * 64 * 4
    assert lib.pald_rows_workspace_bytes(100, 10, _opts(accum="f64")) == 0
    ws = lib.pald_rows_workspace_bytes(100, 10, None)
    ok = dict(D=fake, n=100, ldd=100, x0=0, x1=10, U=None, ldu=0, C=fake, ldc=100, ws=fake, ws_bytes=ws)

    def call(opt=None, **kw):
        a = dict(ok, **kw)
        return lib.pald_cohesion_rows(a["D"], a["n"], a["ldd"], a["x0"], a["x1"], a["U"], a["ldu"], a["C"],
                                      a["ldc"], a["ws"], a["ws_bytes"], None, opt)

    assert call(D=None) == pald.ERR_ARG
    assert call(C=None) == pald.ERR_ARG
    assert call(x0=-1) == pald.ERR_ARG
    assert call(x0=10, x1=10) == pald.ERR_ARG
    assert call(x1=101) == pald.ERR_ARG
    assert call(ldd=99) == pald.ERR_ARG
    assert call(U=fake, ldu=99) == pald.ERR_ARG
    assert call(ws_bytes=ws - 1) == pald.ERR_ARG
    assert call(ws=ctypes.c_void_p(0x10004)) == pald.ERR_ARG
    assert call(opt=_opts(variant="triplet")) == pald.ERR_UNSUPPORTED
    assert call(opt=_opts(y_chunks=2)) == pald.ERR_UNSUPPORTED
    # out of core: the panel must fit the workspace
    small = lib.pald_ooc_workspace_bytes(100, 16)
    assert small > 0 and lib.pald_ooc_workspace_bytes(100, 32) > small
    assert lib.pald_ooc_workspace_bytes(100, 1000) == lib.pald_ooc_workspace_bytes(100, 100)
    assert lib.pald_cohesion_ooc(fake, 100, 100, None, 0, fake, 100, fake, small - 1, None, None) == pald.ERR_ARG
    assert lib.pald_cohesion_ooc(None, 100, 100, None, 0, fake, 100, fake, small, None, None) == pald.ERR_ARG
    assert lib.pald_cohesion_ooc(fake, 100, 99, None, 0, fake, 100, fake, small, None, None) == pald.ERR_ARG
    assert lib.pald_cohesion_ooc(fake, 100, 100, None, 0, fake, 100, fake, small, None,
                                 _opts(accum="f64")) == pald.ERR_UNSUPPORTED


def test_timings_collect_without_records():
    lib = pald.load_library()
    k = len(pald.TIMING_KINDS)
    tot = (ctypes.c_double * k)()
    cnt = (ctypes.c_int64 * k)()
    assert lib.pald_timings_collect(tot, cnt, k) == k == 16
    assert list(cnt) == [0] * k


def test_front_end_and_analysis_argument_errors():
    lib = pald.load_library()
    f = ctypes.c_void_p(0x10000)
    # distances: P, dtype, n, dim, ldp, metric, D, ldd, stream, flags
    assert lib.pald_distances(None, 0, 8, 3, 3, 0, f, 8, None, 0) == pald.ERR_ARG
    assert lib.pald_distances(f, 0, 8, 3, 3, 0, None, 8, None, 0) == pald.ERR_ARG
    assert lib.pald_distances(f, 0, 0, 3, 3, 0, f, 8, None, 0) == pald.ERR_ARG
    assert lib.pald_distances(f, 0, 8, 0, 3, 0, f, 8, None, 0) == pald.ERR_ARG
    assert lib.pald_distances(f, 0, 8, 3, 2, 0, f, 8, None, 0) == pald.ERR_ARG
    assert lib.pald_distances(f, 0, 8, 3, 3, 0, f, 7, None, 0) == pald.ERR_ARG
    assert lib.pald_distances(f, 2, 8, 3, 3, 0, f, 8, None, 0) == pald.ERR_UNSUPPORTED
    assert lib.pald_distances(f, 0, 8, 3, 3, 2, f, 8, None, 0) == pald.ERR_UNSUPPORTED
    assert lib.pald_distances(f, 0, 8, 3, 3, 0, f, 8, None, 2) == pald.ERR_UNSUPPORTED
    # local depths: C, n, ldc, depth, stream, flags
    assert lib.pald_local_depths(None, 8, 8, f, None, 0) == pald.ERR_ARG
    assert lib.pald_local_depths(f, 8, 8, None, None, 0) == pald.ERR_ARG
    assert lib.pald_local_depths(f, 8, 7, f, None, 0) == pald.ERR_ARG
    assert lib.pald_local_depths(f, 0, 8, f, None, 0) == pald.ERR_ARG
    assert lib.pald_local_depths(f, 8, 8, f, None, 4) == pald.ERR_UNSUPPORTED
    # strong ties: C, n, ldc, threshold, row_ptr, col, val, cap, stream, flags
    assert lib.pald_strong_ties(None, 8, 8, 0.5, f, f, None, 4, None, 0) == pald.ERR_ARG
    assert lib.pald_strong_ties(f, 8, 8, 0.5, None, f, None, 4, None, 0) == pald.ERR_ARG
    assert lib.pald_strong_ties(f, 8, 8, 0.5, f, None, None, 4, None, 0) == pald.ERR_ARG
    assert lib.pald_strong_ties(f, 8, 8, 0.5, f, f, None, -1, None, 0) == pald.ERR_ARG
    assert lib.pald_strong_ties(f, 8, 7, 0.5, f, f, None, 4, None, 0) == pald.ERR_ARG
    assert lib.pald_strong_ties(f, 8, 8, float("nan"), f, f, None, 4, None, 0) == pald.ERR_ARG
    assert lib.pald_strong_ties(f, 8, 8, 0.5, f, f, None, 4, None, 8) == pald.ERR_UNSUPPORTED


def test_graph_distances_argument_errors():
    lib = pald.load_library()
    f = ctypes.c_void_p(0x10000)
    ws = 24 * 8
    assert lib.pald_graph_distances_workspace_bytes(0) == 0
    assert lib.pald_graph_distances_workspace_bytes(64) >= 24 * 64
    # row_ptr, col, nnz, n, D, ldd, ws, ws_bytes, stream, flags
    assert lib.pald_graph_distances(None, f, 4, 8, f, 8, f, ws, None, 0) == pald.ERR_ARG
    assert lib.pald_graph_distances(f, None, 4, 8, f, 8, f, ws, None, 0) == pald.ERR_ARG
    assert lib.pald_graph_distances(f, f, 4, 8, None, 8, f, ws, None, 0) == pald.ERR_ARG
    assert lib.pald_graph_distances(f, f, 4, 8, f, 8, None, ws, None, 0) == pald.ERR_ARG
    assert lib.pald_graph_distances(f, f, -1, 8, f, 8, f, ws, None, 0) == pald.ERR_ARG
    assert lib.pald_graph_distances(f, f, 4, 0, f, 8, f, ws, None, 0) == pald.ERR_ARG
    assert lib.pald_graph_distances(f, f, 4, 8, f, 7, f, ws, None, 0) == pald.ERR_ARG
    assert lib.pald_graph_distances(f, f, 4, 8, f, 8, f, ws - 8, None, 0) == pald.ERR_ARG
    assert lib.pald_graph_distances(f, f, 4, 8, f, 8, ctypes.c_void_p(0x10004), ws, None, 0) == pald.ERR_ARG
    assert lib.pald_graph_distances(f, f, 4, 8, f, 8, f, ws, None, 2) == pald.ERR_UNSUPPORTED


def test_header_is_plain_c_and_links(tmp_path):
    """include/pald.h compiles as C99 with warnings as errors, and a C program
    links against libpald.so and calls the host-only entry points."""
    import subprocess

    src = tmp_path / "use_pald.c"
    src.write_text(r"""
#include <stdio.h>
#include <string.h>
#include "pald.h"
int main(void) {
    pald_options opt;
    memset(&opt, 0, sizeof opt);
    opt.variant = PALD_VARIANT_PAIRWISE;
    opt.accum = PALD_ACC_COMPENSATED;
    if (pald_version() < 100) return 1;
    if (strcmp(pald_status_string(PALD_ERR_ARG), "invalid argument") != 0) return 2;
    if (pald_workspace_bytes(1000, &opt) < 1000u * 1000u * 4u) return 3;
    if (pald_focus_sizes(NULL, 8, 8, NULL, 8, NULL, &opt) != PALD_ERR_ARG) return 4;
    int64_t n[3] = {40, 300, 2};
    int32_t items[4 * 64];
    int32_t tiles1[3];
    if (pald_batch_queue(3, n, NULL, 4, items, 64, tiles1) <= 0) return 5;
    printf("ok\n");
    return 0;
}
""")
    exe = tmp_path / "use_pald"
    lib_dir = os.path.dirname(pald.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                           str(src), "-o", str(exe), "-L", lib_dir, "-lpald", f"-Wl,-rpath,{lib_dir}"])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", (out.returncode, out.stdout, out.stderr)
