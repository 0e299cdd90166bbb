"""Partitioned local depths (PaLD) on AMD Instinct MI355X (gfx950).

The computation lives in libpald.so (HIP kernels behind the C ABI of
include/pald.h); `paper_2307_16652_amd.pald` is the Python binding and
`paper_2307_16652_amd.synth` the seeded synthetic-input generators.
"""
from . import synth  # noqa: F401

__all__ = ["pald", "synth", "build"]


def __getattr__(name):
    if name in ("pald", "build"):
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
