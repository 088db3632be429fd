"""Wavelet-tree alternating minimization (AM) for transmission CT on AMD MI355X (gfx950).

The hot path of Degirmenci, O'Sullivan and Politte (arXiv 1508.04458): Haar synthesis of
the active wavelet tree, ray-driven forward projection with Beer's-law means, sign-split
coefficient-domain backprojection with the closed-form AM update, and the adaptive tree
rule, all as HIP kernels behind the C ABI in include/wamct.h (libwamct.so).

  synth    seeded synthetic scans (geometry, phantoms, Poisson counts); no method arithmetic
  api      Context: the C ABI with torch tensors for device memory and streams
"""
from . import synth  # noqa: F401


def __getattr__(name):
    # the HIP binding loads libwamct.so (and torch) only when first used
    if name in ("api", "Context", "validate"):
        import importlib
        api = importlib.import_module(__name__ + ".api")
        return {"api": api, "Context": api.Context, "validate": api.validate}[name]
    raise AttributeError(name)
