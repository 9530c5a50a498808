"""Recursive camera painting on MI355X (gfx950): a K-pass per-pixel-camera
ray tracer behind a C ABI (include/rcp.h), with hand-written HIP kernels for
the BVH build, the displaced-ray trace with shading, and the inter-pass ray
compaction.  ``rcp`` is the ctypes binding; importing this package loads
nothing until a function of ``rcp`` is called.
"""
from . import rcp  # noqa: F401

__all__ = ["rcp"]
