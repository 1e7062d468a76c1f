"""Delayed asynchronous PageRank and Bellman-Ford sweeps on MI355X (gfx950).

The compute path is the HIP library ``libdg.so`` (C ABI in include/dg.h);
``paper_2110_01409_amd.dg`` is its Python binding.  Importing ``dg`` fails
loudly when the library is not built.
"""
__all__ = ["dg"]
