"""MI355X-native graph traversal kernels (SSSP, BFS, CC) behind a C ABI.

The traversal library is ``libgg.so`` (HIP for gfx950), declared in
``include/gg.h``.  :mod:`paper_1903_01665_amd.gg` is the thin ctypes binding;
:mod:`paper_1903_01665_amd.gen` synthesises seeded input graphs.
"""
__all__ = ["gg", "gen"]
