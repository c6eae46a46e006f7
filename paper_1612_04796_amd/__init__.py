"""MI355X-native p-multigrid / weighted overlapping Schwarz solver for the
nodal SIPG discretization of the periodic Poisson equation on 3D Cartesian
grids (Stiller, arXiv 1612.04796).

The compute path is a HIP library for gfx950 behind a C ABI
(``include/sipg_mg.h``); ``paper_1612_04796_amd.sipg`` is the thin ctypes
binding with the same entry-point names.  Importing this package does not
load the library; the first call into the binding does, and fails loudly if
the library has not been built.
"""

__all__ = ["sipg", "workloads"]
