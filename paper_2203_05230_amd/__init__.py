"""MI355X-native implementation of the accurate interface-capturing lattice
Boltzmann step (H. Liang, arXiv:2203.05230).

  lbac       ctypes binding of liblbac.so (C ABI in include/lbac.h)
  workloads  seeded synthetic initial fields and run descriptions
  build      hipcc build of the HIP library for gfx950

Importing the package loads nothing; `lbac.load()` loads the HIP library.
"""
__all__ = ["lbac", "workloads", "build"]
