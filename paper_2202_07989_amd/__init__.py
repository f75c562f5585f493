"""MI355X-native entropy-stable adaptive moving-mesh finite-difference path
(Li, Duan & Tang, arXiv 2202.07989).

Submodules:
  inputs  -- seeded synthetic workloads (no step of the scheme)
  es      -- ctypes binding of libes.so, the HIP/gfx950 C-ABI library
Importing the package loads nothing; ``paper_2202_07989_amd.es`` loads the
GPU library and fails loudly when it is missing.
"""
