"""MI355X-native conservative phase-field lattice Boltzmann hot path (arXiv 2505.12205).

Submodules:
  workloads -- seeded synthetic workloads (parameters and initial fields)
  lbm       -- ctypes binding of the HIP C-ABI library (liblbm.so)
  build     -- hipcc build of the library for gfx950

Importing the package loads nothing; ``paper_2505_12205_amd.lbm`` loads the
HIP library and fails loudly if it is missing.
"""
