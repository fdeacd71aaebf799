"""MI355X (gfx950) immersed-boundary lattice Boltzmann step.

Submodules:
  lbm     ctypes binding of the HIP library's C interface (include/lbm_ib.h)
  inputs  seeded synthetic workloads (geometry, kinematics, frames)
  build   compiles liblbmib.so in-tree for gfx950
"""
