"""MI355X-native FMM-accelerated Global QBX for 2D Helmholtz layer potentials.

Submodules:
  inputs  -- seeded synthetic workloads (no method arithmetic)
  qbx     -- ctypes binding of libqbxfmm.so (host planner + gfx950 kernels)
  build   -- in-tree build of libqbxfmm.so
The binding is imported lazily so that ``inputs`` works without the library.
"""
