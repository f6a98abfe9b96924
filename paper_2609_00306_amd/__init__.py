"""MI355X-native Cholesky decomposition of two-electron integrals over s-type
Gaussians, with J/K builds and the AO->MO transform of the Cholesky vectors.

Submodules:
  inputs  -- seeded synthetic molecules (no arithmetic of the method)
  build   -- compiles csrc/ into libcd.so for gfx950
  cdlib   -- ctypes binding of include/cd.h (imports torch)
"""
__all__ = ["inputs", "build", "cdlib"]
