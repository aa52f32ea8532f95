"""MRIP on MI355X: Multiple Replications In Parallel with hand-written gfx950
kernels behind a C ABI (include/mrip.h).

  mrip    ctypes binding of libmrip.so (same names as the C ABI)
  inputs  seeded input generators (experimental plans, training designs,
          initial network weights); no arithmetic of the method

Submodules are imported on demand so that importing the package loads
nothing.
"""
__all__ = ["mrip", "inputs"]
