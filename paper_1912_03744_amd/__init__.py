"""MI355X (gfx950) ADI solver for the axisymmetric heat equation in a layered
cylinder (Ayriyan & Busa, arXiv 1912.03744), with a batched design-sweep path
and a learned surrogate.

Submodules:
  native     ctypes binding of libadi.so (the C ABI in include/adi.h)
  workloads  seeded synthetic problem parameters
  build      compiles the HIP sources into libadi.so
"""
__all__ = ["native", "workloads", "build"]
