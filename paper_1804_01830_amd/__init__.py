"""ddstress: FFT evaluation of dislocation-density stress on MI355X (gfx950).

Berkov & Gorn, arXiv:1804.01830, Sec. 2: the stress of a site-dependent
dislocation density on a rectangular grid of anisotropic cells as a
zero-padded FFT convolution of the density channels with precomputed
interaction coefficients.

Modules:
  binding    ctypes binding of the HIP library (include/ddstress.h)
  workloads  seeded synthetic densities shaped like the paper's workloads
  build      hipcc build of libddstress.so
"""
from . import workloads  # noqa: F401  (no GPU or library needed)

__all__ = ["workloads"]
