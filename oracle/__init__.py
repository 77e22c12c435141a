"""Plain FP64 CPU oracle for the FFT stress evaluation of Berkov & Gorn,
"Dislocation-induced stress in polycrystalline materials: mesoscopic
simulations in the dislocation density formalism" (arXiv:1804.01830).

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or run it. The product
path (the HIP library and its binding) never imports it, and it imports nothing
from the product path: the two share no code. The only module both sides use is
the seeded input generator ``paper_1804_01830_amd.workloads``, which holds none
of the method's arithmetic; the oracle does not import even that (tests pass its
output in).

What the oracle computes, in the paper's order:

* ``segment``: stress of a finite straight dislocation segment,
  Eq. (4a)-(4c) with Eq. (5) for a line along z (Sec. 2.2), and the
  coordinate-free Eq. (6)-(7) for any line direction (Sec. 2.2).
* ``kernel``: interaction coefficients K_{v,c}(Delta) = Delta V * f_v with
  f = sigma^AB / (Delta l * b) (Eq. 9b), subdivision of near cells into
  near-cubic subcells (Sec. 2.3, Fig. 3), zero self-term (Sec. 2.3).
* ``direct``: the discrete sum Eq. (10), written out over all cell pairs,
  for the whole grid or for chosen target cells.
* ``fft_reference``: the same discrete sum evaluated by the convolution
  theorem with ``scipy.fft`` (a library primitive). Used only as a
  full-field reference on grids where the direct sum is too slow; it is
  pinned to ``direct`` on small grids.
* ``periodic``: periodic boundary conditions in the layer plane (Sec. 4):
  the replica-shell interaction function Eq. (13), the periodic direct sum
  Eq. (12) and its library-FFT reference (circular convolution at the period).
* ``stats``: the in-plane mean square of each stress component per height
  (Eq. 20).
* ``nye``: density channels in the axis basis for line directions that vary
  from cell to cell (linearity in t, Sec. 2.1).
* ``relax``: relaxation of the stress under free top and bottom surfaces
  (Sec. 5): force density Eq. (15), traction conditions Eq. (16c) on ghost
  layers Eq. (18b), explicit pseudo-time steps of Eq. (17), total stress.

Every function is FP64. Readings of points where the paper is silent or
ambiguous are stated in the docstring that applies them.
"""
from .segment import (VOIGT, segment_stress, segment_stress_vertical,
                      segment_stress_general, chord_length)
from .kernel import KernelGeometry, interaction_kernel, kernel_table
from .direct import stress_direct
from .fft_reference import stress_fft_reference
from .periodic import periodic_kernel, stress_direct_periodic, stress_fft_reference_periodic

__all__ = [
    "VOIGT", "segment_stress", "segment_stress_vertical", "segment_stress_general",
    "chord_length", "KernelGeometry", "interaction_kernel", "kernel_table",
    "stress_direct", "stress_fft_reference",
    "periodic_kernel", "stress_direct_periodic", "stress_fft_reference_periodic",
]
