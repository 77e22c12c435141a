"""Interaction coefficients between grid cells (Sec. 2.1 and 2.3 of the paper).

Test infrastructure (see ``oracle/__init__.py``).

The discrete sum Eq. (10) reads, for one dislocation type,
    sigma(r0) = b * sum_i n(r_i) f(e_b, t; r0 - r_i) dV_i .
Because f is linear in e_b (Eq. 4a, Eq. 6), b * f(e_b) = sum_gamma b_gamma f(e_gamma),
so with the density channels rho_c = n * b_gamma (c = 3*l + gamma for line
direction t_l) the sum becomes
    sigma_v(r0) = sum_i sum_c K_{v,c}(r0 - r_i) rho_c(r_i)
with K_{v,3l+gamma}(Delta) = dV * f_v(e_gamma, t_l; Delta) and f = sigma^AB/(Delta l)
for a unit Burgers vector (Eq. 9b). The offset Delta = r0 - r_i runs from the
source cell to the target cell, as in Eq. (1) and Eq. (10).

Near cells (Sec. 2.3, Fig. 3): target and source cells are split into the same
near-cubic subcells and the coefficient is the stress averaged over the target
subcells of the sum over source subcells. Readings taken where the paper gives
no numbers:

* subcells per axis m_a = max(1, floor(d_a / d_min + 1/2)), subcell edge s = d/m;
* a cell offset Delta is "near" when |Delta_a| * d_a <= S * d_max on every axis,
  with S the number of near shells (default 2);
* each subcell carries a segment of its own chord length along t, and the
  stress per unit length of that segment is weighted by the subcell volume;
* because only differences of subcell centres enter, the double sum over
  target and source subcells collapses to a sum over sub-offsets delta with
  |delta_a| < m_a and weight w(delta) = prod_a (m_a - |delta_a|) / m_a^2;
* far cells use the stress at the cell-centre offset of a segment whose
  length is the cell's own chord along t;
* the self-term K(0) is zero: with identical target and source subdivision
  every pair of sub-offsets +delta, -delta cancels by the inversion oddness of
  a centred segment, and the same-subcell term vanishes as the paper argues.
"""
from dataclasses import dataclass

import numpy as np

from .segment import segment_stress, chord_length


@dataclass(frozen=True)
class KernelGeometry:
    """Cell sizes ``d`` = (dx, dy, dz), elastic constants, one line direction
    ``t`` and the number of near shells. All lengths in one unit. ``refine``
    multiplies the subcell count on every axis (1: the subdivision described
    above); the subcells stay as near-cubic as the plain ones, so raising it
    only refines the near-cell sums (used to check their convergence)."""
    d: tuple
    t: tuple
    mu: float
    nu: float
    near_shells: int = 2
    refine: int = 1

    @property
    def unit_t(self):
        t = np.asarray(self.t, dtype=np.float64)
        return t / np.linalg.norm(t)

    @property
    def subdivision(self):
        d = np.asarray(self.d, dtype=np.float64)
        dmin = d.min()
        return np.array([max(1, int(np.floor(d[a] / dmin + 0.5))) * int(self.refine) for a in range(3)])

    @property
    def sub_box(self):
        return np.asarray(self.d, dtype=np.float64) / self.subdivision

    @property
    def cell_volume(self):
        d = np.asarray(self.d, dtype=np.float64)
        return float(d[0] * d[1] * d[2])

    def is_near(self, offsets):
        """Boolean mask of the offsets (M, 3) that are subdivided."""
        d = np.asarray(self.d, dtype=np.float64)
        lim = self.near_shells * d.max()
        return np.all(np.abs(offsets) * d <= lim, axis=-1)

    def sub_offsets(self):
        """Sub-offsets delta (Q, 3) and their weights w(delta) (Q,)."""
        m = self.subdivision
        axes = [np.arange(-(m[a] - 1), m[a]) for a in range(3)]
        dz, dy, dx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        delta = np.stack([dx.ravel(), dy.ravel(), dz.ravel()], axis=-1)
        w = np.prod((m - np.abs(delta)) / (m * m).astype(np.float64), axis=-1)
        return delta, w


def interaction_kernel(geom, offsets, chunk=1 << 18):
    """K(Delta) for integer cell offsets ``offsets`` (M, 3) (x, y, z order).
    Returns (M, 6, 3): Voigt component x Burgers component gamma, for the
    single line direction of ``geom``."""
    offsets = np.asarray(offsets, dtype=np.int64).reshape(-1, 3)
    M = offsets.shape[0]
    out = np.zeros((M, 6, 3))
    d = np.asarray(geom.d, dtype=np.float64)
    t = geom.unit_t
    dV = geom.cell_volume
    h_cell = chord_length(d, t)
    s = geom.sub_box
    h_sub = chord_length(s, t)
    zero = np.all(offsets == 0, axis=-1)
    near = geom.is_near(offsets) & ~zero
    far = ~near & ~zero

    # far cells: point value at the centre offset (Eq. 9b times dV)
    idx = np.nonzero(far)[0]
    for lo in range(0, idx.size, chunk):
        sel = idx[lo:lo + chunk]
        p = offsets[sel] * d
        out[sel] = segment_stress(p, h_cell, t, geom.mu, geom.nu) * (dV / h_cell)

    # near cells: weighted sum over sub-offsets
    idx = np.nonzero(near)[0]
    if idx.size:
        delta, w = geom.sub_offsets()
        for lo in range(0, idx.size, max(1, chunk // len(w))):
            sel = idx[lo:lo + max(1, chunk // len(w))]
            p = (offsets[sel] * d)[:, None, :] + (delta * s)[None, :, :]
            f = segment_stress(p.reshape(-1, 3), h_sub, t, geom.mu, geom.nu)
            f = f.reshape(len(sel), len(w), 6, 3)
            out[sel] = np.einsum("q,mqvg->mvg", w, f) * (dV / h_sub)
    return out


def kernel_table(geom, n):
    """K on every offset Delta with |Delta_a| <= n_a - 1, as an array
    (6, 3, 2nz-1, 2ny-1, 2nx-1) indexed by Delta + (n - 1)."""
    nx, ny, nz = n
    gz, gy, gx = np.meshgrid(np.arange(-(nz - 1), nz), np.arange(-(ny - 1), ny),
                             np.arange(-(nx - 1), nx), indexing="ij")
    offs = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=-1)
    K = interaction_kernel(geom, offs)
    K = K.reshape(2 * nz - 1, 2 * ny - 1, 2 * nx - 1, 6, 3)
    return np.ascontiguousarray(np.moveaxis(K, (3, 4), (0, 1)))
