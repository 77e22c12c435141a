"""Density channels in the axis basis (the Nye tensor) for line directions
that vary from cell to cell.

Test infrastructure (see ``oracle/__init__.py``).

Sec. 2.1 treats the stress of a volume element as linear in the line
direction t. That holds exactly for an infinitesimal segment (its field is
linear in the segment vector dl t) and only approximately for the finite
chord a cell represents. Taking it as exact, a density n of dislocations with
direction t and Burgers vector b in a cell acts like the three axis-direction
densities n t_l (l = x, y, z) with the same b, so with the three fixed line
directions e_x, e_y, e_z the channels are
    rho_{3 l + gamma} = n t_l b_gamma      (the Nye tensor alpha_{l gamma}),
summed over the dislocation families present in the cell. The error of the
decomposition lives in the near field, where the chord of a tilted line and
those of the axes differ; far from the source it vanishes with the segment's
size over the distance.
"""
import numpy as np

AXES = ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))


def nye_channels(n, t, b):
    """n (..., cells...), t and b (3, cells...) -> rho (9, cells...) with
    rho[3 l + gamma] = n t_l b_gamma; t is used as given (unit length is the
    caller's convention)."""
    n = np.asarray(n, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.empty((9,) + n.shape)
    for l in range(3):
        for g in range(3):
            out[3 * l + g] = (n * t[l]) * b[g]
    return out
