"""In-plane statistics of the stress field (Sec. 6, Eq. 20).

Test infrastructure (see ``oracle/__init__.py``).

    s_v^2(h_k) = (1 / (Nx Ny)) sum_{i,j} sigma_v(x_i, y_j, h_k)^2

for every stress component v and height h_k: the mean square over the layer
plane. As printed, Eq. (20) does not subtract the plane mean (the paper's
random Burgers vectors make it vanish), so neither does this.
"""
import numpy as np


def plane_mean_square(sigma):
    """sigma (..., 6, Nz, Ny, Nx) -> s^2 (..., 6, Nz) in FP64."""
    s = np.asarray(sigma, dtype=np.float64)
    return np.mean(s * s, axis=(-2, -1))
