"""Eq. (10) evaluated through the convolution theorem with ``scipy.fft``.

Test infrastructure (see ``oracle/__init__.py``). The paper notes that the
translation invariance of f turns Eq. (10) into a discrete convolution that an
FFT evaluates (Sec. 2.3). This module applies that statement with a library
FFT to the oracle's own kernel so that grids too large for the direct sum
still get a full-field FP64 reference. Zero padding to at least 2N-1 points
per axis makes the circular convolution equal to the linear one. It is pinned
to ``direct.stress_direct`` on small grids by the tests.
"""
import numpy as np
import scipy.fft as sfft

from .kernel import KernelGeometry, interaction_kernel


def _padded(n):
    p = 1
    while p < 2 * n - 1:
        p *= 2
    return p


def stress_fft_reference(rho, d, lines, mu, nu, near_shells=2, workers=None):
    """Same result as ``stress_direct(..., targets=None)``, computed by FFT.
    rho: (C, Nz, Ny, Nx). Returns (6, Nz, Ny, Nx)."""
    rho = np.asarray(rho, dtype=np.float64)
    C, nz, ny, nx = rho.shape
    lines = np.asarray(lines, dtype=np.float64).reshape(-1, 3)
    P = (_padded(nz), _padded(ny), _padded(nx))
    # offsets in wrap order: index i <-> offset i for i < n, i - P for i > P - n
    def wrap_axis(n, p):
        idx = np.arange(p)
        off = np.where(idx < n, idx, idx - p)
        valid = (idx < n) | (idx > p - n)
        return off, valid
    oz, vz = wrap_axis(nz, P[0])
    oy, vy = wrap_axis(ny, P[1])
    ox, vx = wrap_axis(nx, P[2])
    gz, gy, gx = np.meshgrid(oz, oy, ox, indexing="ij")
    valid = vz[:, None, None] & vy[None, :, None] & vx[None, None, :]
    offs = np.stack([gx[valid], gy[valid], gz[valid]], axis=-1)
    out_hat = np.zeros((6, P[0], P[1], P[2] // 2 + 1), dtype=np.complex128)
    for l, t in enumerate(lines):
        g = KernelGeometry(d=tuple(map(float, d)), t=tuple(map(float, t)), mu=float(mu),
                           nu=float(nu), near_shells=int(near_shells))
        K = interaction_kernel(g, offs)                                 # (M, 6, 3)
        for gam in range(3):
            r = np.zeros(P)
            r[:nz, :ny, :nx] = rho[3 * l + gam]
            r_hat = sfft.rfftn(r, workers=workers)
            for v in range(6):
                k = np.zeros(P)
                k[valid] = K[:, v, gam]
                out_hat[v] += sfft.rfftn(k, workers=workers) * r_hat
    out = np.empty((6, nz, ny, nx))
    for v in range(6):
        out[v] = sfft.irfftn(out_hat[v], s=P, workers=workers)[:nz, :ny, :nx]
    return out
