"""Periodic boundary conditions in the layer plane (Sec. 4 of the paper).

Test infrastructure (see ``oracle/__init__.py``).

With the sample continued periodically along x and/or y, a source cell acts
through all of its replicas. Eq. (12)-(13) replace the interaction function
by its sum over replica shells,
    F(Delta) = sum_{k,l} K(Delta + (k Nx, l Ny, 0)),
cut at a shell number n_sh (the paper: 15 to 20 shells for better than 3 %).
The sum over cells then runs over one period with F, a circular convolution
in the periodic directions.

Readings taken where the paper leaves the construction open:

* the sum over square shells |k|, |l| <= n_sh is taken around the centred
  representative of the offset: Delta_a is first reduced to
  [-N_a/2, N_a/2) modulo N_a, so F is exactly periodic;
* at the half period (N_a even, Delta_a = -N_a/2) the two representatives
  -N_a/2 and +N_a/2 are equally central; F takes the mean of both sums, which
  keeps F exactly odd under inversion, as K is;
* the near-cell subdivision applies to a replica term when its own offset is
  near; the self-term K(0) = 0 (only the central replica of Delta = 0);
* z is never periodic (free or open top and bottom of a layer).
"""
import numpy as np
import scipy.fft as sfft

from .kernel import interaction_kernel
from .direct import _geoms


def _axis_reps(off, n, periodic):
    """Representatives and weights of offsets ``off`` (M,) along one axis:
    [(reps (M,), weights (M,)), ...] (one entry, or two at the half period)."""
    off = np.asarray(off, dtype=np.int64)
    if not periodic:
        return [(off, np.ones(off.shape))]
    r = np.mod(off + n // 2, n) - n // 2                  # in [-n/2, n/2)
    half = (n % 2 == 0) & (r == -(n // 2))
    w = np.where(half, 0.5, 1.0)
    return [(r, w), (np.where(half, -r, r), np.where(half, 0.5, 0.0))]


def periodic_kernel(geom, offsets, n, periodic, shells):
    """F(Delta) for integer offsets (M, 3): K summed over the replica shells of
    the periodic axes. ``n`` = (Nx, Ny, Nz); ``periodic`` = (px, py) booleans.
    Returns (M, 6, 3)."""
    offsets = np.asarray(offsets, dtype=np.int64).reshape(-1, 3)
    px, py = bool(periodic[0]), bool(periodic[1])
    kx = range(-shells, shells + 1) if px else [0]
    ky = range(-shells, shells + 1) if py else [0]
    out = np.zeros((offsets.shape[0], 6, 3))
    for rx, wx in _axis_reps(offsets[:, 0], n[0], px):
        for ry, wy in _axis_reps(offsets[:, 1], n[1], py):
            w = wx * wy
            sel = w != 0.0
            if not np.any(sel):
                continue
            for a in kx:
                for b in ky:
                    shifted = np.stack([rx[sel] + a * n[0], ry[sel] + b * n[1], offsets[sel, 2]], axis=-1)
                    out[sel] += w[sel, None, None] * interaction_kernel(geom, shifted)
    return out


def stress_direct_periodic(rho, d, lines, mu, nu, periodic=(True, True), shells=15, near_shells=2,
                           targets=None):
    """Stress by direct summation over one period of source cells with the
    replica-summed interaction function.

    rho: (C, Nz, Ny, Nx) FP64 channels (C = 3 * len(lines)); returns
    (6, Nz, Ny, Nx), Voigt order (xx, yy, zz, yz, xz, xy). With ``targets``
    (T, 3) integer cells (i, j, k) it returns (6, T) and sums over the source
    cells that carry density only (a cell whose channels are all zero adds
    nothing), so a sparse density on a large grid stays cheap."""
    rho = np.asarray(rho, dtype=np.float64)
    C, nz, ny, nx = rho.shape
    lines = np.asarray(lines, dtype=np.float64).reshape(-1, 3)
    if C != 3 * len(lines):
        raise ValueError("rho must have 3 channels per line direction")
    geoms = _geoms(d, lines, mu, nu, near_shells)
    if targets is not None:
        targets = np.asarray(targets, dtype=np.int64).reshape(-1, 3)
        kk, jj, ii = np.nonzero(np.any(rho != 0.0, axis=0))
        src = np.stack([ii, jj, kk], axis=-1)
        offs = (targets[:, None, :] - src[None, :, :]).reshape(-1, 3)       # (T * S, 3)
        out = np.zeros((6, len(targets)))
        for l, g in enumerate(geoms):
            F = periodic_kernel(g, offs, (nx, ny, nz), periodic, shells).reshape(len(targets), len(src), 6, 3)
            out += np.einsum("tsvg,gs->vt", F, rho[3 * l:3 * l + 3, kk, jj, ii])
        return out
    # F on every offset Delta_a in (-N_a, N_a): (2nz-1, 2ny-1, 2nx-1, 6, 3)
    gz, gy, gx = np.meshgrid(np.arange(-(nz - 1), nz), np.arange(-(ny - 1), ny),
                             np.arange(-(nx - 1), nx), indexing="ij")
    offs = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=-1)
    out = np.zeros((6, nz, ny, nx))
    for l, g in enumerate(geoms):
        F = periodic_kernel(g, offs, (nx, ny, nz), periodic, shells)
        tab = np.moveaxis(F.reshape(2 * nz - 1, 2 * ny - 1, 2 * nx - 1, 6, 3), (3, 4), (0, 1))
        r = rho[3 * l:3 * l + 3].reshape(3 * nz * ny * nx)
        for k0 in range(nz):
            for j0 in range(ny):
                for i0 in range(nx):
                    win = tab[:, :, k0:k0 + nz, j0:j0 + ny, i0:i0 + nx][:, :, ::-1, ::-1, ::-1]
                    out[:, k0, j0, i0] += win.reshape(6, -1) @ r
    return out


def _padded(n):
    p = 1
    while p < 2 * n - 1:
        p *= 2
    return p


def stress_fft_reference_periodic(rho, d, lines, mu, nu, periodic=(True, True), shells=15, near_shells=2,
                                  workers=None):
    """Same result as ``stress_direct_periodic``, through the convolution
    theorem with ``scipy.fft``: a periodic axis is transformed at its own
    length N (F is N-periodic there, so the circular convolution is the
    periodic sum), every other axis is zero padded to a power of two >= 2N-1.
    rho: (C, Nz, Ny, Nx). Returns (6, Nz, Ny, Nx)."""
    rho = np.asarray(rho, dtype=np.float64)
    C, nz, ny, nx = rho.shape
    lines = np.asarray(lines, dtype=np.float64).reshape(-1, 3)
    if C != 3 * len(lines):
        raise ValueError("rho must have 3 channels per line direction")
    px, py = bool(periodic[0]), bool(periodic[1])
    P = (_padded(nz), ny if py else _padded(ny), nx if px else _padded(nx))

    def axis(n, p, per):
        idx = np.arange(p)
        if per:
            return idx, np.ones(p, dtype=bool)
        return np.where(idx < n, idx, idx - p), (idx < n) | (idx > p - n)
    oz, vz = axis(nz, P[0], False)
    oy, vy = axis(ny, P[1], py)
    ox, vx = axis(nx, P[2], px)
    gz, gy, gx = np.meshgrid(oz, oy, ox, indexing="ij")
    valid = vz[:, None, None] & vy[None, :, None] & vx[None, None, :]
    offs = np.stack([gx[valid], gy[valid], gz[valid]], axis=-1)
    out_hat = np.zeros((6, P[0], P[1], P[2] // 2 + 1), dtype=np.complex128)
    for l, g in enumerate(_geoms(d, lines, mu, nu, near_shells)):
        F = periodic_kernel(g, offs, (nx, ny, nz), (px, py), shells)   # (M, 6, 3)
        for gam in range(3):
            r = np.zeros(P)
            r[:nz, :ny, :nx] = rho[3 * l + gam]
            r_hat = sfft.rfftn(r, workers=workers)
            for v in range(6):
                k = np.zeros(P)
                k[valid] = F[:, v, gam]
                out_hat[v] += sfft.rfftn(k, workers=workers) * r_hat
    out = np.empty((6, nz, ny, nx))
    for v in range(6):
        out[v] = sfft.irfftn(out_hat[v], s=P, workers=workers)[:nz, :ny, :nx]
    return out
