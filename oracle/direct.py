"""Direct evaluation of the discrete stress sum, Eq. (10) of the paper, summed
over dislocation types as Eq. (3b) prescribes.

Test infrastructure (see ``oracle/__init__.py``).

    sigma_v(r0) = sum_{cells i} sum_{c < C} K_{v,c}(r0 - r_i) rho_c(r_i)

Cell (i, j, k) has its centre at (i dx, j dy, k dz). Arrays are indexed
[c][k][j][i] (x fastest). Channel c = 3*l + gamma carries the density of
dislocations with line direction t_l times their Burgers component gamma.
The sum runs over every source cell of the grid: open boundaries, no
periodic images (the sample is embedded in an infinite medium, Sec. 3).
"""
import numpy as np

from .kernel import KernelGeometry, interaction_kernel, kernel_table


def _geoms(d, lines, mu, nu, near_shells):
    return [KernelGeometry(d=tuple(map(float, d)), t=tuple(map(float, t)), mu=float(mu),
                           nu=float(nu), near_shells=int(near_shells)) for t in lines]


def stress_direct(rho, d, lines, mu, nu, near_shells=2, targets=None, chunk=1 << 17):
    """Stress by direct summation over all cell pairs.

    rho:      (C, Nz, Ny, Nx) FP64 density channels, C = 3 * len(lines).
    d:        cell sizes (dx, dy, dz).
    lines:    (L, 3) line directions (normalised here).
    targets:  None for every cell of the grid, else (T, 3) integer target
              cells (i, j, k).
    Returns (6, Nz, Ny, Nx) or (6, T), Voigt order (xx, yy, zz, yz, xz, xy).
    """
    rho = np.asarray(rho, dtype=np.float64)
    C, nz, ny, nx = rho.shape
    lines = np.asarray(lines, dtype=np.float64).reshape(-1, 3)
    if C != 3 * len(lines):
        raise ValueError("rho must have 3 channels per line direction")
    geoms = _geoms(d, lines, mu, nu, near_shells)

    if targets is None:
        # kernel on every offset, then the sum for each target cell
        tabs = [kernel_table(g, (nx, ny, nz)) for g in geoms]   # (6,3,2nz-1,2ny-1,2nx-1)
        out = np.zeros((6, nz, ny, nx))
        for l, tab in enumerate(tabs):
            r = rho[3 * l:3 * l + 3].reshape(3 * nz * ny * nx)
            for k0 in range(nz):
                for j0 in range(ny):
                    for i0 in range(nx):
                        # K(r0 - r_i): offset index (k0 - k) + nz - 1 for k = 0..nz-1
                        win = tab[:, :, k0:k0 + nz, j0:j0 + ny, i0:i0 + nx][:, :, ::-1, ::-1, ::-1]
                        out[:, k0, j0, i0] += win.reshape(6, -1) @ r
        return out

    targets = np.asarray(targets, dtype=np.int64).reshape(-1, 3)
    gz, gy, gx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    src = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=-1)      # [k][j][i] order
    flat = rho.reshape(C, -1)
    out = np.zeros((6, len(targets)))
    for ti, tgt in enumerate(targets):
        for lo in range(0, src.shape[0], chunk):
            s = src[lo:lo + chunk]
            offs = tgt[None, :] - s
            for l, g in enumerate(geoms):
                K = interaction_kernel(g, offs)                        # (M, 6, 3)
                out[:, ti] += np.einsum("mvg,gm->v", K, flat[3 * l:3 * l + 3, lo:lo + chunk])
    return out
