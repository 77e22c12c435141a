"""Seeded synthetic density fields shaped like the paper's workloads.

This module only builds inputs: grids, cell sizes, elastic constants, line
directions and density channels. It holds none of the method's arithmetic and
is the one module that both the HIP path's callers and the oracle's tests use.

A workload is a dict with
    name, n = (Nx, Ny, Nz), d = (dx, dy, dz), mu, nu,
    lines: (L, 3) unit line directions,
    rho:   (B, 3L, Nz, Ny, Nx) float64, channel c = 3*l + gamma holding the
           line density of direction l times its Burgers component gamma.

Recipes (coordinates in units of dx; sample centre ((Nx-1)/2, (Ny-1)/2)):

* disk_edge: vertical edge dislocations (t = e_z, b = e_x) in a disk, density
  exp(-r^2 / (2 w^2)) inside radius r_max, constant in z (Sec. 3, Eq. 11 with
  the vertical decay dropped).
* disk_mixed: t = e_z, per cell a random angle phi and b = (cos phi, sin phi, 1)/sqrt 2,
  density a radial Gaussian times (1 + 0.1 U(-1, 1)) inside r_max.
* poly_layer: columnar Voronoi grains (vertical grain boundaries, Sec. 6),
  per grain one of six in-plane a-type Burgers vectors at 60 degrees and either
  an edge line (t = e_z) or a mixed line inclined by 15.6 degrees in the
  xz-plane (the incline quoted in Sec. 6.3); density exp(-z / z_decay) from the
  layer bottom, homogeneous in each plane (Sec. 6, Eq. 19 replaced by an
  exponential profile).
"""
import numpy as np

MIXED_INCLINE_DEG = 15.6
E_Z = (0.0, 0.0, 1.0)


def mixed_line():
    a = np.radians(MIXED_INCLINE_DEG)
    return (float(np.sin(a)), 0.0, float(np.cos(a)))


def _radius(nx, ny):
    x = np.arange(nx) - (nx - 1) / 2.0
    y = np.arange(ny) - (ny - 1) / 2.0
    return np.sqrt(x[None, :] ** 2 + y[:, None] ** 2)          # [y][x]


def disk_edge(nx=32, ny=32, nz=4, d=(1.0, 1.0, 4.0), width=8.0, r_max=14.0,
              mu=1.0, nu=0.3):
    r = _radius(nx, ny)
    dens = np.where(r <= r_max, np.exp(-r * r / (2.0 * width * width)), 0.0)
    rho = np.zeros((1, 3, nz, ny, nx))
    rho[0, 0] = dens[None, :, :]
    return dict(name=f"disk-edge-{nx}x{ny}x{nz}", n=(nx, ny, nz), d=tuple(d), mu=mu, nu=nu,
                lines=np.array([E_Z]), rho=rho)


def disk_mixed(nx=128, ny=128, nz=32, d=(1.0, 1.0, 2.0), width=30.0, r_max=56.0,
               noise=0.1, mu=1.0, nu=0.3, seed=2):
    rng = np.random.default_rng(seed)
    r = _radius(nx, ny)
    base = np.where(r <= r_max, np.exp(-r * r / (2.0 * width * width)), 0.0)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=(nz, ny, nx))
    jitter = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    n = base[None] * (1.0 + noise * jitter)
    s = 1.0 / np.sqrt(2.0)
    rho = np.stack([n * np.cos(phi) * s, n * np.sin(phi) * s, n * s])[None]
    return dict(name=f"disk-mixed-{nx}x{ny}x{nz}", n=(nx, ny, nz), d=tuple(d), mu=mu, nu=nu,
                lines=np.array([E_Z]), rho=rho)


def voronoi_grains(nx, ny, n_grains, rng, periodic=False):
    """Grain index per (y, x) cell: nearest of ``n_grains`` centres uniform in
    [0, Nx) x [0, Ny), Euclidean distance (the minimum-image distance when
    ``periodic``, so grains continue across the period), ties to the lowest
    index."""
    cx = rng.uniform(0.0, nx, size=n_grains)
    cy = rng.uniform(0.0, ny, size=n_grains)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    grain = np.zeros((ny, nx), dtype=np.int64)
    best = np.full((ny, nx), np.inf)
    for g in range(n_grains):
        ddx = np.abs(x - cx[g])
        ddy = np.abs(y - cy[g])
        if periodic:
            ddx = np.minimum(ddx, nx - ddx)
            ddy = np.minimum(ddy, ny - ddy)
        dist = ddx[None, :] ** 2 + ddy[:, None] ** 2
        closer = dist < best
        grain[closer] = g
        best[closer] = dist[closer]
    return grain


def poly_layer(nx=256, ny=256, nz=64, d=(1.0, 1.0, 2.0), grain=16.0, z_decay=8.0,
               mu=1.0, nu=0.2, seed=3, p_mixed=0.5, batch_seeds=None, periodic=False):
    """Columnar polycrystal layer; ``batch_seeds`` stacks several realisations.
    ``periodic``: grains continue across the in-plane period (for plans with
    periodic boundaries along x and y)."""
    seeds = [seed] if batch_seeds is None else list(batch_seeds)
    n_grains = max(1, int(round(nx * ny / float(grain) ** 2)))
    z = np.arange(nz) * d[2]
    prof = np.exp(-z / z_decay)
    rho = np.zeros((len(seeds), 6, nz, ny, nx))
    for bi, sd in enumerate(seeds):
        rng = np.random.default_rng(sd)
        gmap = voronoi_grains(nx, ny, n_grains, rng, periodic)
        angle = np.radians(60.0) * rng.integers(0, 6, size=n_grains)
        is_mixed = rng.uniform(size=n_grains) < p_mixed
        bx = np.cos(angle)[gmap]
        by = np.sin(angle)[gmap]
        line = is_mixed[gmap].astype(np.int64)          # 0: edge (t = e_z), 1: mixed
        for l in range(2):
            sel = (line == l).astype(np.float64)
            rho[bi, 3 * l + 0] = prof[:, None, None] * (sel * bx)[None]
            rho[bi, 3 * l + 1] = prof[:, None, None] * (sel * by)[None]
    name = f"poly-layer{'-pbc' if periodic else ''}-{nx}x{ny}x{nz}-g{grain:g}"
    return dict(name=name, n=(nx, ny, nz), d=tuple(d), mu=mu, nu=nu,
                lines=np.array([E_Z, mixed_line()]), rho=rho)


def poly_sweep(nx=128, ny=128, nz=32, grains=(4, 8, 16, 32), per_grain=16, **kw):
    """Realisations over several grain sizes with one shared plan (same shape,
    cells, constants and line directions): 16 seeds per grain size,
    seed = 1000 * G + s."""
    parts = [poly_layer(nx, ny, nz, grain=float(g), batch_seeds=[1000 * g + s for s in range(per_grain)],
                        **kw) for g in grains]
    out = dict(parts[0])
    out["rho"] = np.concatenate([p["rho"] for p in parts], axis=0)
    out["name"] = f"poly-sweep-{len(out['rho'])}x{nx}x{ny}x{nz}"
    return out


def random_field(n, n_lines=1, batch=1, seed=0, d=(1.0, 1.0, 1.0), mu=1.0, nu=0.3, lines=None):
    """Uniform(-1, 1) density channels on an arbitrary grid (parity tests)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    if lines is None:
        base = [E_Z, mixed_line(), (0.0, 1.0 / np.sqrt(2.0), 1.0 / np.sqrt(2.0))]
        lines = np.array(base[:n_lines])
    rho = rng.uniform(-1.0, 1.0, size=(batch, 3 * len(lines), nz, ny, nx))
    return dict(name=f"random-{nx}x{ny}x{nz}-L{len(lines)}-B{batch}", n=(nx, ny, nz), d=tuple(d),
                mu=mu, nu=nu, lines=np.asarray(lines, dtype=np.float64), rho=rho)


def random_stress(n, seed=0, d=(1.0, 1.0, 1.0), mu=1.0, nu=0.3, smooth=False):
    """A load for the free-surface relaxation: six Voigt stress components on
    an Nx x Ny x Nz node grid, Uniform(-1, 1) per node, or with ``smooth`` a
    sum of four random in-plane Fourier modes (periodic in x and y) times a
    random quadratic in z."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    if not smooth:
        sig = rng.uniform(-1.0, 1.0, size=(6, nz, ny, nx))
    else:
        x = np.arange(nx) / nx
        y = np.arange(ny) / ny
        z = np.arange(nz) / max(1, nz - 1)
        sig = np.zeros((6, nz, ny, nx))
        for v in range(6):
            for _ in range(4):
                kx, ky = rng.integers(0, 4, size=2)
                ph = rng.uniform(0.0, 2.0 * np.pi)
                plane = np.cos(2.0 * np.pi * (kx * x[None, :] + ky * y[:, None]) + ph)
                c = rng.uniform(-1.0, 1.0, size=3)
                prof = c[0] + c[1] * z + c[2] * z * z
                sig[v] += prof[:, None, None] * plane[None]
    return dict(name=f"stress-{nx}x{ny}x{nz}", n=(nx, ny, nz), d=tuple(d), mu=mu, nu=nu, sigma=sig)


def poly_layer_lines(nx=256, ny=256, nz=64, d=(1.0, 1.0, 2.0), grain=16.0, z_decay=8.0, mu=1.0, nu=0.2, seed=3,
                     max_tilt_deg=30.0, periodic=True, batch_seeds=None):
    """Columnar polycrystal layer whose dislocation lines vary from grain to
    grain: per grain a line direction tilted from e_z by an angle uniform in
    [0, max_tilt] at a uniform azimuth, and a Burgers vector (cos 60 i,
    sin 60 i, 0), i ~ U{0..5}; line density n(z) = exp(-z / z_decay). Per-cell
    fields n (nb, Nz, Ny, Nx), t and b (nb, 3, Nz, Ny, Nx) for the axis-basis
    (Nye) channels."""
    seeds = [seed] if batch_seeds is None else list(batch_seeds)
    n_grains = max(1, int(round(nx * ny / float(grain) ** 2)))
    z = np.arange(nz) * d[2]
    prof = np.exp(-z / z_decay)
    nb = len(seeds)
    n = np.zeros((nb, nz, ny, nx))
    t = np.zeros((nb, 3, nz, ny, nx))
    b = np.zeros((nb, 3, nz, ny, nx))
    for bi, sd in enumerate(seeds):
        rng = np.random.default_rng(sd)
        gmap = voronoi_grains(nx, ny, n_grains, rng, periodic)
        tilt = np.radians(max_tilt_deg) * rng.uniform(0.0, 1.0, size=n_grains)
        az = rng.uniform(0.0, 2.0 * np.pi, size=n_grains)
        ang = np.radians(60.0) * rng.integers(0, 6, size=n_grains)
        tg = np.stack([np.sin(tilt) * np.cos(az), np.sin(tilt) * np.sin(az), np.cos(tilt)])[:, gmap]
        bg = np.stack([np.cos(ang), np.sin(ang), np.zeros(n_grains)])[:, gmap]
        n[bi] = prof[:, None, None] * np.ones((ny, nx))[None]
        t[bi] = tg[:, None]
        b[bi] = bg[:, None]
    name = f"poly-lines{'-pbc' if periodic else ''}-{nx}x{ny}x{nz}-g{grain:g}"
    return dict(name=name, n=(nx, ny, nz), d=tuple(d), mu=mu, nu=nu, density=n, t=t, b=b)
