"""Relaxation of the dislocation stress under free top and bottom surfaces
(Sec. 5 of the paper, Eq. 14-18).

Test infrastructure (see ``oracle/__init__.py``).

The total stress is sigma = sigma^dis + sigma(u), where the displacement u
solves the Navier-Cauchy equation Eq. (14),
    A grad div u - B rot rot u + f^ext = 0,
with A = E (1 - nu) / ((1 + nu)(1 - 2 nu)) = lambda + 2 mu and
B = E / (2 (1 + nu)) = mu, driven by the force density f^ext = div sigma^dis
(Eq. 15), periodic in x and y (Eq. 16a) and with the traction-free conditions
Eq. (16b) on z = 0 and z = h, written for u as Eq. (16c). It is found as the
stationary state of the explicit pseudo-time iteration Eq. (17),
    u(t + dt) = u(t) + dt (A grad div u - B rot rot u + f^ext),
with dt = min(d)^2 / (5A - 3B), and ghost layers below and above the film
that carry Eq. (16c) (Eq. 18a-b).

Readings taken where the paper leaves the discretisation open:

* nodes sit at the cell centres; the free surfaces pass through the first
  and the last layer of nodes (Eq. 18a centres the z difference on k = 1),
  so the film is (Nz - 1) dz thick and Nz >= 3 is required;
* grad div - rot rot = (A - B) grad div + B laplacian, with central second
  differences (u_{i+1} - 2 u_i + u_{i-1}) / d^2 and the mixed derivatives as
  products of central first differences (u_{i+1} - u_{i-1}) / (2 d) (the
  four-point stencil); x and y wrap around (Eq. 16a);
* f^ext by central differences in x and y, in z by central differences
  inside the film and second-order one-sided differences on the two surface
  layers (sigma^dis exists only inside the film);
* the ghost layers are rewritten from the real layers after every step
  (Eq. 18b for u_x at the bottom, the same construction for u_y, for u_z
  from the third condition of Eq. 16c, and for the top surface, whose
  outward normal is +z); before the first step they are set from u = 0;
* the iteration count is the caller's (the paper names no stopping rule);
  ``update_norm`` gives max |v| of the current state as a convergence measure;
* the output is the total stress sigma^dis + sigma(u) at the nodes, sigma(u)
  by Hooke's law with the same central differences (the ghost layers supply
  the z differences on the surfaces, so the total sigma_xz, sigma_yz,
  sigma_zz vanish there to rounding).

Arrays are [component][k][j][i] (x fastest). u carries the ghost layers:
(3, Nz + 2, Ny, Nx) with layer k + 1 holding node layer k. Stress in Voigt
order (xx, yy, zz, yz, xz, xy).
"""
import numpy as np

VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def moduli(mu, nu):
    """A and B of Eq. (14) from the shear modulus and the Poisson ratio
    (E = 2 mu (1 + nu))."""
    E = 2.0 * mu * (1.0 + nu)
    A = E * (1.0 - nu) / ((1.0 + nu) * (1.0 - 2.0 * nu))
    B = E / (2.0 * (1.0 + nu))
    return A, B, E


def paper_time_step(d, mu, nu):
    """dt = min(d)^2 / (5A - 3B) (Sec. 5)."""
    A, B, _ = moduli(mu, nu)
    return min(d) ** 2 / (5.0 * A - 3.0 * B)


def _dx(a, h, axis):
    """Central first difference along a periodic axis."""
    return (np.roll(a, -1, axis=axis) - np.roll(a, 1, axis=axis)) / (2.0 * h)


def _dxx(a, h, axis):
    return (np.roll(a, -1, axis=axis) - 2.0 * a + np.roll(a, 1, axis=axis)) / (h * h)


def _sym(s, a, b):
    """Voigt component of the symmetric tensor s (6, ...) at (a, b)."""
    for v, (p, q) in enumerate(VOIGT_PAIRS):
        if (p, q) == (a, b) or (q, p) == (a, b):
            return s[v]
    raise ValueError


def load_terms(sigma_dis, d, mu, nu):
    """f^ext (Eq. 15) on the nodes, (3, Nz, Ny, Nx), and the right-hand sides
    phi of Eq. (16c) on the bottom and top surfaces, (2, 3, Ny, Nx) in the
    order (phi_xz, phi_yz, phi_zz)."""
    s = np.asarray(sigma_dis, dtype=np.float64)
    nz = s.shape[1]
    if nz < 3:
        raise ValueError("the relaxation needs Nz >= 3 node layers")
    dx, dy, dz = d
    f = np.zeros((3,) + s.shape[1:])
    for a in range(3):
        sx, sy, sz = _sym(s, a, 0), _sym(s, a, 1), _sym(s, a, 2)
        f[a] = _dx(sx, dx, 2) + _dx(sy, dy, 1)
        dzs = np.empty_like(sz)
        dzs[1:-1] = (sz[2:] - sz[:-2]) / (2.0 * dz)
        dzs[0] = (-3.0 * sz[0] + 4.0 * sz[1] - sz[2]) / (2.0 * dz)
        dzs[-1] = (3.0 * sz[-1] - 4.0 * sz[-2] + sz[-3]) / (2.0 * dz)
        f[a] += dzs
    _, _, E = moduli(mu, nu)
    phi = np.zeros((2, 3) + s.shape[2:])
    for side, k in ((0, 0), (1, nz - 1)):
        phi[side, 0] = -(1.0 + nu) / E * _sym(s, 0, 2)[k]
        phi[side, 1] = -(1.0 + nu) / E * _sym(s, 1, 2)[k]
        phi[side, 2] = -(1.0 + nu) * (1.0 - 2.0 * nu) / E * _sym(s, 2, 2)[k]
    return f, phi


def set_ghosts(u, phi, d, nu):
    """Rewrite the ghost layers of u (in place) from its real layers so that
    the discretised Eq. (16c) holds on both surfaces (Eq. 18b)."""
    dx, dy, dz = d
    nz = u.shape[1] - 2
    # bottom: surface layer 1, inner neighbour 2, ghost 0
    s, inner = 1, 2
    g_x = _dx(u[2, s], dx, 1)
    g_y = _dx(u[2, s], dy, 0)
    div_xy = _dx(u[0, s], dx, 1) + _dx(u[1, s], dy, 0)
    u[0, 0] = u[0, inner] + 2.0 * dz * (g_x - 2.0 * phi[0, 0])
    u[1, 0] = u[1, inner] + 2.0 * dz * (g_y - 2.0 * phi[0, 1])
    u[2, 0] = u[2, inner] - 2.0 * dz * (phi[0, 2] - nu * div_xy) / (1.0 - nu)
    # top: surface layer nz, inner neighbour nz - 1, ghost nz + 1
    s, inner = nz, nz - 1
    g_x = _dx(u[2, s], dx, 1)
    g_y = _dx(u[2, s], dy, 0)
    div_xy = _dx(u[0, s], dx, 1) + _dx(u[1, s], dy, 0)
    u[0, nz + 1] = u[0, inner] + 2.0 * dz * (2.0 * phi[1, 0] - g_x)
    u[1, nz + 1] = u[1, inner] + 2.0 * dz * (2.0 * phi[1, 1] - g_y)
    u[2, nz + 1] = u[2, inner] + 2.0 * dz * (phi[1, 2] - nu * div_xy) / (1.0 - nu)
    return u


def _grad(ua, d):
    """Central first differences of one component on the real layers:
    (d/dx, d/dy, d/dz), each (Nz, Ny, Nx); ua includes the ghost layers."""
    dx, dy, dz = d
    core = ua[1:-1]
    return (_dx(core, dx, 2), _dx(core, dy, 1), (ua[2:] - ua[:-2]) / (2.0 * dz))


def navier(u, d, mu, nu):
    """A grad div u - B rot rot u on the real nodes, (3, Nz, Ny, Nx), written
    as (A - B) grad div u + B laplacian u."""
    A, B, _ = moduli(mu, nu)
    dx, dy, dz = d
    h = (dx, dy, dz)
    out = np.zeros((3,) + u.shape[1:])[:, 1:-1]
    # second derivatives D_ab u_c on the real layers
    def second(c, a, b):
        uc = u[c]
        if a == b:
            if a == 2:
                return (uc[2:] - 2.0 * uc[1:-1] + uc[:-2]) / (dz * dz)
            return _dxx(uc[1:-1], h[a], 2 - a)
        if 2 in (a, b):
            p = a if b == 2 else b                       # the in-plane axis
            dzu = (uc[2:] - uc[:-2]) / (2.0 * dz)
            return _dx(dzu, h[p], 2 - p)
        return _dx(_dx(uc[1:-1], dx, 2), dy, 1)
    for a in range(3):
        lap = second(a, 0, 0) + second(a, 1, 1) + second(a, 2, 2)
        graddiv = second(0, a, 0) + second(1, a, 1) + second(2, a, 2)
        out[a] = (A - B) * graddiv + B * lap
    return out


def initial_state(sigma_dis, d, mu, nu):
    """u = 0 on the nodes, ghost layers from Eq. (16c); with f and phi."""
    s = np.asarray(sigma_dis, dtype=np.float64)
    f, phi = load_terms(s, d, mu, nu)
    u = np.zeros((3, s.shape[1] + 2) + s.shape[2:])
    set_ghosts(u, phi, d, nu)
    return u, f, phi


def relax(sigma_dis, d, mu, nu, n_iter, dt=None, u=None):
    """n_iter explicit steps of Eq. (17) from u = 0 (or from the given state,
    which must carry current ghost layers). Returns u with ghost layers."""
    if dt is None:
        dt = paper_time_step(d, mu, nu)
    u0, f, phi = initial_state(sigma_dis, d, mu, nu)
    u = u0 if u is None else np.array(u, dtype=np.float64)
    for _ in range(int(n_iter)):
        v = navier(u, d, mu, nu) + f
        u[:, 1:-1] += dt * v
        set_ghosts(u, phi, d, nu)
    return u


def update_norm(u, sigma_dis, d, mu, nu):
    """max |A grad div u - B rot rot u + f^ext| over the nodes."""
    f, _ = load_terms(sigma_dis, d, mu, nu)
    return float(np.abs(navier(u, d, mu, nu) + f).max())


def total_stress(u, sigma_dis, d, mu, nu):
    """sigma^dis + sigma(u) on the nodes, Voigt order, (6, Nz, Ny, Nx)."""
    A, B, _ = moduli(mu, nu)
    lam = A - 2.0 * B
    grads = [_grad(u[c], d) for c in range(3)]          # grads[c][a] = d u_c / d x_a
    div = grads[0][0] + grads[1][1] + grads[2][2]
    out = np.array(sigma_dis, dtype=np.float64, copy=True)
    for v, (a, b) in enumerate(VOIGT_PAIRS):
        eps = 0.5 * (grads[a][b] + grads[b][a])
        out[v] += 2.0 * B * eps + (lam * div if a == b else 0.0)
    return out
