"""Stress of a finite straight dislocation segment (Sec. 2.2 of the paper).

Test infrastructure (see ``oracle/__init__.py``): only tests, smoke() and the
bench's cpu_baseline use this module.

Conventions used throughout the oracle
--------------------------------------
* Points are given relative to the segment centre; the segment runs from
  A = -(h/2) t to B = +(h/2) t, so t points from A to B.
* Results are returned for the three unit Burgers vectors b = e_x, e_y, e_z
  at once: shape ``(..., 6, 3)`` with the last axis the Burgers component
  gamma. Both formulas are linear in b (Eq. 4a and Eq. 6), so the stress of
  any b is ``sigma @ b``.
* The six stress components are in Voigt order (xx, yy, zz, yz, xz, xy).

Readings of the paper applied here
----------------------------------
* Eq. (4a) is the printed formula set for a semi-infinite line along z ending
  at z'; Eq. (5) takes the finite segment as sigma(z'_B) - sigma(z'_A). The
  set is analytic wherever the point is off the z axis, so it is evaluated
  everywhere off the axis, with R + lambda rewritten as r^2 / (R - lambda)
  when lambda < 0 to avoid cancellation (the same quantity, computed stably).
  Points above the segment centre are evaluated through the inversion
  oddness of a centred segment, sigma(p) = -sigma(-p); this keeps the
  evaluation away from the half-line's singular ray, which is the role the
  paper gives to the other two (unprinted) formula sets.
* Eq. (6) is evaluated at each end point E with R = p - E (vector from the
  end point to the observation point), R_t = R + |R| t, L = R.t and
  rho = R - L t; the bracket |_A^B is the value at B minus the value at A.
  When the point lies behind the segment centre ((p . t) < 0) the same
  physical segment is described with t -> -t, b -> -b and the end points
  swapped, which moves the singular ray R_t = 0 to the other side.
"""
import numpy as np

# Voigt order (xx, yy, zz, yz, xz, xy) as (row, column) index pairs.
VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def chord_length(box, t):
    """Length of the chord through the centre of a box of edge lengths ``box``
    along the unit direction ``t``: min over axes with t_a != 0 of box_a/|t_a|.

    This is the segment length Delta l that represents the dislocations of a
    cell (or subcell) of that box. The paper fixes it as the prism height for
    lines along the prism (Sec. 2.1); for oblique lines this is the reading
    taken (the segment stays inside the cell and touches its faces).
    """
    box = np.asarray(box, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    vals = [box[a] / abs(t[a]) for a in range(3) if t[a] != 0.0]
    return float(min(vals))


def _semi_infinite_vertical(x, y, lam, mu, nu):
    """Eq. (4a)-(4c): stress of the semi-infinite vertical line ending at z',
    for the three unit Burgers vectors, as a function of the in-plane offset
    (x, y) and lambda = z' - z. Returns (..., 6, 3)."""
    s0 = mu / (4.0 * np.pi * (1.0 - nu))
    r2 = x * x + y * y
    R2 = r2 + lam * lam
    R = np.sqrt(R2)
    R3 = R2 * R
    # R + lambda, written as r^2/(R - lambda) where lambda < 0 (same value).
    with np.errstate(divide="ignore", invalid="ignore"):
        r_plus = np.where(lam >= 0.0, R + lam, r2 / (R - lam))
    Rl2 = R * r_plus                                   # Eq. (4b): R_{lambda+}^2
    Sx = x * x / R2 + x * x / Rl2                      # Eq. (4c)
    Sy = y * y / R2 + y * y / Rl2
    out = np.zeros(np.shape(x) + (6, 3))
    # b = e_x
    out[..., 0, 0] = y / Rl2 * (1.0 + Sx)                       # xx
    out[..., 1, 0] = -y / Rl2 * (1.0 - Sy)                      # yy
    out[..., 2, 0] = y * (2.0 * nu / Rl2 + lam / R3)            # zz
    out[..., 3, 0] = nu / R - y * y / R3                        # yz
    out[..., 4, 0] = -x * y / R3                                # xz
    out[..., 5, 0] = -x / Rl2 * (1.0 - Sy)                      # xy
    # b = e_y
    out[..., 0, 1] = x / Rl2 * (1.0 - Sx)
    out[..., 1, 1] = -x / Rl2 * (1.0 + Sy)
    out[..., 2, 1] = -x * (2.0 * nu / Rl2 + lam / R3)
    out[..., 3, 1] = x * y / R3
    out[..., 4, 1] = -(nu / R - x * x / R3)
    out[..., 5, 1] = y / Rl2 * (1.0 - Sx)
    # b = e_z
    out[..., 3, 2] = -x * (1.0 - nu) / Rl2
    out[..., 4, 2] = y * (1.0 - nu) / Rl2
    return s0 * out


def segment_stress_vertical(p, h, mu, nu):
    """Stress of the segment of length ``h`` along +z centred at the origin,
    Eq. (4a)-(4c) combined by Eq. (5). ``p``: (..., 3) observation points.
    Returns (..., 6, 3). Singular on the segment itself."""
    p = np.asarray(p, dtype=np.float64)
    above = p[..., 2] > 0.0
    q = np.where(above[..., None], -p, p)          # evaluate at or below the centre
    x, y, z = q[..., 0], q[..., 1], q[..., 2]
    zB, zA = 0.5 * h, -0.5 * h
    sig = (_semi_infinite_vertical(x, y, zB - z, mu, nu)
           - _semi_infinite_vertical(x, y, zA - z, mu, nu))       # Eq. (5)
    return np.where(above[..., None, None], -sig, sig)


def _eq6_end(R, b, t, mu, nu):
    """Value of the bracket of Eq. (6) at one end point, R = p - E.
    ``R``: (..., 3); ``b``, ``t``: (3,). Returns (..., 3, 3)."""
    Rn = np.sqrt(np.sum(R * R, axis=-1))
    L = R @ t                                           # L = R . t
    rho = R - L[..., None] * t                          # rho = R - L t
    rho2 = np.sum(rho * rho, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        r_plus = np.where(L >= 0.0, Rn + L, rho2 / (Rn - L))   # |R| + L, stably
    Y = rho + r_plus[..., None] * t                     # R_t = R + |R| t
    Y2 = np.sum(Y * Y, axis=-1)
    # Eq. (7a)
    Phi = (2.0 / Y2)[..., None, None] * (
        rho[..., :, None] * Y[..., None, :] + Y[..., :, None] * rho[..., None, :]
        + (L / Rn)[..., None, None] * Y[..., :, None] * Y[..., None, :])
    # Eq. (7b) operators
    bxY = np.cross(b, Y)
    bxt = np.cross(b, t)
    sym_bYt = 0.5 * (bxY[..., :, None] * t[None, :] + t[:, None] * bxY[..., None, :])
    sym_btY = 0.5 * (bxt[:, None] * Y[..., None, :] + Y[..., :, None] * bxt[None, :])
    trip = np.cross(Y, t) @ b                           # (b, R_t, t) = b . (R_t x t)
    eye_tt = np.eye(3) + np.outer(t, t)
    bracket = (sym_bYt - sym_btY / (1.0 - nu)
               - (trip / (2.0 * (1.0 - nu)))[..., None, None] * (eye_tt + Phi))
    return (mu / (np.pi * Y2))[..., None, None] * bracket


def segment_stress_general(p, h, t, mu, nu):
    """Stress of the segment of length ``h`` along the unit vector ``t``,
    centred at the origin, by the coordinate-free Eq. (6)-(7).
    ``p``: (..., 3). Returns (..., 6, 3) (Voigt x Burgers component)."""
    p = np.asarray(p, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    t = t / np.linalg.norm(t)
    A = -0.5 * h * t
    B = 0.5 * h * t
    front = (p @ t) >= 0.0
    out = np.zeros(p.shape[:-1] + (6, 3))
    for g in range(3):
        b = np.zeros(3)
        b[g] = 1.0
        # both forms are computed and the valid one kept; the other may sit on
        # its singular ray, hence the silenced floating-point warnings
        with np.errstate(divide="ignore", invalid="ignore"):
            fwd = _eq6_end(p - B, b, t, mu, nu) - _eq6_end(p - A, b, t, mu, nu)
            # same segment as B->A with t -> -t, b -> -b
            rev = _eq6_end(p - A, -b, -t, mu, nu) - _eq6_end(p - B, -b, -t, mu, nu)
        full = np.where(front[..., None, None], fwd, rev)
        for v, (i, j) in enumerate(VOIGT):
            out[..., v, g] = full[..., i, j]
    return out


def segment_stress(p, h, t, mu, nu):
    """Segment stress with the formula the paper gives for the line
    direction: Eq. (4a)+(5) when t is exactly e_z, Eq. (6) otherwise."""
    t = np.asarray(t, dtype=np.float64)
    t = t / np.linalg.norm(t)
    if t[0] == 0.0 and t[1] == 0.0 and t[2] > 0.0:
        return segment_stress_vertical(p, h, mu, nu)
    return segment_stress_general(p, h, t, mu, nu)
