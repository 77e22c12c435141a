"""Pins of the oracle's stress relaxation under free surfaces, Sec. 5,
Eq. (14)-(18) (no GPU).

* closed form: a load uniform in the plane and linear in z relaxes to zero
  z-traction everywhere and sigma_xx = sigma^dis_xx - nu / (1 - nu) sigma^dis_zz
  (every difference of the scheme is exact on that solution);
* manufactured solution: with sigma^dis = -sigma(u*) for a smooth periodic u*,
  the relaxed total stress vanishes up to the discretisation error, which
  falls by about 4 when the cells are halved (second order);
* the stencil against Eq. (14) and the force against Eq. (15) on smooth
  fields (second-order consistency);
* after any ghost update the total sigma_xz, sigma_yz, sigma_zz vanish on
  both surfaces (Eq. 16b), for an arbitrary state;
* a circular shift of the load shifts the displacement, and the iteration is
  linear in the load.
"""
import numpy as np
import pytest

from oracle.relax import (VOIGT_PAIRS, initial_state, load_terms, moduli, navier, paper_time_step, relax,
                          set_ghosts, total_stress, update_norm)

MU, NU = 1.0, 0.3


def _nodes(n, d):
    nx, ny, nz = n
    z = np.arange(nz) * d[2]
    y = np.arange(ny) * d[1]
    x = np.arange(nx) * d[0]
    return np.meshgrid(z, y, x, indexing="ij")


def _relax_to_rest(sig, d, mu, nu, chunk=500, tol=1e-11, max_chunks=80):
    u = None
    for _ in range(max_chunks):
        u = relax(sig, d, mu, nu, chunk, u=u)
        if update_norm(u, sig, d, mu, nu) <= tol * max(1.0, np.abs(sig).max()):
            return u
    raise AssertionError("relaxation did not come to rest")


def test_laterally_uniform_linear_load_gives_the_closed_form():
    n, d = (4, 3, 9), (1.0, 1.0, 0.5)
    Z, _, _ = _nodes(n, d)
    rng = np.random.default_rng(3)
    a, b = rng.uniform(-1, 1, 6), rng.uniform(-1, 1, 6)
    sig = np.stack([a[v] + b[v] * Z for v in range(6)])
    u = _relax_to_rest(sig, d, MU, NU)
    tot = total_stress(u, sig, d, MU, NU)
    scale = np.abs(sig).max()
    for v in (2, 3, 4):                                   # zz, yz, xz
        assert np.abs(tot[v]).max() < 1e-9 * scale
    k = NU / (1.0 - NU)
    assert np.abs(tot[0] - (sig[0] - k * sig[2])).max() < 1e-9 * scale
    assert np.abs(tot[1] - (sig[1] - k * sig[2])).max() < 1e-9 * scale
    assert np.abs(tot[5] - sig[5]).max() < 1e-9 * scale


def _manufactured(n, d, mu, nu):
    """u* periodic in x, y (period Nx dx, Ny dy), smooth in z, and
    sigma^dis = -sigma(u*) at the nodes."""
    Z, Y, X = _nodes(n, d)
    Lx, Ly = n[0] * d[0], n[1] * d[1]
    kx, ky, kz = 2 * np.pi / Lx, 2 * np.pi / Ly, 1.3
    sx, cx = np.sin(kx * X), np.cos(kx * X)
    sy, cy = np.sin(ky * Y), np.cos(ky * Y)
    sz, cz = np.sin(kz * Z), np.cos(kz * Z)
    # u* and its gradient G[c][a] = d u_c / d x_a
    u = [sx * cy * cz, cx * sy * sz, sx * sy * cz]
    G = [[kx * cx * cy * cz, -ky * sx * sy * cz, -kz * sx * cy * sz],
         [-kx * sx * sy * sz, ky * cx * cy * sz, kz * cx * sy * cz],
         [kx * cx * sy * cz, ky * sx * cy * cz, -kz * sx * sy * sz]]
    A, B, _ = moduli(mu, nu)
    lam = A - 2 * B
    div = G[0][0] + G[1][1] + G[2][2]
    sig = np.stack([-(B * (G[a][b] + G[b][a]) + (lam * div if a == b else 0.0)) for a, b in VOIGT_PAIRS])
    return sig


def test_manufactured_solution_converges_at_second_order():
    errs = []
    for m in (8, 16):
        h = 1.0 / m
        n, d = (m, m, m // 2 + 1), (h, h, h)
        sig = _manufactured(n, d, MU, NU)
        u = _relax_to_rest(sig, d, MU, NU, tol=1e-10)
        tot = total_stress(u, sig, d, MU, NU)
        errs.append(np.abs(tot).max() / np.abs(sig).max())
    ratio = errs[0] / errs[1]
    assert errs[1] < 0.05 and 3.0 < ratio < 5.0, (errs, ratio)


def test_stencil_and_force_are_second_order_consistent():
    # smooth periodic field sampled on a grid with one extra layer below and
    # above, so that the ghost layers hold the field itself
    A, B, _ = moduli(MU, NU)
    res = []
    for m in (8, 16):
        h = 1.0 / m
        n, d = (m, m, m // 2 + 1), (h, h, h)
        nx, ny, nz = n
        z = (np.arange(nz + 2) - 1) * h
        Z, Y, X = np.meshgrid(z, np.arange(ny) * h, np.arange(nx) * h, indexing="ij")
        k = 2 * np.pi
        u = np.stack([np.sin(k * X) * np.cos(k * Y) * np.exp(Z), np.cos(k * X) * np.sin(k * Y) * Z,
                      np.sin(k * X + k * Y) * np.cos(Z)])
        got = navier(u, d, MU, NU)
        # analytic (A - B) grad div u + B lap u at the real nodes
        Zc, Yc, Xc = Z[1:-1], Y[1:-1], X[1:-1]
        s, c = np.sin, np.cos
        e = np.exp(Zc)
        ux_xx = -k * k * s(k * Xc) * c(k * Yc) * e
        ux_yy = -k * k * s(k * Xc) * c(k * Yc) * e
        ux_zz = s(k * Xc) * c(k * Yc) * e
        uy_xx = -k * k * c(k * Xc) * s(k * Yc) * Zc
        uy_yy = -k * k * c(k * Xc) * s(k * Yc) * Zc
        uy_zz = 0.0 * Zc
        w = k * Xc + k * Yc
        uz_xx = -k * k * s(w) * c(Zc)
        uz_yy = -k * k * s(w) * c(Zc)
        uz_zz = -s(w) * c(Zc)
        ux_xy = -k * k * c(k * Xc) * s(k * Yc) * e
        ux_xz = k * c(k * Xc) * c(k * Yc) * e
        uy_xy = -k * k * s(k * Xc) * c(k * Yc) * Zc
        uy_yz = k * c(k * Xc) * c(k * Yc)
        uz_xz = -k * c(w) * s(Zc)
        uz_yz = -k * c(w) * s(Zc)
        gd = [ux_xx + uy_xy + uz_xz, ux_xy + uy_yy + uz_yz, ux_xz + uy_yz + uz_zz]
        lap = [ux_xx + ux_yy + ux_zz, uy_xx + uy_yy + uy_zz, uz_xx + uz_yy + uz_zz]
        want = np.stack([(A - B) * gd[a] + B * lap[a] for a in range(3)])
        e_op = np.abs(got - want).max() / np.abs(want).max()
        # force: div of a smooth stress field
        sig = np.stack([s(k * Xc) * e, c(k * Yc) * Zc, s(w) * Zc ** 2, c(k * Xc) * Zc, s(k * Yc) * e, c(w) * Zc])
        f, _ = load_terms(sig, d, MU, NU)
        # f_a = d sigma_ax / dx + d sigma_ay / dy + d sigma_az / dz (the xz component
        # depends on y and z only, the yz component on x and z only)
        fw = np.stack([k * c(k * Xc) * e - k * s(w) * Zc + s(k * Yc) * e,
                       -k * s(w) * Zc - k * s(k * Yc) * Zc + c(k * Xc),
                       0.0 * Zc + 0.0 * Zc + 2 * s(w) * Zc])
        e_f = np.abs(f - fw).max() / np.abs(fw).max()
        surf = [0, nz - 1]
        e_fs = np.abs(f[:, surf] - fw[:, surf]).max() / np.abs(fw).max()
        res.append((e_op, e_f, e_fs))
    for i in range(3):
        ratio = res[0][i] / res[1][i]
        assert 3.0 < ratio < 5.0, (res, i)


def test_force_is_exact_for_a_quadratic_profile():
    # the z differences of Eq. (15), central inside and one-sided on the
    # surfaces, are exact for sigma^dis quadratic in z
    n, d = (3, 2, 6), (1.0, 1.0, 0.4)
    Z, _, _ = _nodes(n, d)
    rng = np.random.default_rng(4)
    c = rng.uniform(-1, 1, size=(6, 3))
    sig = np.stack([c[v, 0] + c[v, 1] * Z + c[v, 2] * Z ** 2 for v in range(6)])
    f, _ = load_terms(sig, d, MU, NU)
    dz = lambda v: c[v, 1] + 2 * c[v, 2] * Z
    want = np.stack([dz(4), dz(3), dz(2)])               # d sigma_xz, d sigma_yz, d sigma_zz / dz
    assert np.abs(f - want).max() < 1e-13


@pytest.mark.parametrize("nu", [0.3, 0.2])
def test_surfaces_are_traction_free_after_any_ghost_update(nu):
    n, d = (6, 5, 4), (1.0, 1.5, 0.7)
    rng = np.random.default_rng(8)
    sig = rng.uniform(-1, 1, size=(6, n[2], n[1], n[0]))
    u, f, phi = initial_state(sig, d, MU, nu)
    u[:, 1:-1] = rng.uniform(-1, 1, size=u[:, 1:-1].shape)        # any state of the nodes
    set_ghosts(u, phi, d, nu)
    tot = total_stress(u, sig, d, MU, nu)
    for v in (2, 3, 4):
        for k in (0, n[2] - 1):
            assert np.abs(tot[v, k]).max() < 1e-13 * np.abs(sig).max() * 10
    # inside the film the traction is not zero for an arbitrary state
    assert np.abs(tot[2, 1:-1]).max() > 1e-3


def test_shift_covariance_and_linearity():
    n, d = (6, 4, 5), (1.0, 1.0, 1.0)
    rng = np.random.default_rng(9)
    s1 = rng.uniform(-1, 1, size=(6, n[2], n[1], n[0]))
    s2 = rng.uniform(-1, 1, size=(6, n[2], n[1], n[0]))
    u1 = relax(s1, d, MU, NU, 40)
    u2 = relax(s2, d, MU, NU, 40)
    u12 = relax(2.0 * s1 - 0.5 * s2, d, MU, NU, 40)
    assert np.abs(u12 - (2.0 * u1 - 0.5 * u2)).max() < 1e-12 * np.abs(u12).max()
    ur = relax(np.roll(s1, (2, 1), axis=(3, 2)), d, MU, NU, 40)
    assert np.abs(ur - np.roll(u1, (2, 1), axis=(3, 2))).max() < 1e-12 * np.abs(u1).max()


def test_paper_time_step():
    A, B, _ = moduli(MU, NU)
    assert abs(paper_time_step((1.0, 2.0, 0.5), MU, NU) - 0.25 / (5 * A - 3 * B)) < 1e-15
    # A = lambda + 2 mu, B = mu
    assert abs(B - MU) < 1e-15 and abs(A - (2 * MU * NU / (1 - 2 * NU) + 2 * MU)) < 1e-12
