"""Pins of the oracle's segment stress against closed forms and exact
properties (no GPU). The textbook fields of infinite straight edge and screw
dislocations are the classical results the paper starts from (Sec. 1, Sec. 2.2):
with D = mu b / (2 pi (1 - nu)), for t = e_z and b = e_x
    sxx = -D y (3x^2 + y^2)/r^4, syy = D y (x^2 - y^2)/r^4, szz = -2 nu D y/r^2,
    sxy =  D x (x^2 - y^2)/r^4,  sxz = syz = 0,
and for b = e_z (screw)  sxz = -mu y/(2 pi r^2), syz = mu x/(2 pi r^2).
A long centred segment approaches these at its mid-plane with an error of
order (r/H)^2.
"""
import numpy as np
import pytest

from oracle.segment import (VOIGT, segment_stress_vertical, segment_stress_general,
                            segment_stress, chord_length)

MU, NU = 1.7, 0.27


def _to_tensor(s6):
    T = np.zeros(s6.shape[:-1] + (3, 3))
    for v, (i, j) in enumerate(VOIGT):
        T[..., i, j] = s6[..., v]
        T[..., j, i] = s6[..., v]
    return T


def _to_voigt(T):
    return np.stack([T[..., i, j] for (i, j) in VOIGT], axis=-1)


def textbook_edge_x(p, mu, nu):
    x, y = p[..., 0], p[..., 1]
    r2 = x * x + y * y
    D = mu / (2 * np.pi * (1 - nu))
    z = np.zeros_like(x)
    return np.stack([-D * y * (3 * x * x + y * y) / r2 ** 2, D * y * (x * x - y * y) / r2 ** 2,
                     -2 * nu * D * y / r2, z, z, D * x * (x * x - y * y) / r2 ** 2], axis=-1)


def textbook_screw(p, mu):
    x, y = p[..., 0], p[..., 1]
    r2 = x * x + y * y
    z = np.zeros_like(x)
    return np.stack([z, z, z, mu * x / (2 * np.pi * r2), -mu * y / (2 * np.pi * r2), z], axis=-1)


def _rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


@pytest.fixture(scope="module")
def midplane_points():
    rng = np.random.default_rng(11)
    r = rng.uniform(0.5, 5.0, size=64)
    a = rng.uniform(0, 2 * np.pi, size=64)
    return np.stack([r * np.cos(a), r * np.sin(a), np.zeros(64)], axis=-1)


@pytest.mark.parametrize("impl", ["eq4", "eq6"])
def test_long_segment_is_textbook_edge_and_screw(impl, midplane_points):
    H = 1e5
    p = midplane_points
    if impl == "eq4":
        s = segment_stress_vertical(p, H, MU, NU)
    else:
        s = segment_stress_general(p, H, [0, 0, 1], MU, NU)
    scale = MU / np.sum(p[:, :2] ** 2, axis=-1) ** 0.5
    err_edge = np.abs(s[..., 0] - textbook_edge_x(p, MU, NU)).max(axis=-1) / scale
    err_screw = np.abs(s[..., 2] - textbook_screw(p, MU)).max(axis=-1) / scale
    assert err_edge.max() < 1e-8 and err_screw.max() < 1e-8
    # b = e_y: the e_x field rotated by +90 degrees about z
    Q = _rot_z(np.pi / 2)
    ref = _to_voigt(Q @ _to_tensor(textbook_edge_x(p @ Q, MU, NU)) @ Q.T)
    err_y = np.abs(s[..., 1] - ref).max(axis=-1) / scale
    assert err_y.max() < 1e-8


def test_mid_plane_error_shrinks_like_r_over_h_squared():
    p = np.array([[1.3, 0.4, 0.0]])
    errs = []
    for H in (40.0, 80.0, 160.0):
        s = segment_stress_vertical(p, H, MU, NU)[0, :, 0]
        errs.append(np.abs(s - textbook_edge_x(p, MU, NU)[0]).max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_eq4_and_eq6_agree_for_vertical_lines():
    rng = np.random.default_rng(5)
    p = rng.normal(size=(4000, 3)) * 2.5
    for h in (0.25, 1.0, 3.0):
        keep = ~((np.abs(p[:, 2]) < 0.5 * h) & (np.hypot(p[:, 0], p[:, 1]) < 1e-3))
        a = segment_stress_vertical(p[keep], h, MU, NU)
        b = segment_stress_general(p[keep], h, [0, 0, 1], MU, NU)
        rel = np.abs(a - b).max(axis=(1, 2)) / np.abs(b).max(axis=(1, 2))
        assert rel.max() < 1e-12


def test_on_axis_points_beyond_the_ends():
    p = np.array([[0, 0, -1.5], [0, 0, 2.0], [0, 0, -0.75]])
    a = segment_stress_vertical(p, 1.0, MU, NU)
    b = segment_stress_general(p, 1.0, [0, 0, 1], MU, NU)
    assert np.all(np.isfinite(a)) and np.allclose(a, b, rtol=1e-13, atol=1e-15)
    # on the axis only the xz (b_y) and yz (b_x) components survive
    mask = np.ones((6, 3), dtype=bool)
    mask[3, 0] = mask[4, 1] = False
    assert np.abs(a[:, mask]).max() == 0.0


def test_rotation_covariance_of_eq6():
    rng = np.random.default_rng(6)
    # tilted line: the vertical segment rotated by Q
    th = np.radians(15.6)
    Q = np.array([[np.cos(th), 0, np.sin(th)], [0, 1, 0], [-np.sin(th), 0, np.cos(th)]])
    Q = _rot_z(0.7) @ Q
    t = Q @ np.array([0, 0, 1.0])
    p = rng.normal(size=(500, 3)) * 2.0
    h = 0.9
    gen = segment_stress_general(p, h, t, MU, NU)               # (M, 6, 3)
    loc = segment_stress_vertical(p @ Q, h, MU, NU)             # points in the local frame
    for g in range(3):
        b_loc = Q.T[:, g]                                      # e_g expressed in local axes
        s_loc = np.einsum("mvk,k->mv", loc, b_loc)
        ref = _to_voigt(Q @ _to_tensor(s_loc) @ Q.T)
        rel = np.abs(gen[..., g] - ref).max(axis=-1) / np.abs(ref).max(axis=-1)
        assert rel.max() < 1e-12


def test_inversion_oddness_and_collinear_superposition():
    rng = np.random.default_rng(7)
    t = np.array([0.3, -0.5, 0.81])
    t /= np.linalg.norm(t)
    p = rng.normal(size=(300, 3)) * 2.0
    s = segment_stress_general(p, 1.1, t, MU, NU)
    assert np.abs(s + segment_stress_general(-p, 1.1, t, MU, NU)).max() < 1e-13 * np.abs(s).max()
    # a segment of length 2h is the sum of its two halves (centres at -/+ h/2 along t)
    h = 0.8
    whole = segment_stress_general(p, 2 * h, t, MU, NU)
    halves = (segment_stress_general(p + 0.5 * h * t, h, t, MU, NU)
              + segment_stress_general(p - 0.5 * h * t, h, t, MU, NU))
    rel = np.abs(whole - halves).max(axis=(1, 2)) / np.abs(whole).max(axis=(1, 2))
    assert rel.max() < 1e-11
    sv = segment_stress_vertical(p, 2 * h, MU, NU)
    hv = segment_stress_vertical(p + [0, 0, 0.5 * h], h, MU, NU) + segment_stress_vertical(p - [0, 0, 0.5 * h], h, MU, NU)
    assert (np.abs(sv - hv).max(axis=(1, 2)) / np.abs(sv).max(axis=(1, 2))).max() < 1e-11


def test_far_field_decay_powers():
    # Sec. 4: for a vertical segment sxx, syy, szz, sxy fall off like dl/r^2,
    # sxz and syz like dl/r^3 (in-plane distance, off the mid-plane).
    r = np.array([200.0, 400.0])
    p = np.stack([r * np.cos(0.3), r * np.sin(0.3), np.full(2, 0.37)], axis=-1)
    s = segment_stress_vertical(p, 1.0, MU, NU)
    with np.errstate(divide="ignore", invalid="ignore"):
        slope = np.log(np.abs(s[1]) / np.abs(s[0])) / np.log(2.0)
    assert np.allclose(slope[[0, 1, 5], 0], -2.0, atol=0.02)     # xx, yy, xy from b_x
    assert np.allclose(slope[4, 0], -3.0, atol=0.02)              # xz from b_x


def test_chord_length():
    assert chord_length((1, 1, 4), (0, 0, 1)) == 4.0
    assert chord_length((1, 2, 3), (1, 0, 0)) == 1.0
    a = np.radians(15.6)
    assert np.isclose(chord_length((1, 1, 2), (np.sin(a), 0, np.cos(a))), min(1 / np.sin(a), 2 / np.cos(a)))


def test_dispatch_uses_eq4_for_e_z_only():
    p = np.array([[0.4, 0.3, -0.2]])
    assert np.array_equal(segment_stress(p, 1.0, [0, 0, 2.0], MU, NU), segment_stress_vertical(p, 1.0, MU, NU))
    t = np.array([0.1, 0, 1.0])
    assert np.array_equal(segment_stress(p, 1.0, t, MU, NU),
                          segment_stress_general(p, 1.0, t / np.linalg.norm(t), MU, NU))
