"""Pins of the oracle's periodic boundary conditions, Eq. (12)-(13) (no GPU).

* brute force: the replica-shell sum written as a sum over explicit images of
  every source cell inside a square window centred on the target, built from
  the open-boundary kernel alone;
* reduction to the open boundary: without shells and with every pair offset
  below half a period, the periodic sum is the open-boundary sum; with no
  periodic axis it is the open-boundary sum everywhere;
* exact symmetries: F is odd under inversion and N-periodic, so the stress
  moves with a circular shift of the density;
* a density that is uniform in the layer plane gives no in-plane-odd stress
  for vertical lines (only the even xz/yz pattern survives the plane sum);
* the FFT reference (circular convolution at the period) matches the direct
  periodic sum;
* the shell sums converge: 15 and 20 shells agree to better than 3 %.
"""
import itertools

import numpy as np
import pytest

from oracle.direct import stress_direct
from oracle.kernel import KernelGeometry, interaction_kernel
from oracle.periodic import periodic_kernel, stress_direct_periodic, stress_fft_reference_periodic

TILT = (np.sin(np.radians(15.6)), 0.0, np.cos(np.radians(15.6)))


def _rho(seed, n, L):
    nx, ny, nz = n
    return np.random.default_rng(seed).uniform(-1, 1, size=(3 * L, nz, ny, nx))


def _window_weight(D, half):
    """1 strictly inside |D| < half, 1/2 on |D| == half, 0 outside."""
    a = abs(D)
    return 1.0 if a < half else (0.5 if a == half else 0.0)


def _brute_window(rho, d, lines, mu, nu, shells, periodic):
    """Each target sees every image of every source cell whose offset lies in
    the window |Delta_a| <= (shells + 1/2) N_a of each periodic axis, at half
    weight on the window's edge."""
    C, nz, ny, nx = rho.shape
    geoms = [KernelGeometry(d=d, t=tuple(t), mu=mu, nu=nu) for t in lines]
    reach = shells + 1
    img_x = range(-reach, reach + 1) if periodic[0] else [0]
    img_y = range(-reach, reach + 1) if periodic[1] else [0]
    out = np.zeros((6, nz, ny, nx))
    for k0, j0, i0 in itertools.product(range(nz), range(ny), range(nx)):
        offs, wts, src = [], [], []
        for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
            for a in img_x:
                for b in img_y:
                    D = (i0 - (i + a * nx), j0 - (j + b * ny), k0 - k)
                    w = 1.0
                    if periodic[0]:
                        w *= _window_weight(D[0], (shells + 0.5) * nx)
                    if periodic[1]:
                        w *= _window_weight(D[1], (shells + 0.5) * ny)
                    if w:
                        offs.append(D)
                        wts.append(w)
                        src.append((k, j, i))
        offs = np.array(offs)
        wts = np.array(wts)
        src = np.array(src)
        for l, g in enumerate(geoms):
            K = interaction_kernel(g, offs)                       # (M, 6, 3)
            r = rho[3 * l:3 * l + 3, src[:, 0], src[:, 1], src[:, 2]]   # (3, M)
            out[:, k0, j0, i0] += np.einsum("m,mvg,gm->v", wts, K, r)
    return out


@pytest.mark.parametrize("n,periodic,shells", [((4, 3, 2), (True, True), 2),
                                                 ((3, 4, 2), (True, False), 3),
                                                 ((4, 2, 2), (False, True), 1)])
def test_periodic_sum_equals_image_window_brute_force(n, periodic, shells):
    lines = np.array([(0, 0, 1), TILT])
    d = (1.0, 1.5, 2.0)
    rho = _rho(11, n, 2)
    got = stress_direct_periodic(rho, d, lines, 1.1, 0.3, periodic=periodic, shells=shells)
    ref = _brute_window(rho, d, lines, 1.1, 0.3, shells, periodic)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_no_periodic_axis_is_the_open_boundary_sum():
    lines = np.array([TILT])
    rho = _rho(2, (4, 3, 3), 1)
    a = stress_direct_periodic(rho, (1.0, 1.0, 1.5), lines, 1.0, 0.3, periodic=(False, False), shells=4)
    b = stress_direct(rho, (1.0, 1.0, 1.5), lines, 1.0, 0.3)
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


def test_zero_shells_and_small_support_is_the_open_boundary_sum():
    # density inside a 3 x 3 in-plane block of an 8 x 8 period: every pair
    # offset among those cells is below half a period, so no image enters
    lines = np.array([(0, 0, 1), TILT])
    rho = np.zeros((6, 2, 8, 8))
    rho[:, :, 2:5, 1:4] = _rho(5, (3, 3, 2), 2)
    d = (1.0, 1.5, 2.0)
    a = stress_direct_periodic(rho, d, lines, 1.0, 0.3, periodic=(True, True), shells=0)
    b = stress_direct(rho, d, lines, 1.0, 0.3)
    sl = (slice(None), slice(None), slice(2, 5), slice(1, 4))
    assert np.abs(a[sl] - b[sl]).max() < 1e-13 * np.abs(b[sl]).max()
    # outside the block, distances wrap, so the two differ there
    assert np.abs(a - b).max() > 1e-6 * np.abs(b).max()


@pytest.mark.parametrize("n", [(4, 6, 3), (5, 3, 2)])
def test_periodic_kernel_is_odd_and_periodic(n):
    nx, ny, nz = n
    g = KernelGeometry(d=(1.0, 1.5, 2.0), t=TILT, mu=1.0, nu=0.3)
    gz, gy, gx = np.meshgrid(np.arange(-(nz - 1), nz), np.arange(-ny, ny + 1), np.arange(-nx, nx + 1),
                             indexing="ij")
    offs = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=-1)
    F = periodic_kernel(g, offs, n, (True, True), 3)
    Fneg = periodic_kernel(g, -offs, n, (True, True), 3)
    scale = np.abs(F).max()
    assert np.abs(F + Fneg).max() < 1e-14 * scale
    shifted = offs + np.array([nx, -2 * ny, 0])
    assert np.abs(periodic_kernel(g, shifted, n, (True, True), 3) - F).max() < 1e-14 * scale
    zero = np.all(offs == 0, axis=-1)
    assert np.abs(F[zero]).max() < 1e-14 * scale


def test_circular_shift_moves_the_stress():
    lines = np.array([(0, 0, 1), TILT])
    rho = _rho(7, (5, 4, 2), 2)
    d = (1.0, 1.0, 2.0)
    a = stress_direct_periodic(rho, d, lines, 1.0, 0.3, shells=2)
    b = stress_direct_periodic(np.roll(rho, (1, 3), axis=(2, 3)), d, lines, 1.0, 0.3, shells=2)
    assert np.abs(np.roll(a, (1, 3), axis=(2, 3)) - b).max() < 1e-12 * np.abs(a).max()


def test_uniform_plane_density_of_vertical_lines_has_no_odd_components():
    # in-plane inversion maps the set of images onto itself only with the
    # centred, half-weighted window: xx, yy, zz and xy cancel pairwise
    nz = 3
    prof = np.array([1.0, 0.4, -0.2])
    rho = np.zeros((3, nz, 4, 6))
    rho[0] = prof[:, None, None]
    rho[1] = 0.5 * prof[:, None, None]
    out = stress_direct_periodic(rho, (1.0, 1.0, 3.0), [(0, 0, 1)], 1.0, 0.3, shells=3)
    odd = out[[0, 1, 2, 5]]
    even = out[[3, 4]]
    assert np.abs(even).max() > 1e-3
    assert np.abs(odd).max() < 1e-12 * np.abs(even).max()
    # and the field is the same in every column of the plane
    assert np.abs(out - out[:, :, :1, :1]).max() < 1e-12 * np.abs(even).max()


@pytest.mark.parametrize("periodic", [(True, True), (True, False)])
def test_fft_reference_matches_direct_periodic_sum(periodic):
    lines = np.array([(0, 0, 1), TILT])
    rho = _rho(9, (4, 6, 3), 2)
    d = (1.0, 1.5, 2.0)
    a = stress_direct_periodic(rho, d, lines, 1.0, 0.3, periodic=periodic, shells=2)
    b = stress_fft_reference_periodic(rho, d, lines, 1.0, 0.3, periodic=periodic, shells=2)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-13


def test_replica_shells_converge_within_three_percent():
    # vertical segment in a 32 x 32 period, a few offsets in the cell: the
    # sums at 15 and 20 shells agree to better than 3 % (Sec. 4, Fig. 7)
    n = (32, 32, 8)
    g = KernelGeometry(d=(1.0, 1.0, 1.0), t=(0, 0, 1), mu=1.0, nu=0.3)
    offs = np.array([[3, 1, 0], [7, -4, 2], [-10, 5, 1], [1, 0, 3]])
    F15 = periodic_kernel(g, offs, n, (True, True), 15)
    F20 = periodic_kernel(g, offs, n, (True, True), 20)
    F10 = periodic_kernel(g, offs, n, (True, True), 10)
    for m in range(len(offs)):
        nrm = np.linalg.norm(F20[m])
        assert np.linalg.norm(F15[m] - F20[m]) < 0.03 * nrm
        assert np.linalg.norm(F15[m] - F20[m]) < np.linalg.norm(F10[m] - F20[m])


def test_sampled_targets_match_the_full_periodic_sum():
    lines = np.array([(0, 0, 1), TILT])
    rho = _rho(13, (4, 4, 3), 2)
    rho[:, :, 1, :] = 0.0                         # some empty source cells
    d = (1.0, 1.5, 2.0)
    full = stress_direct_periodic(rho, d, lines, 1.0, 0.3, periodic=(True, False), shells=2)
    tg = np.array([[0, 0, 0], [3, 1, 2], [2, 3, 1], [1, 2, 0]])
    samp = stress_direct_periodic(rho, d, lines, 1.0, 0.3, periodic=(True, False), shells=2, targets=tg)
    assert np.abs(samp - full[:, tg[:, 2], tg[:, 1], tg[:, 0]]).max() < 1e-13 * np.abs(full).max()


def test_single_layer_of_the_smallest_period_has_zero_stress():
    # every offset of a 2 x 2 x 1 period is 0 or a half period in the plane and
    # 0 along z: F is odd and periodic there, so it vanishes
    lines = np.array([(0, 0, 1), TILT])
    rho = _rho(17, (2, 2, 1), 2)
    out = stress_direct_periodic(rho, (1.0, 1.5, 2.0), lines, 1.0, 0.3, shells=4)
    ref = stress_direct_periodic(rho, (1.0, 1.5, 2.0), lines, 1.0, 0.3, periodic=(False, False))
    assert np.abs(ref).max() > 1e-2
    assert np.abs(out).max() < 1e-14 * np.abs(ref).max() * 100
