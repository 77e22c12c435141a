"""Pins of the oracle's discrete sum Eq. (10) (no GPU): brute force over cell
pairs, the convolution structure (impulse response, linearity, translation
invariance), the textbook field of a long dislocation column, the mirror
symmetries of the disk with vertical edge dislocations (Sec. 3), and the
agreement of the library-FFT reference with the direct sum."""
import itertools

import numpy as np
import pytest

from oracle.direct import stress_direct
from oracle.fft_reference import stress_fft_reference
from oracle.kernel import KernelGeometry, interaction_kernel
from oracle.segment import segment_stress
from paper_1804_01830_amd import workloads

TILT = (np.sin(np.radians(15.6)), 0.0, np.cos(np.radians(15.6)))


def _small(seed=1, n=(3, 4, 2), lines=((0, 0, 1), TILT), d=(1.0, 1.5, 2.0)):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    rho = rng.uniform(-1, 1, size=(3 * len(lines), nz, ny, nx))
    return rho, d, np.array(lines, dtype=float)


def test_direct_sum_equals_pure_python_brute_force():
    rho, d, lines = _small()
    C, nz, ny, nx = rho.shape
    geoms = [KernelGeometry(d=d, t=tuple(t), mu=1.2, nu=0.3) for t in lines]
    ref = np.zeros((6, nz, ny, nx))
    for k0, j0, i0 in itertools.product(range(nz), range(ny), range(nx)):
        for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
            for l, g in enumerate(geoms):
                K = interaction_kernel(g, np.array([[i0 - i, j0 - j, k0 - k]]))[0]
                for gam in range(3):
                    ref[:, k0, j0, i0] += K[:, gam] * rho[3 * l + gam, k, j, i]
    full = stress_direct(rho, d, lines, 1.2, 0.3)
    assert np.abs(full - ref).max() < 1e-13 * np.abs(ref).max()
    tg = np.array([[0, 0, 0], [2, 3, 1], [1, 2, 0]])
    samp = stress_direct(rho, d, lines, 1.2, 0.3, targets=tg)
    assert np.abs(samp - ref[:, tg[:, 2], tg[:, 1], tg[:, 0]]).max() < 1e-13 * np.abs(ref).max()


def test_fft_reference_matches_direct_sum():
    rho, d, lines = _small(seed=3, n=(5, 3, 4))
    a = stress_direct(rho, d, lines, 1.0, 0.3)
    b = stress_fft_reference(rho, d, lines, 1.0, 0.3)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-13


def test_impulse_response_is_the_kernel():
    n = (6, 5, 4)
    d = (1.0, 1.0, 2.0)
    rho = np.zeros((6, 4, 5, 6))
    src = (2, 3, 1)                               # (i, j, k)
    rho[4, src[2], src[1], src[0]] = 1.0          # line 1 (tilted), gamma = y
    out = stress_direct(rho, d, [(0, 0, 1), TILT], 1.0, 0.3)
    g = KernelGeometry(d=d, t=TILT, mu=1.0, nu=0.3)
    for tgt in ([0, 0, 0], [5, 4, 3], [2, 3, 1], [3, 3, 1]):
        K = interaction_kernel(g, np.array([np.array(tgt) - src]))[0]
        assert np.array_equal(out[:, tgt[2], tgt[1], tgt[0]], K[:, 1])


def test_linearity_and_translation_invariance():
    rho, d, lines = _small(seed=4, n=(4, 4, 3))
    rho2, _, _ = _small(seed=5, n=(4, 4, 3))
    a = stress_direct(rho, d, lines, 1.0, 0.3)
    b = stress_direct(rho2, d, lines, 1.0, 0.3)
    ab = stress_direct(2.0 * rho - 0.5 * rho2, d, lines, 1.0, 0.3)
    assert np.abs(ab - (2.0 * a - 0.5 * b)).max() < 1e-13 * np.abs(ab).max()
    # shift a density that lives in a sub-box by one cell along x and z
    big = np.zeros((6, 5, 6, 7))
    big[:, 0:3, 0:4, 0:4] = rho
    sh = np.zeros_like(big)
    sh[:, 1:4, 0:4, 1:5] = rho
    s0 = stress_direct(big, d, lines, 1.0, 0.3)
    s1 = stress_direct(sh, d, lines, 1.0, 0.3)
    assert np.abs(s1[:, 1:, :, 1:] - s0[:, :-1, :, :-1]).max() < 1e-13 * np.abs(s0).max()


def test_long_column_reproduces_textbook_fields():
    """A column of density 1/(dx dy) through a tall grid acts as one long
    straight dislocation. For targets with no subdivided (near) source cell
    the sum telescopes exactly to the single-segment stress of Eq. (4a)+(5);
    for all targets the mid-height stress approaches the textbook field, the
    near targets to the accuracy of the subdivision (a few 1e-3 here)."""
    nx, ny, nz = 21, 21, 48
    d = (1.0, 1.0, 4.0)
    H = nz * d[2]
    mu, nu = 1.0, 0.3
    c = (10, 10)
    targets = np.array([[c[0] + 9, c[1] - 9, 24], [c[0] - 9, c[1] + 1, 23],
                        [c[0] + 6, c[1] + 2, 23], [c[0] - 3, c[1] + 7, 24], [c[0] + 4, c[1], 24]])
    far = np.array([True, True, False, False, False])
    D = mu / (2 * np.pi * (1 - nu))
    for gam in (0, 2):                                   # edge (b = e_x), screw (b = e_z)
        rho = np.zeros((3, nz, ny, nx))
        rho[gam, :, c[1], c[0]] = 1.0 / (d[0] * d[1])
        out = stress_direct(rho, d, [(0, 0, 1)], mu, nu, targets=targets)
        p = (targets - np.array([c[0], c[1], 0])) * np.array(d)
        p = p - np.array([0.0, 0.0, (nz - 1) * d[2] / 2.0])
        seg = segment_stress(p, H, (0, 0, 1), mu, nu)[:, :, gam].T
        rel = np.abs(out - seg).max(axis=0) / np.abs(seg).max(axis=0)
        assert np.all(rel[far] < 1e-12) and np.all(rel[~far] < 5e-3)
        x, y = p[:, 0], p[:, 1]
        r2 = x * x + y * y
        z0 = np.zeros_like(x)
        if gam == 0:
            tb = np.stack([-D * y * (3 * x * x + y * y) / r2 ** 2, D * y * (x * x - y * y) / r2 ** 2,
                           -2 * nu * D * y / r2, z0, z0, D * x * (x * x - y * y) / r2 ** 2])
        else:
            tb = np.stack([z0, z0, z0, mu * x / (2 * np.pi * r2), -mu * y / (2 * np.pi * r2), z0])
        rel = np.abs(out - tb).max(axis=0) / np.abs(tb).max(axis=0)
        assert np.all(rel < 3.0 * r2 / (H / 2) ** 2 + np.where(far, 0.0, 5e-3))


@pytest.mark.slow
def test_disk_edge_mirror_symmetries():
    """Sec. 3: with b = e_x, t = e_z and a density even in x and y, sxx, syy,
    szz are odd in y and even in x, sxy is odd in x and even in y, sxz is odd
    in x and y, syz is even in both; with a z-independent density, sxz and syz
    are odd about the mid-plane and the rest even."""
    w = workloads.disk_edge()
    s = stress_direct(w["rho"][0], w["d"], w["lines"], w["mu"], w["nu"])
    scale = np.abs(s).max()
    fx = lambda a: a[..., ::-1]          # x -> -x
    fy = lambda a: a[..., ::-1, :]       # y -> -y
    fz = lambda a: a[..., ::-1, :, :]    # z mirror about the mid-plane
    par = {0: (1, -1, 1), 1: (1, -1, 1), 2: (1, -1, 1), 5: (-1, 1, 1), 4: (-1, -1, -1), 3: (1, 1, -1)}
    for v, (px, py, pz) in par.items():
        assert np.abs(fx(s[v]) - px * s[v]).max() < 1e-12 * scale
        assert np.abs(fy(s[v]) - py * s[v]).max() < 1e-12 * scale
        assert np.abs(fz(s[v]) - pz * s[v]).max() < 1e-12 * scale
    # sigma_yz keeps one sign over the disk plane (Sec. 3)
    mid = s[3, 1]
    assert np.all(mid[np.abs(mid) > 1e-3 * np.abs(mid).max()] > 0) or \
        np.all(mid[np.abs(mid) > 1e-3 * np.abs(mid).max()] < 0)


def test_zero_density_gives_zero_stress():
    out = stress_direct(np.zeros((3, 2, 3, 4)), (1, 1, 1), [(0, 0, 1)], 1.0, 0.3)
    assert np.all(out == 0.0)
