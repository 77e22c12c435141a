"""Pins of the plane statistics, Eq. (20) (no GPU): closed forms for constant
planes and for cosines of whole wavenumbers (mean square A^2 / 2), and the
scaling s^2(a sigma) = a^2 s^2(sigma)."""
import numpy as np

from oracle.stats import plane_mean_square


def test_constant_planes():
    sig = np.zeros((6, 3, 4, 5))
    for v in range(6):
        for k in range(3):
            sig[v, k] = (v + 1) * (k - 1.5)
    got = plane_mean_square(sig)
    for v in range(6):
        for k in range(3):
            assert abs(got[v, k] - ((v + 1) * (k - 1.5)) ** 2) < 1e-13


def test_cosines_of_whole_wavenumbers():
    nx, ny = 16, 12
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    sig = np.zeros((2, 6, 2, ny, nx))
    amps = np.arange(1, 25, dtype=float).reshape(2, 6, 2)
    for b in range(2):
        for v in range(6):
            for k in range(2):
                kx, ky = 1 + v % 3, k + b
                sig[b, v, k] = amps[b, v, k] * np.cos(2 * np.pi * (kx * x[None, :] + ky * y[:, None]) + 0.3 * v)
    got = plane_mean_square(sig)
    assert np.abs(got - amps ** 2 / 2).max() < 1e-12 * (amps ** 2).max()


def test_quadratic_scaling():
    rng = np.random.default_rng(1)
    sig = rng.normal(size=(6, 4, 7, 9))
    assert np.abs(plane_mean_square(3.0 * sig) - 9.0 * plane_mean_square(sig)).max() < 1e-12
