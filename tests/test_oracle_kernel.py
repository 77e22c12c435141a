"""Pins of the oracle's interaction coefficients (no GPU): exact identities of
the definition (Eq. 9b with the cell volume, the near-cell subdivision of
Sec. 2.3 / Fig. 3, the zero self-term), checked against independent brute
force and against the segment formula of a long column."""
import itertools

import numpy as np
import pytest

from oracle.kernel import KernelGeometry, interaction_kernel, kernel_table
from oracle.segment import segment_stress, chord_length

MU, NU = 1.0, 0.3
TILT = (np.sin(np.radians(15.6)), 0.0, np.cos(np.radians(15.6)))


def test_subdivision_parameters():
    g = KernelGeometry(d=(1.0, 1.0, 4.0), t=(0, 0, 1), mu=MU, nu=NU)
    assert list(g.subdivision) == [1, 1, 4]
    g = KernelGeometry(d=(1.0, 1.0, 2.0), t=(0, 0, 1), mu=MU, nu=NU)
    assert list(g.subdivision) == [1, 1, 2]
    g = KernelGeometry(d=(2.0, 0.5, 1.2), t=(0, 0, 1), mu=MU, nu=NU)
    assert list(g.subdivision) == [4, 1, 2]
    delta, w = g.sub_offsets()
    assert np.isclose(w.sum(), 1.0)                    # weights of a mean over target subcells
    assert len(w) == 7 * 1 * 3


@pytest.mark.parametrize("t", [(0, 0, 1), TILT])
def test_self_term_zero_and_kernel_odd(t):
    g = KernelGeometry(d=(1.0, 1.0, 2.0), t=t, mu=MU, nu=NU)
    offs = np.array(list(itertools.product(range(-3, 4), range(-3, 4), range(-2, 3))))
    K = interaction_kernel(g, offs)
    Km = interaction_kernel(g, -offs)
    assert np.abs(K + Km).max() <= 1e-13 * np.abs(K).max()
    assert np.all(K[np.all(offs == 0, axis=1)] == 0.0)
    # the symmetric sum over sub-offsets that the zero self-term stands for
    delta, w = g.sub_offsets()
    nz = np.any(delta != 0, axis=1)
    s = g.sub_box
    f = segment_stress(delta[nz] * s, chord_length(s, g.unit_t), g.unit_t, MU, NU)
    assert np.abs(np.einsum("q,qvg->vg", w[nz], f)).max() < 1e-14 * np.abs(f).max()


@pytest.mark.parametrize("t", [(0, 0, 1), TILT])
def test_near_kernel_equals_explicit_subcell_pairs(t):
    """Collapsed sub-offset weights vs the double loop over target and source
    subcells (mean over targets, volume-weighted sum over sources)."""
    d = np.array([1.0, 1.0, 2.0]) if t == (0, 0, 1) else np.array([2.0, 1.0, 1.0])
    g = KernelGeometry(d=tuple(d), t=t, mu=MU, nu=NU)
    m = g.subdivision
    s = d / m
    tt = g.unit_t
    h = chord_length(s, tt)
    cells = [np.array(c) for c in itertools.product(*[range(k) for k in m])]
    centres = [(c + 0.5) * s - 0.5 * d for c in cells]
    M = len(cells)
    for off in ([1, 0, 0], [0, 1, 1], [-1, 2, 0], [0, 0, 1]):
        off = np.array(off)
        acc = np.zeros((6, 3))
        for pt in centres:                 # target subcells
            for ps in centres:             # source subcells
                p = off * d + pt - ps
                acc += segment_stress(p[None], h, tt, MU, NU)[0] / h * (g.cell_volume / M)
        acc /= M
        K = interaction_kernel(g, off[None])[0]
        assert np.abs(K - acc).max() < 1e-13 * np.abs(acc).max()


def test_far_kernel_is_scaled_segment_stress():
    g = KernelGeometry(d=(1.0, 2.0, 3.0), t=TILT, mu=MU, nu=NU)
    off = np.array([[9, -4, 5], [-12, 1, -3]])
    assert not g.is_near(off).any()
    h = chord_length(g.d, g.unit_t)
    ref = segment_stress(off * np.array(g.d), h, g.unit_t, MU, NU) * (g.cell_volume / h)
    assert np.array_equal(interaction_kernel(g, off), ref)


def test_column_telescopes_to_one_long_segment():
    """A column of cells with density 1/(dx dy) is one long vertical segment:
    the kernel sum over the column equals the Eq. (4a)+(5) stress of a single
    segment of length Nz*dz (Eq. 5 telescopes)."""
    d = np.array([1.0, 1.0, 4.0])
    g = KernelGeometry(d=tuple(d), t=(0, 0, 1), mu=MU, nu=NU)
    nz = 16
    for tgt in ([11, 3, 5], [-9, -10, 0], [13, 0, 15]):
        tgt = np.array(tgt)
        offs = tgt[None, :] - np.stack([np.zeros(nz, int), np.zeros(nz, int), np.arange(nz)], axis=1)
        assert not g.is_near(offs).any()
        K = interaction_kernel(g, offs).sum(axis=0) / (d[0] * d[1])
        p = tgt * d - np.array([0.0, 0.0, (nz - 1) * d[2] / 2.0])
        ref = segment_stress(p[None], nz * d[2], (0, 0, 1), MU, NU)[0]
        assert np.abs(K - ref).max() < 1e-12 * np.abs(ref).max()


def test_kernel_table_indexing():
    g = KernelGeometry(d=(1.0, 1.5, 2.0), t=TILT, mu=MU, nu=NU)
    n = (3, 4, 2)
    tab = kernel_table(g, n)
    assert tab.shape == (6, 3, 3, 7, 5)
    for off in ([2, -3, 1], [0, 0, 0], [-2, 1, -1]):
        ref = interaction_kernel(g, np.array([off]))[0]
        got = tab[:, :, off[2] + 1, off[1] + 3, off[0] + 2]
        assert np.array_equal(got, ref)


def test_kernel_scales_with_mu():
    a = KernelGeometry(d=(1.0, 1.0, 2.0), t=TILT, mu=1.0, nu=0.25)
    b = KernelGeometry(d=(1.0, 1.0, 2.0), t=TILT, mu=3.0, nu=0.25)
    off = np.array([[1, 0, 0], [5, 5, 3]])
    assert np.allclose(3.0 * interaction_kernel(a, off), interaction_kernel(b, off), rtol=1e-14, atol=0)


@pytest.mark.parametrize("t", [(0, 0, 1), TILT])
def test_near_cell_coefficients_converge_under_refinement(t):
    """Sec. 2.3: the near-cell coefficient is the mean over target subcells of
    the sum over source subcells, a midpoint-rule approximation of the
    cell-averaged interaction; doubling the subcells per axis (m -> 2m -> 4m
    -> 8m) must converge at second order: successive changes shrink about
    fourfold. A wrong sub-offset weight, subcell chord or subcell volume
    breaks the rate (the sums then tend to another limit or diverge)."""
    offs = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1], [2, 0, 0], [2, 1, 1], [-1, 2, -1]])
    Ks = [interaction_kernel(KernelGeometry(d=(1.0, 1.0, 2.0), t=t, mu=MU, nu=NU, refine=f), offs)
          for f in (1, 2, 4, 8)]
    for i, o in enumerate(offs):
        d = [np.abs(Ks[k][i] - Ks[k + 1][i]).max() for k in range(3)]
        r = [d[0] / d[1], d[1] / d[2]]
        assert 2.5 < r[0] < 5.5 and 2.8 < r[1] < 5.0, (o, d, r)


def test_stress_converges_when_the_cells_are_halved():
    """Sec. 2.3, last paragraph: halving the cell size must not change the
    result noticeably. A smooth density blob (edge lines along z, b = e_x)
    is sampled on grids with d = (1, 1, 2), (1/2, 1/2, 1) and (1/4, 1/4, 1/2)
    over the same region; the stress at common physical points changes by
    less than 3 % between the two finest grids, and successive changes fall
    at second order (a missing cell volume would scale each level by 8)."""
    from oracle.direct import stress_direct
    d0 = np.array([1.0, 1.0, 2.0])
    span = np.array([9.0, 9.0, 10.0])
    c, w = span / 2, 1.6
    tc = np.array([[5, 5, 2], [2, 5, 2], [5, 7, 3], [8, 1, 0], [4, 4, 4]])
    res = []
    for lev in range(3):
        dd = d0 / 2 ** lev
        n = [int(round(span[a] / dd[a])) + 1 for a in range(3)]
        z, y, x = (np.arange(n[a]) * dd[a] for a in (2, 1, 0))
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        rho = np.zeros((3, n[2], n[1], n[0]))
        rho[0] = np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2 * w * w))
        res.append(stress_direct(rho, tuple(dd), [(0, 0, 1)], MU, NU, targets=tc * 2 ** lev))
    d01 = np.linalg.norm(res[0] - res[1])
    d12 = np.linalg.norm(res[1] - res[2])
    assert d12 < 0.03 * np.linalg.norm(res[2])
    assert 3.0 < d01 / d12 < 5.5
