"""Pins of the axis-basis (Nye) channels (no GPU):

* lines along an axis: the Nye channels are the plain channels of that axis
  and the stress equals the one-direction sum exactly;
* (n, t, b) and (n, -t, -b) describe the same dislocations: same channels;
* a tilted line: the Nye stress approaches the exact per-direction stress
  away from the source (the segment's field is linear in dl t only as dl / r
  goes to zero) and differs from it in the near field.
"""
import numpy as np

from oracle.direct import stress_direct
from oracle.kernel import KernelGeometry, interaction_kernel
from oracle.nye import AXES, nye_channels

TILT = np.array([np.sin(np.radians(15.6)), 0.0, np.cos(np.radians(15.6))])


def test_axis_lines_reduce_to_the_plain_channels():
    rng = np.random.default_rng(1)
    shape = (3, 4, 5)
    n = rng.uniform(0, 1, size=shape)
    b = rng.uniform(-1, 1, size=(3,) + shape)
    t = np.zeros((3,) + shape)
    t[2] = 1.0
    rho = nye_channels(n, t, b)
    assert np.all(rho[:6] == 0.0)
    assert np.array_equal(rho[6:9], n[None] * b)
    d = (1.0, 1.0, 2.0)
    full = stress_direct(rho, d, AXES, 1.0, 0.3)
    one = stress_direct(n[None] * b, d, [(0.0, 0.0, 1.0)], 1.0, 0.3)
    assert np.abs(full - one).max() <= 1e-13 * np.abs(one).max()


def test_reversed_line_and_burgers_vector_give_the_same_channels():
    rng = np.random.default_rng(2)
    n = rng.uniform(0, 1, size=(4, 4))
    t = rng.normal(size=(3, 4, 4))
    b = rng.normal(size=(3, 4, 4))
    assert np.array_equal(nye_channels(n, t, b), nye_channels(n, -t, -b))


def test_tilted_line_far_field_converges_to_the_exact_kernel():
    # one source cell with a tilted line: the Nye sum over the axis kernels
    # against the kernel of the tilted line itself, along a ray of offsets
    d = (1.0, 1.0, 1.0)
    bvec = np.array([0.3, -0.5, 0.8])
    exact = KernelGeometry(d=d, t=tuple(TILT), mu=1.0, nu=0.3)
    axes = [KernelGeometry(d=d, t=a, mu=1.0, nu=0.3) for a in AXES]
    errs = []
    for r in (3, 6, 12, 24, 48):
        off = np.array([[r, r // 2, r // 3]])
        ke = interaction_kernel(exact, off)[0] @ bvec
        kn = sum(TILT[l] * (interaction_kernel(axes[l], off)[0] @ bvec) for l in range(3))
        errs.append(np.linalg.norm(kn - ke) / np.linalg.norm(ke))
    # the relative error falls with the distance and is small far away
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-3 and errs[0] > 10 * errs[-1], errs
