"""Host checks of the error measures the GPU parity tests use (tests/gpu_util.py)."""
import numpy as np

from gpu_util import rel_l2, rel_l2_split


def test_split_measures_small_components_against_the_whole_norm():
    rng = np.random.default_rng(0)
    ref = rng.normal(size=(6, 4, 3, 2))
    ref[2] *= 1e-6                      # nearly zero
    ref[5] = 0.0                        # exactly zero
    got = ref + 1e-8 * rng.normal(size=ref.shape)
    own, small = rel_l2_split(got, ref)
    assert sorted(own) == [0, 1, 3, 4] and sorted(small) == [2, 5]
    whole = np.linalg.norm(ref)
    for v, e in own.items():
        assert np.isclose(e, np.linalg.norm(got[v] - ref[v]) / np.linalg.norm(ref[v]))
    for v, e in small.items():
        assert np.isclose(e, np.linalg.norm(got[v] - ref[v]) / whole)
    comp, w = rel_l2(got, ref)
    assert np.allclose(comp[[0, 1, 3, 4]], [own[v] for v in (0, 1, 3, 4)])
    assert np.isclose(w, np.linalg.norm(got - ref) / whole)


def test_exact_zero_reference_must_be_met_exactly():
    ref = np.zeros((6, 2, 2, 2))
    assert rel_l2_split(ref.copy(), ref) == ({}, {v: 0.0 for v in range(6)})
    got = ref.copy()
    got[1, 0, 0, 0] = 1e-30
    own, small = rel_l2_split(got, ref)
    assert small[1] == np.inf and small[0] == 0.0
