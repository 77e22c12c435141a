"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function ``include/ddstress.h`` declares, and validates descriptors
(ddstress_plan_footprint does no device work)."""
import os
import re

import pytest

from paper_1804_01830_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ddstress.h")).read()
    return sorted(set(re.findall(r"\b(ddstress_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    assert sorted(B.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.ddstress_version().decode().startswith("ddstress")


def _desc(**kw):
    base = dict(n=(8, 8, 4), d=(1, 1, 2), mu=1.0, nu=0.3, lines=[(0, 0, 1)], precision=32, batch=1)
    base.update(kw)
    return B.make_desc(**base)


def test_footprint_of_a_valid_descriptor():
    cached, work, build = B.footprint(_desc())
    # kernel spectrum: 6 C (Wx tiles) Py Pz floats, at least 6*3*9*16*8 values
    assert cached >= 6 * 3 * 9 * 16 * 8 * 4 and work > 0 and build > 0


@pytest.mark.parametrize("kw", [
    dict(n=(0, 8, 4)), dict(d=(1, -1, 2)), dict(d=(1, float("nan"), 2)), dict(mu=0.0), dict(nu=0.5),
    dict(nu=-1.0), dict(lines=[]), dict(lines=[(0, 0, 0)]), dict(lines=[(0, 0, 1)] * 4), dict(precision=16),
    dict(batch=0), dict(near_shells=-1), dict(periodic=(True, False), pbc_shells=-1),
])
def test_invalid_descriptors_are_rejected(kw):
    with pytest.raises(B.DDStressError) as e:
        B.footprint(_desc(**kw))
    assert e.value.status == B.E_INVALID
    assert B.load().ddstress_last_error().decode()


def test_unsupported_sizes_and_flags():
    for kw in (dict(n=(513, 8, 8)), dict(flags=8), dict(n=(6, 8, 4), periodic=(True, False)),
               dict(n=(8, 12, 4), periodic=(False, True)), dict(n=(1, 8, 4), periodic=(True, True)),
               dict(periodic=(True, True), pbc_shells=33)):
        with pytest.raises(B.DDStressError) as e:
            B.footprint(_desc(**kw))
        assert e.value.status == B.E_UNSUPPORTED


def test_periodic_descriptors():
    # a non-power-of-two x is fine while only y is periodic; the shell count is
    # ignored without a periodic flag
    for kw in (dict(n=(6, 8, 4), periodic=(False, True)), dict(pbc_shells=-1),
               dict(periodic=(True, True), pbc_shells=32), dict(n=(2, 2, 1), periodic=(True, True))):
        B.footprint(_desc(**kw))
    open_ = B.footprint(_desc(n=(16, 16, 4)))
    per = B.footprint(_desc(n=(16, 16, 4), periodic=(True, True)))
    assert per[1] < open_[1] and per[2] < open_[2]


def test_padded_lengths():
    assert B.padded_lengths((32, 128, 1)) == (64, 256, 2)
    assert B.padded_lengths((5, 3, 7)) == (16, 8, 16)
    assert B.padded_lengths((32, 128, 8), periodic=(True, False)) == (32, 256, 16)
    assert B.padded_lengths((32, 128, 8), periodic=(True, True)) == (32, 128, 16)


def test_footprint_predicts_mirror_compression():
    tilt = (0.26892, 0.0, 0.96316)
    full = B.footprint(_desc(lines=[(0, 0, 1)], flags=B.FLAG_FULL_SPECTRUM))[0]
    both = B.footprint(_desc(lines=[(0, 0, 1)]))[0]
    ymir = B.footprint(_desc(lines=[(0, 0, 1), tilt]))[0]
    ymir_full = B.footprint(_desc(lines=[(0, 0, 1), tilt], flags=B.FLAG_FULL_SPECTRUM))[0]
    # grid 8 x 8 x 4 -> Py = 16, Pz = 8: kept rows 9 of 16 and 5 of 8
    assert both < full and ymir < ymir_full
    spec_full = full - 2048 * 8            # minus the FP32 twiddle table
    spec_both = both - 2048 * 8
    assert spec_both * 16 * 8 == spec_full * 9 * 5


def test_tuning_key_separates_periodic_plans():
    from paper_1804_01830_amd import tuning as Tn
    a = Tn.shape_key(_desc(n=(16, 16, 4)), "gfx950-256cu")
    b = Tn.shape_key(_desc(n=(16, 16, 4), periodic=(True, True)), "gfx950-256cu")
    c = Tn.shape_key(_desc(n=(16, 16, 4), periodic=(False, True)), "gfx950-256cu")
    assert len({a, b, c}) == 3 and "pbc" not in a and "pbcxy" in b and "pbcy" in c



@pytest.mark.parametrize("kw,status", [
    (dict(n=(8, 8, 2)), B.E_INVALID), (dict(n=(0, 8, 4)), B.E_INVALID), (dict(precision=16), B.E_INVALID),
    (dict(nu=0.5), B.E_INVALID), (dict(mu=-1.0), B.E_INVALID), (dict(dt=-1e-3), B.E_INVALID),
    (dict(d=(1.0, 0.0, 1.0)), B.E_INVALID), (dict(n=(8, 8, 5000)), B.E_UNSUPPORTED),
])
def test_relaxation_descriptors_are_validated_before_any_device_work(kw, status):
    base = dict(n=(8, 8, 4), d=(1.0, 1.0, 1.0), mu=1.0, nu=0.3, precision=64, dt=0.0)
    base.update(kw)
    with pytest.raises(B.DDStressError) as e:
        B.Relax(**base)
    assert e.value.status == status


def test_plane_statistics_arguments_are_validated_before_any_device_work():
    import ctypes
    lib = B.load()
    n = (ctypes.c_int32 * 3)(8, 8, 4)
    bad_n = (ctypes.c_int32 * 3)(8, 0, 4)
    dummy = ctypes.c_void_p(16)                  # never dereferenced: validation fails first
    for args in ((None, 32, n, 1, dummy), (dummy, 32, n, 1, None), (dummy, 16, n, 1, dummy),
                 (dummy, 32, n, 0, dummy), (dummy, 64, bad_n, 1, dummy)):
        assert lib.ddstress_plane_mean_square(*args, None) == B.E_INVALID


def test_relaxation_solve_rejects_bad_arguments_without_a_plan():
    lib = B.load()
    import ctypes
    steps, norm = ctypes.c_int32(), ctypes.c_double()
    assert lib.ddstress_relax_solve(None, 1e-6, 10, 1, ctypes.byref(steps), ctypes.byref(norm), None) == B.E_INVALID


@pytest.mark.parametrize("n,precision,ok", [
    ((512, 512, 256), 32, True), ((512, 512, 257), 32, False),
    ((512, 512, 128), 64, True), ((512, 512, 129), 64, False), ((257, 257, 129), 64, False),
    ((512, 256, 512), 32, True), ((256, 512, 512), 64, False),
])
def test_z_pass_offsets_are_bounded(n, precision, ok):
    """The fused z pass addresses one density plane [Nz][Py][Wx] with 32-bit
    byte offsets; a grid whose rows z < Pz/2 would need more is refused with
    DDSTRESS_E_UNSUPPORTED before anything is allocated (a larger plane would
    wrap the offsets and read wrong rows)."""
    desc = _desc(n=n, precision=precision)
    if ok:
        B.footprint(desc)
        return
    with pytest.raises(B.DDStressError) as e:
        B.footprint(desc)
    assert e.value.status == B.E_UNSUPPORTED
    assert "32-bit" in B.load().ddstress_last_error().decode()
