"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: relative L2 error per stress component and over the whole tensor
<= 1e-12 for the FP64 path and <= 1e-5 for the FP32 path (FP32 transforms and
contraction, FP64 interaction coefficients and their transform).
"""
import functools
import sys

import numpy as np
import pytest

from gpu_util import gpu_stress, rel_l2, rel_l2_split
from oracle import stress_direct, interaction_kernel, KernelGeometry
from paper_1804_01830_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {64: 1e-12, 32: 1e-5}
TILT = W.mixed_line()
DIAG = (0.0, 1.0 / np.sqrt(2.0), 1.0 / np.sqrt(2.0))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# Full-field cases: ragged sizes, several kx tiles, batches, one to three line
# directions, anisotropic cells (subdivision along one or two axes).
CASES = {
    "disk-edge-32x32x4": lambda: W.disk_edge(),
    "rand-5x3x7-L3": lambda: W.random_field((5, 3, 7), n_lines=3, seed=1, d=(1.0, 1.5, 2.0)),
    "rand-17x9x3-L2-B2": lambda: W.random_field((17, 9, 3), n_lines=2, batch=2, seed=2, d=(1.0, 1.0, 3.0)),
    "rand-33x20x9-L2": lambda: W.random_field((33, 20, 9), n_lines=2, seed=3, d=(2.0, 1.0, 1.0)),
    "rand-1x1x1": lambda: W.random_field((1, 1, 1), n_lines=1, seed=4),
    "rand-1x6x2": lambda: W.random_field((1, 6, 2), n_lines=1, seed=5, d=(1.0, 1.0, 2.0)),
    "rand-40x1x12-diag": lambda: W.random_field((40, 1, 12), seed=6, d=(1.0, 1.0, 1.0), lines=[DIAG]),
    # the longest supported axes (512 cells: transforms of length 1024)
    "rand-512x2x2-max-x": lambda: W.random_field((512, 2, 2), n_lines=1, seed=11),
    "rand-2x512x2-max-y": lambda: W.random_field((2, 512, 2), n_lines=1, seed=11),
    "rand-2x2x512-max-z-L3": lambda: W.random_field((2, 2, 512), n_lines=3, seed=11),
    # planes that take the fused inverse y-x kernel in FP32 (Px = Py = 256)
    "rand-72x70x2-B2": lambda: W.random_field((72, 70, 2), n_lines=1, batch=2, seed=13, d=(1.0, 1.0, 2.0)),
}


@functools.lru_cache(maxsize=None)
def _case(name):
    w = CASES[name]()
    ref = np.stack([stress_direct(w["rho"][b], w["d"], w["lines"], w["mu"], w["nu"])
                    for b in range(w["rho"].shape[0])])
    return w, ref


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("name", list(CASES))
def test_full_field_parity(name, precision):
    w, ref = _case(name)
    _say(f"[parity] {name} precision={precision} n={w['n']} B={w['rho'].shape[0]}")
    got = gpu_stress(w, precision)
    comp, whole = rel_l2(got, ref)
    own, small = rel_l2_split(got, ref)
    _say(f"  rel L2 per component {np.array2string(comp, precision=2)} whole {whole:.2e}")
    _say("  against their own norm: " + ", ".join(f"{v}: {e:.2e}" for v, e in own.items())
         + ("; small components against the whole norm: " + ", ".join(f"{v}: {e:.2e}" for v, e in small.items())
            if small else ""))
    assert np.all(comp <= TOL[precision]) and whole <= TOL[precision]
    assert all(e <= TOL[precision] for e in own.values()) and all(e <= TOL[precision] for e in small.values())


def test_zero_density_gives_exact_zero():
    w = W.random_field((9, 7, 5), n_lines=2, seed=7)
    w["rho"][:] = 0.0
    for prec in (32, 64):
        assert np.all(gpu_stress(w, prec) == 0.0)


def test_kernel_realspace_matches_oracle_entrywise():
    import torch
    from paper_1804_01830_amd import binding as B
    n, d = (6, 5, 4), (1.0, 1.5, 2.0)
    lines = [(0.0, 0.0, 1.0), TILT, DIAG]
    desc = B.make_desc(n, d, 1.3, 0.27, lines, precision=64)
    P = B.padded_lengths(n)
    ax = [np.where(np.arange(P[a]) < n[a], np.arange(P[a]), np.arange(P[a]) - P[a]) for a in range(3)]
    valid = [(np.arange(P[a]) < n[a]) | (np.arange(P[a]) > P[a] - n[a]) for a in range(3)]
    gz, gy, gx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    vz, vy, vx = np.meshgrid(valid[2], valid[1], valid[0], indexing="ij")
    mask = vz & vy & vx
    offs = np.stack([gx[mask], gy[mask], gz[mask]], axis=-1)
    for l, t in enumerate(lines):
        out = torch.empty((3, 6, P[2], P[1], P[0]), dtype=torch.float64, device="cuda")
        B.kernel_realspace(desc, l, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = interaction_kernel(KernelGeometry(d=d, t=t, mu=1.3, nu=0.27), offs)      # (M, 6, 3)
        g = np.transpose(got, (2, 3, 4, 1, 0))[mask]                                  # (M, 6, 3)
        assert np.all(got[:, :, ~mask] == 0.0)
        err = np.abs(g - ref).max() / np.abs(ref).max()
        _say(f"[kernel] line {l}: max abs err / max = {err:.2e}")
        assert err < 1e-13


def test_impulse_response_is_the_kernel_slice():
    n = (12, 10, 6)
    d = (1.0, 1.0, 2.0)
    w = W.random_field(n, n_lines=2, seed=0, d=d)
    w["rho"][:] = 0.0
    src = (4, 7, 2)
    w["rho"][0, 4, src[2], src[1], src[0]] = 1.0          # line 1 (tilted), gamma = y
    got = gpu_stress(w, 64)[0]
    gz, gy, gx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    offs = np.stack([gx.ravel() - src[0], gy.ravel() - src[1], gz.ravel() - src[2]], axis=-1)
    K = interaction_kernel(KernelGeometry(d=d, t=tuple(w["lines"][1]), mu=w["mu"], nu=w["nu"]), offs)
    ref = K[:, :, 1].T.reshape(6, *got.shape[1:])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("precision", [64, 32])
def test_disk_mixed_128_sampled_targets(precision):
    """Full-size disk with mixed Burgers vectors (128 x 128 x 32, dz = 2 dx)
    in the launch configuration the benchmark times, checked on sampled cells
    (corners, faces, disk centre and random cells) against the direct sum."""
    w = W.disk_mixed()
    rng = np.random.default_rng(21)
    tg = np.array([[0, 0, 0], [127, 127, 31], [64, 63, 16], [127, 0, 15], [60, 70, 0], [3, 90, 31]]
                  + [[rng.integers(128), rng.integers(128), rng.integers(32)] for _ in range(6)])
    ref = stress_direct(w["rho"][0], w["d"], w["lines"], w["mu"], w["nu"], targets=tg)
    got = gpu_stress(w, precision)[0][:, tg[:, 2], tg[:, 1], tg[:, 0]]
    comp, whole = rel_l2(got, ref)
    _say(f"[disk-mixed-128] precision={precision} per component {np.array2string(comp, precision=2)} "
         f"whole {whole:.2e}")
    assert np.all(comp <= TOL[precision]) and whole <= TOL[precision]


def test_stress_before_density_is_a_state_error():
    from paper_1804_01830_amd import binding as B
    desc = B.make_desc((4, 4, 4), (1, 1, 1), 1.0, 0.3, [(0, 0, 1)], precision=32)
    plan = B.Plan(desc)
    out = plan.new_output()
    with pytest.raises(B.DDStressError) as e:
        plan.stress(out)
    assert e.value.status == B.E_STATE
    plan.close()


def _load_golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name + ".json")) as f:
        return json.load(f)


@pytest.mark.parametrize("precision", [32, 64])
def test_poly_layer_256_golden(precision):
    """Full-size 256 x 256 x 64 polycrystal layer (two line directions,
    C = 6) against stored oracle values at 10 cells."""
    g = _load_golden("poly_layer_256x256x64")
    w = W.poly_layer()
    assert list(w["n"]) == g["n"] and np.allclose(w["lines"], g["lines"])
    tg = np.array(g["targets"])
    ref = np.array(g["sigma_voigt"]).T
    got = gpu_stress(w, precision)[0][:, tg[:, 2], tg[:, 1], tg[:, 0]]
    comp, whole = rel_l2(got, ref)
    _say(f"[poly-layer-256] precision={precision} per component {np.array2string(comp, precision=2)} "
         f"whole {whole:.2e}")
    assert np.all(comp <= TOL[precision]) and whole <= TOL[precision]


def test_poly_sweep_batch64_golden():
    """The 64-realisation batch on one plan (B = 64, FP32): realisations 0
    and 63 against stored oracle values."""
    w = W.poly_sweep()
    got = gpu_stress(w, 32)
    for name in ("poly_sweep_128x128x32_b0", "poly_sweep_128x128x32_b63"):
        g = _load_golden(name)
        tg = np.array(g["targets"])
        ref = np.array(g["sigma_voigt"]).T
        sel = got[g["batch_index"]][:, tg[:, 2], tg[:, 1], tg[:, 0]]
        comp, whole = rel_l2(sel, ref)
        _say(f"[{name}] per component {np.array2string(comp, precision=2)} whole {whole:.2e}")
        assert np.all(comp <= TOL[32]) and whole <= TOL[32]


@pytest.mark.parametrize("lines,mir", [([(0.0, 0.0, 1.0)], (1, 1)), ([(0.0, 0.0, 1.0), TILT], (1, 0)),
                                       ([DIAG], (0, 0)), ([(1.0, 0.0, 0.0), (0.0, 1.0, 0.0)], (1, 1))])
def test_mirror_compressed_spectrum_matches_full(lines, mir):
    """The spectrum kept for ky <= Py/2 (kz <= Pz/2) with per-plane signs gives
    the stress of the full spectrum; the layout follows the line directions."""
    import torch
    from paper_1804_01830_amd import binding as B
    w = W.random_field((20, 14, 10), seed=17, d=(1.0, 1.0, 2.0), lines=lines)
    outs = []
    for flags in (0, B.FLAG_FULL_SPECTRUM):
        desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=64, flags=flags)
        plan = B.Plan(desc)
        info = plan.info()
        want = mir if flags == 0 else (0, 0)
        assert (info.mirror_y, info.mirror_z) == want
        rho = torch.from_numpy(w["rho"]).to("cuda")
        plan.set_density(rho)
        out = plan.new_output()
        plan.stress(out)
        torch.cuda.synchronize()
        outs.append((out.cpu().numpy(), info.cached_bytes))
        plan.close()
    (a, ca), (b, cb) = outs
    assert np.linalg.norm(a - b) <= 1e-14 * np.linalg.norm(b)
    assert ca <= cb


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("lines", [1, 2, 3])
def test_grouped_long_z_classes(precision, lines):
    """The grouped fused z form on a 1024-point z transform takes the larger
    element classes (8 per thread with six channels). Forced through the
    tuning struct it agrees with the direct sum where its block fits (FP32, up
    to six channels); elsewhere (LDS > 64 KiB) the plan is refused, and a
    default plan with many realisations falls back to the single-group form."""
    from paper_1804_01830_amd import binding as B
    import torch
    w = W.random_field((3, 2, 300), n_lines=lines, seed=12)
    desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=precision)
    d = B.Plan(desc).info()
    t = B.Tuning()
    t.rows_x, t.tk_y, t.tk_z, t.ex, t.ey = d.rows_x, d.tile_y, 1, d.ex, d.ey
    t.z_groups = d.channels
    fits = precision == 32 and lines <= 2
    if not fits:
        with pytest.raises(B.DDStressError) as e:
            B.Plan(desc, tuning=t)
        assert e.value.status == B.E_INVALID
        many = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=precision, batch=16)
        assert B.Plan(many).info().z_groups == 1
        return
    ref = stress_direct(w["rho"][0], w["d"], w["lines"], w["mu"], w["nu"])[None]
    plan = B.Plan(desc, tuning=t)
    info = plan.info()
    assert info.z_groups == d.channels and info.padded[2] == 1024
    _say(f"[grouped-long] precision={precision} C={d.channels} ez={info.ez}")
    dt = torch.float32 if precision == 32 else torch.float64
    rho = torch.from_numpy(w["rho"]).to("cuda", dtype=dt)
    out = plan.new_output()
    plan.set_density(rho)
    plan.stress(out)
    torch.cuda.synchronize()
    comp, whole = rel_l2(out.double().cpu().numpy(), ref)
    assert np.all(comp <= TOL[precision]) and whole <= TOL[precision]
    plan.close()


# z transforms of length 256 (Nz 65..128) and 512 (Nz 129..256): every
# admissible fused z form (single-group and grouped, every element class and
# tile width that fits), including the staged spectrum of the single-group form
# (B >= 2, z lengths up to 256), against the direct sum.
LONG_Z = {
    "rand-9x7x100-L1-B3": lambda: W.random_field((9, 7, 100), n_lines=1, batch=3, seed=31, d=(1.0, 1.0, 2.0)),
    "rand-6x5x90-L2-B2": lambda: W.random_field((6, 5, 90), n_lines=2, batch=2, seed=32, d=(1.0, 1.0, 2.0)),
    "rand-5x4x200-L1-B2": lambda: W.random_field((5, 4, 200), n_lines=1, batch=2, seed=33),
    "rand-4x3x150-L3": lambda: W.random_field((4, 3, 150), n_lines=3, seed=34, d=(1.0, 1.5, 2.0)),
}


@functools.lru_cache(maxsize=None)
def _long_case(name):
    w = LONG_Z[name]()
    ref = np.stack([stress_direct(w["rho"][b], w["d"], w["lines"], w["mu"], w["nu"])
                    for b in range(w["rho"].shape[0])])
    return w, ref


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("name", list(LONG_Z))
def test_long_z_every_form(name, precision):
    import torch
    from paper_1804_01830_amd import binding as B
    w, ref = _long_case(name)
    nb = w["rho"].shape[0]
    desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=precision, batch=nb)
    base = B.Plan(desc)
    d0 = base.info()
    base.close()
    Pz, C = d0.padded[2], d0.channels
    assert Pz in (256, 512)
    dt = torch.float32 if precision == 32 else torch.float64
    rho = torch.from_numpy(w["rho"]).to("cuda", dtype=dt).contiguous()
    b0 = 4 if precision == 32 else 2
    ran = []
    for groups in (1, C):
        for ez in (b0, 2 * b0, 4 * b0, 8 * b0):
            if ez > 16:
                continue
            for tk in (1, 2, 4, 8, 16):
                t = B.Tuning()
                t.rows_x, t.tk_y, t.ex, t.ey = d0.rows_x, d0.tile_y, d0.ex, d0.ey
                t.tk_z, t.ez, t.z_groups = tk, ez, groups
                try:
                    plan = B.Plan(desc, tuning=t)
                except B.DDStressError as e:
                    assert e.status == B.E_INVALID
                    continue
                _say(f"[long-z] {name} precision={precision} Pz={Pz} groups={groups} ez={ez} tk={tk}")
                plan.set_density(rho)
                out = plan.new_output()
                plan.stress(out)
                torch.cuda.synchronize()
                got = out.double().cpu().numpy()
                plan.close()
                comp, whole = rel_l2(got, ref)
                assert np.all(comp <= TOL[precision]) and whole <= TOL[precision], (groups, ez, tk, comp, whole)
                ran.append((groups, ez, tk))
    _say(f"  {len(ran)} forms: {ran}")
    assert any(g == 1 for g, _, _ in ran)
    assert len({e for _, e, _ in ran}) >= 2            # a longer element class ran too
    if C <= 6 and (precision == 32 or C == 3):
        assert any(g == C for g, _, _ in ran)          # the grouped form fits here


@pytest.mark.parametrize("precision", [32, 64])
def test_poly_layer_256x256x128_golden(precision):
    """The largest served shape, 256 x 256 x 128 (Pz = 256, Px = Py = 512),
    FP32 through an autotuned plan (the launch shapes the server and the
    benchmark use) and FP64 with the default shapes, against stored oracle
    values at 10 cells."""
    import torch
    from paper_1804_01830_amd import binding as B
    from paper_1804_01830_amd import tuning as Tn
    g = _load_golden("poly_layer_256x256x128")
    w = W.poly_layer(nz=128)
    assert list(w["n"]) == g["n"] and np.allclose(w["lines"], g["lines"])
    desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=precision)
    tune = Tn.get_tuning(desc) if precision == 32 else None
    plan = B.Plan(desc, tuning=tune)
    info = plan.info()
    _say(f"[poly-layer-256x256x128] precision={precision} padded={tuple(info.padded)} tile_z={info.tile_z} "
         f"ez={info.ez} z_groups={info.z_groups}")
    dt = torch.float32 if precision == 32 else torch.float64
    plan.set_density(torch.from_numpy(w["rho"]).to("cuda", dtype=dt))
    out = plan.new_output()
    plan.stress(out)
    torch.cuda.synchronize()
    tg = np.array(g["targets"])
    got = out[0][:, tg[:, 2], tg[:, 1], tg[:, 0]].double().cpu().numpy()
    plan.close()
    comp, whole = rel_l2(got, np.array(g["sigma_voigt"]).T)
    _say(f"  per component {np.array2string(comp, precision=2)} whole {whole:.2e}")
    assert np.all(comp <= TOL[precision]) and whole <= TOL[precision]


@pytest.mark.parametrize("case", [
    dict(n=(128, 128, 32), d=(1.0, 1.0, 2.0), lines=[(0.0, 0.0, 1.0)]),
    dict(n=(256, 256, 64), d=(1.0, 1.0, 2.0), lines=[(0.0, 0.0, 1.0), TILT]),
    dict(n=(20, 14, 10), d=(1.0, 1.5, 2.0), lines=[DIAG, TILT, (1.0, 0.0, 0.0)]),
    dict(n=(64, 64, 16), d=(1.0, 1.0, 2.0), lines=[(0.0, 0.0, 1.0), TILT], periodic=(True, True)),
    dict(n=(2, 2, 512), d=(1.0, 1.0, 1.0), lines=[(0.0, 0.0, 1.0)]),
])
def test_kernel_spectrum_is_imaginary(case):
    """K is odd (K(-D) = -K(D), Sec. 2.3 with the symmetric subdivision), so
    its transform is purely imaginary and the plan keeps Im K^ only; the real
    part it measures while building must be rounding-level (plan creation
    checks the same bound and would refuse the plan otherwise)."""
    from paper_1804_01830_amd import binding as B
    desc = B.make_desc(case["n"], case["d"], 1.0, 0.3, case["lines"], precision=64,
                       periodic=case.get("periodic", (False, False)))
    plan = B.Plan(desc)
    info = plan.info()
    plan.close()
    ratio = info.kernel_real_max / info.kernel_imag_max
    _say(f"[spectrum] n={case['n']} periodic={case.get('periodic')} max|Re|={info.kernel_real_max:.3e} "
         f"max|Im|={info.kernel_imag_max:.3e} ratio={ratio:.2e}")
    assert info.kernel_imag_max > 0.0 and ratio <= 1e-13


# The wave form of the fused z pass (FP32, z length 64: Nz 17..32): one wave
# per 8-column tile and realisation, forced through the tuning struct, on
# ragged grids, one to three line directions and batches that leave some
# waves of a block idle.
WAVE = {
    "rand-21x13x20-L1-B3": lambda: W.random_field((21, 13, 20), n_lines=1, batch=3, seed=41, d=(1.0, 1.0, 2.0)),
    # two line directions whose planes all have a z parity (kz <= 32 stored): the tile fits 64 KiB
    "rand-9x30x32-L2-B5": lambda: W.random_field((9, 30, 32), batch=5, seed=42, d=(1.0, 1.5, 2.0),
                                                 lines=[(0.0, 0.0, 1.0), (1.0, 0.0, 0.0)]),
    "rand-40x24x25-L1-B2-tilt": lambda: W.random_field((40, 24, 25), batch=2, seed=44, d=(1.0, 1.0, 2.0),
                                                       lines=[TILT]),
}


@functools.lru_cache(maxsize=None)
def _wave_case(name):
    w = WAVE[name]()
    ref = np.stack([stress_direct(w["rho"][b], w["d"], w["lines"], w["mu"], w["nu"])
                    for b in range(w["rho"].shape[0])])
    return w, ref


@pytest.mark.parametrize("name", list(WAVE))
def test_wave_form_matches_the_oracle(name):
    import torch
    from paper_1804_01830_amd import binding as B
    w, ref = _wave_case(name)
    nb = w["rho"].shape[0]
    desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=32, batch=nb)
    d0 = B.Plan(desc).info()
    assert d0.padded[2] == 64
    t = B.Tuning()
    t.rows_x, t.tk_y, t.ex, t.ey = d0.rows_x, d0.tile_y, d0.ex, d0.ey
    t.tk_z, t.ez, t.z_groups = 8, 8, 1
    rho = torch.from_numpy(w["rho"]).to("cuda", dtype=torch.float32).contiguous()
    outs = []
    for tuning in (t, None):
        plan = B.Plan(desc, tuning=tuning)
        info = plan.info()
        plan.set_density(rho)
        out = plan.new_output()
        plan.stress(out)
        torch.cuda.synchronize()
        outs.append(out.double().cpu().numpy())
        if tuning is t:
            assert (info.ez, info.tile_z, info.z_groups) == (8, 8, 1)
            # a call on fewer realisations (idle waves in every block)
            part = torch.empty((1, 6, *rho.shape[2:]), dtype=torch.float32, device="cuda")
            plan.stress_batch(rho[nb - 1:].contiguous(), part, 1)
            torch.cuda.synchronize()
            assert torch.equal(part[0], out[nb - 1])
        plan.close()
    comp, whole = rel_l2(outs[0], ref)
    _say(f"[wave form] {name}: per component {np.array2string(comp, precision=2)} whole {whole:.2e}")
    assert np.all(comp <= TOL[32]) and whole <= TOL[32]
    # against the default (single-group, element class 4) form: FP32 rounding apart
    assert np.linalg.norm(outs[0] - outs[1]) <= 1e-6 * np.linalg.norm(outs[1])


def test_wave_form_refuses_other_tiles_groups_and_large_tiles():
    """The wave form takes 8-column tiles and one thread group, and its
    staged spectrum tile must fit 64 KiB of LDS (three line directions with
    no z parity need more)."""
    from paper_1804_01830_amd import binding as B
    for lines, bad in (([(0, 0, 1)], ((16, 1), (4, 1), (8, 3))), ([(0, 0, 1), TILT, DIAG], ((8, 1),))):
        desc = B.make_desc((20, 16, 30), (1, 1, 2), 1.0, 0.3, lines, precision=32, batch=2)
        d0 = B.Plan(desc).info()
        for tk, groups in bad:
            t = B.Tuning()
            t.rows_x, t.tk_y, t.ex, t.ey = d0.rows_x, d0.tile_y, d0.ex, d0.ey
            t.tk_z, t.ez, t.z_groups = tk, 8, groups
            with pytest.raises(B.DDStressError) as e:
                B.Plan(desc, tuning=t)
            assert e.value.status == B.E_INVALID
