"""Parity of periodic-boundary plans (Sec. 4, Eq. 12-13) with the FP64 oracle.

The device builds the replica-shell coefficients F and transforms the
periodic axes at their own length; the oracle sums the same shells in numpy
and evaluates the circular convolution with a library FFT (itself pinned to
the periodic direct sum on the CPU). Tolerances as for open plans: relative
L2 error <= 1e-12 (FP64) and <= 1e-5 (FP32) per component and overall.
"""
import functools
import sys

import numpy as np
import pytest

from gpu_util import gpu_stress, rel_l2
from oracle import KernelGeometry
from oracle.periodic import periodic_kernel, stress_direct_periodic, stress_fft_reference_periodic
from paper_1804_01830_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {64: 1e-12, 32: 1e-5}
TILT = W.mixed_line()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# name: (workload, periodic (x, y), shells; 0 = the library default of 15)
CASES = {
    "pbc-16x16x4-L2-B2-s4": (lambda: W.random_field((16, 16, 4), n_lines=2, batch=2, seed=31, d=(1.0, 1.5, 2.0)),
                             (True, True), 4),
    "pbcy-20x32x5-L2-s3": (lambda: W.random_field((20, 32, 5), n_lines=2, seed=32, d=(1.0, 1.0, 2.0)),
                           (False, True), 3),
    "pbcx-32x9x3-L3-s2": (lambda: W.random_field((32, 9, 3), n_lines=3, seed=33, d=(2.0, 1.0, 1.0)),
                          (True, False), 2),
    # the smallest period: every in-plane offset is 0 or the half period
    "pbc-2x2x3-s3": (lambda: W.random_field((2, 2, 3), n_lines=2, seed=34), (True, True), 3),
    "pbc-8x8x2-default-shells": (lambda: W.random_field((8, 8, 2), n_lines=1, seed=35, lines=[TILT]),
                                 (True, True), 0),
    # the longest periodic axis (transform length 512 = N)
    "pbcx-512x2x2-max-s1": (lambda: W.random_field((512, 2, 2), n_lines=1, seed=36), (True, False), 1),
    # Px = Py = 256 planes: the FP32 path takes the fused x-y kernels with a full-length x row
    "pbcx-256x72x2-s2": (lambda: W.random_field((256, 72, 2), n_lines=1, seed=37, d=(1.0, 1.0, 2.0)),
                         (True, False), 2),
}


@functools.lru_cache(maxsize=None)
def _case(name):
    make, periodic, shells = CASES[name]
    w = make()
    sh = 15 if shells == 0 else shells
    ref = np.stack([stress_fft_reference_periodic(w["rho"][b], w["d"], w["lines"], w["mu"], w["nu"],
                                                  periodic=periodic, shells=sh)
                    for b in range(w["rho"].shape[0])])
    return w, periodic, shells, ref


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("name", list(CASES))
def test_periodic_full_field_parity(name, precision):
    w, periodic, shells, ref = _case(name)
    _say(f"[pbc] {name} precision={precision} n={w['n']} periodic={periodic} shells={shells}")
    got = gpu_stress(w, precision, periodic=periodic, pbc_shells=shells)
    comp, whole = rel_l2(got, ref)
    _say(f"  rel L2 per component {np.array2string(comp, precision=2)} whole {whole:.2e}")
    assert np.all(comp <= TOL[precision]) and whole <= TOL[precision]


@pytest.mark.parametrize("periodic", [(True, True), (True, False), (False, True)])
def test_periodic_kernel_realspace_matches_oracle_entrywise(periodic):
    import torch
    from paper_1804_01830_amd import binding as B
    n, d = (8, 4, 3), (1.0, 1.5, 2.0)
    lines = [(0.0, 0.0, 1.0), TILT]
    desc = B.make_desc(n, d, 1.3, 0.27, lines, precision=64, periodic=periodic, pbc_shells=3)
    P = B.padded_lengths(n, periodic)
    ax, valid = [], []
    for a in range(3):
        i = np.arange(P[a])
        if a < 2 and periodic[a]:
            ax.append(i)
            valid.append(np.ones(P[a], dtype=bool))
        else:
            ax.append(np.where(i < n[a], i, i - P[a]))
            valid.append((i < n[a]) | (i > P[a] - n[a]))
    gz, gy, gx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    vz, vy, vx = np.meshgrid(valid[2], valid[1], valid[0], indexing="ij")
    mask = vz & vy & vx
    offs = np.stack([gx[mask], gy[mask], gz[mask]], axis=-1)
    for l, t in enumerate(lines):
        out = torch.empty((3, 6, P[2], P[1], P[0]), dtype=torch.float64, device="cuda")
        B.kernel_realspace(desc, l, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = periodic_kernel(KernelGeometry(d=d, t=t, mu=1.3, nu=0.27), offs, n, periodic, 3)   # (M, 6, 3)
        g = np.transpose(got, (2, 3, 4, 1, 0))[mask]
        assert np.all(got[:, :, ~mask] == 0.0)
        err = np.abs(g - ref).max() / np.abs(ref).max()
        _say(f"[pbc kernel] periodic={periodic} line {l}: max abs err / max = {err:.2e}")
        assert err < 1e-13


def test_circular_shift_moves_the_device_stress():
    w = W.random_field((16, 8, 3), n_lines=2, seed=38, d=(1.0, 1.0, 2.0))
    a = gpu_stress(w, 64, periodic=(True, True), pbc_shells=2)
    w2 = dict(w)
    w2["rho"] = np.roll(w["rho"], (3, 5), axis=(3, 4))
    b = gpu_stress(w2, 64, periodic=(True, True), pbc_shells=2)
    assert np.abs(np.roll(a, (3, 5), axis=(3, 4)) - b).max() <= 1e-12 * np.abs(a).max()


@functools.lru_cache(maxsize=None)
def _poly_pbc():
    w = W.poly_layer(periodic=True)
    rng = np.random.default_rng(41)
    keep = np.zeros(w["rho"].shape[2:], dtype=bool)
    for _ in range(6):
        keep[rng.integers(64), rng.integers(256), rng.integers(256)] = True
    keep[0, 0, 0] = keep[63, 255, 255] = keep[5, 128, 0] = True
    w["rho"] = np.where(keep[None, None], w["rho"], 0.0)
    w["rho"][0, :, keep] = rng.uniform(-1.0, 1.0, size=(6, int(keep.sum()))).T
    tg = np.array([[0, 0, 0], [255, 255, 63], [128, 5, 32], [0, 128, 5], [255, 0, 0], [17, 200, 1]]
                  + [[rng.integers(256), rng.integers(256), rng.integers(64)] for _ in range(4)])
    ref = stress_direct_periodic(w["rho"][0], w["d"], w["lines"], w["mu"], w["nu"], periodic=(True, True),
                                 shells=15, targets=tg)
    return w, tg, ref, int(keep.sum())


@pytest.mark.parametrize("precision", [64, 32])
def test_poly_layer_pbc_256_sampled_targets(precision):
    """Full-size periodic layer (256 x 256 x 64, dz = 2 dx, edge and mixed
    lines, default 15 shells) with a sparse density (a few source cells with
    random channels), checked on sampled cells against the periodic direct sum."""
    w, tg, ref, nsrc = _poly_pbc()
    _say(f"[poly-layer-pbc-256] precision={precision}: {nsrc} source cells, {len(tg)} targets")
    got = gpu_stress(w, precision, periodic=(True, True))[0][:, tg[:, 2], tg[:, 1], tg[:, 0]]
    comp, whole = rel_l2(got, ref)
    _say(f"  per component {np.array2string(comp, precision=2)} whole {whole:.2e}")
    assert np.all(comp <= TOL[precision]) and whole <= TOL[precision]


def test_single_layer_of_the_smallest_period_has_zero_stress():
    # 2 x 2 x 1 with both axes periodic: every offset is 0 or a half period in
    # the plane and 0 along z, where F is odd and periodic, hence zero
    w = W.random_field((2, 2, 1), n_lines=2, seed=39)
    g = KernelGeometry(d=w["d"], t=tuple(w["lines"][1]), mu=w["mu"], nu=w["nu"])
    scale = np.abs(periodic_kernel(g, np.array([[1, 0, 0]]), (2, 2, 1), (False, False), 0)).max()
    for prec, tol in ((64, 1e-13), (32, 1e-5)):
        got = gpu_stress(w, prec, periodic=(True, True), pbc_shells=3)
        _say(f"[pbc 2x2x1] precision={prec}: max |sigma| / max |K| = {np.abs(got).max() / scale:.2e}")
        assert np.abs(got).max() <= tol * scale * np.abs(w["rho"]).sum()


def test_periodic_plans_refuse_non_power_of_two_axes():
    from paper_1804_01830_amd import binding as B
    desc = B.make_desc((24, 16, 4), (1, 1, 1), 1.0, 0.3, [(0, 0, 1)], precision=32, periodic=(True, True))
    with pytest.raises(B.DDStressError) as e:
        B.Plan(desc)
    assert e.value.status == B.E_UNSUPPORTED


def test_periodic_batches_graphs_and_shared_plans_are_bit_consistent():
    """A periodic plan through the launch variants: partial batches, graph
    replays (eager work between them) and a plan sharing its spectrum give
    the bits of the direct full call."""
    import torch
    from paper_1804_01830_amd import binding as B
    w = W.random_field((32, 16, 4), n_lines=2, batch=3, seed=40, d=(1.0, 1.0, 2.0))
    desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=32, batch=3, periodic=(True, True),
                       pbc_shells=2)
    plan = B.Plan(desc)
    assert tuple(plan.info().padded) == (32, 16, 8)
    rho = torch.from_numpy(w["rho"]).to("cuda", dtype=torch.float32).contiguous()
    ref = torch.empty((3, 6, 4, 16, 32), dtype=torch.float32, device="cuda")
    plan.stress_batch(rho, ref, 3)
    one = torch.empty((1, 6, 4, 16, 32), dtype=torch.float32, device="cuda")
    plan.stress_batch(rho[:1], one, 1)
    torch.cuda.synchronize()
    assert torch.equal(one, ref[:1])
    plan.set_graph(True)
    out = torch.empty_like(ref)
    for rep in range(3):
        out.fill_(float("nan"))
        plan.stress_batch(rho, out, 3)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep}"
        assert torch.isfinite(torch.randn(1 << 18, device="cuda").sum())
    plan.set_graph(False)
    shared = plan.share(1)
    for r in range(3):
        shared.stress_batch(rho[r:r + 1].contiguous(), one, 1)
        torch.cuda.synchronize()
        assert torch.equal(one[0], ref[r])
    shared.close()
    plan.close()


def test_periodic_mirror_compression_matches_the_full_spectrum():
    """The y mirror of a periodic plan (kept rows ky <= Py/2 with signs) gives
    the stress of the full spectrum to rounding."""
    from paper_1804_01830_amd import binding as B
    w = W.random_field((16, 32, 3), n_lines=2, seed=45, d=(1.0, 1.0, 2.0))
    got = {}
    for flags in (0, B.FLAG_FULL_SPECTRUM):
        import torch
        desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=64, flags=flags,
                           periodic=(True, True), pbc_shells=3)
        plan = B.Plan(desc)
        info = plan.info()
        got[flags] = (info.mirror_y, info.mirror_z)
        plan.set_density(torch.from_numpy(w["rho"]).cuda())
        got[(flags, "s")] = plan.stress(plan.new_output()).cpu().numpy()
        plan.close()
    assert got[0][0] == 1 and got[B.FLAG_FULL_SPECTRUM] == (0, 0)
    a, b = got[(0, "s")], got[(B.FLAG_FULL_SPECTRUM, "s")]
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


@functools.lru_cache(maxsize=None)
def _largest_plane():
    w = W.random_field((512, 512, 2), n_lines=1, seed=46, d=(1.0, 1.0, 1.0))
    ref = stress_fft_reference_periodic(w["rho"][0], w["d"], w["lines"], w["mu"], w["nu"], periodic=(True, True),
                                        shells=1)
    return w, ref


@pytest.mark.parametrize("precision", [64, 32])
def test_periodic_largest_plane(precision):
    """512 x 512 periodic plane (the longest periodic axes), one shell."""
    w, ref = _largest_plane()
    got = gpu_stress(w, precision, periodic=(True, True), pbc_shells=1)[0]
    comp, whole = rel_l2(got, ref)
    _say(f"[pbc 512x512] precision={precision} per component {np.array2string(comp, precision=2)} whole {whole:.2e}")
    assert np.all(comp <= TOL[precision]) and whole <= TOL[precision]
