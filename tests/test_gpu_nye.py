"""Axis-basis (Nye) channels on the device: the channel kernel against the
oracle's definition, accumulation of several dislocation families, and the
whole path with the three axis line directions (C = 9) against the direct
sum of the same channels (FP64 <= 1e-12, FP32 <= 1e-5 relative L2)."""
import sys

import numpy as np
import pytest

from gpu_util import rel_l2
from oracle.direct import stress_direct
from oracle.nye import AXES, nye_channels
from paper_1804_01830_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(x, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=dt).contiguous()


@pytest.mark.parametrize("precision", [64, 32])
def test_channels_match_the_definition(precision):
    import torch
    from paper_1804_01830_amd import binding as B
    w = W.poly_layer_lines(40, 24, 6, grain=6.0, batch_seeds=[1, 2])
    dt = torch.float32 if precision == 32 else torch.float64
    rho = B.nye_density(_dev(w["density"], dt), _dev(w["t"], dt), _dev(w["b"], dt)).cpu().numpy()
    nd, td, bd = (x.astype(np.float32 if precision == 32 else np.float64) for x in (w["density"], w["t"], w["b"]))
    for r in range(2):
        ref = nye_channels(nd[r], td[r], bd[r])
        if precision == 64:
            assert np.array_equal(rho[r], ref)
        else:
            assert np.abs(rho[r] - ref).max() <= 2e-7 * np.abs(ref).max()


def test_families_accumulate():
    import torch
    from paper_1804_01830_amd import binding as B
    w1 = W.poly_layer_lines(16, 16, 4, grain=4.0, seed=5)
    w2 = W.poly_layer_lines(16, 16, 4, grain=4.0, seed=6)
    dt = torch.float64
    rho = B.nye_density(_dev(w1["density"], dt), _dev(w1["t"], dt), _dev(w1["b"], dt))
    B.nye_density(_dev(w2["density"], dt), _dev(w2["t"], dt), _dev(w2["b"], dt), rho=rho, accumulate=True)
    ref = nye_channels(w1["density"][0], w1["t"][0], w1["b"][0]) + nye_channels(w2["density"][0], w2["t"][0],
                                                                               w2["b"][0])
    assert np.abs(rho.cpu().numpy()[0] - ref).max() <= 1e-15 * np.abs(ref).max()


@pytest.mark.parametrize("precision", [64, 32])
def test_axis_basis_stress_matches_the_direct_sum(precision):
    import torch
    from paper_1804_01830_amd import binding as B
    w = W.poly_layer_lines(20, 12, 6, d=(1.0, 1.0, 2.0), grain=5.0, batch_seeds=[7, 8], periodic=False)
    dt = torch.float32 if precision == 32 else torch.float64
    rho = B.nye_density(_dev(w["density"], dt), _dev(w["t"], dt), _dev(w["b"], dt))
    desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], B.AXIS_LINES, precision=precision, batch=2)
    plan = B.Plan(desc)
    plan.set_density(rho)
    got = plan.stress(plan.new_output()).double().cpu().numpy()
    plan.close()
    ref = np.stack([stress_direct(nye_channels(w["density"][r], w["t"][r], w["b"][r]), w["d"], AXES, w["mu"],
                                  w["nu"]) for r in range(2)])
    comp, whole = rel_l2(got, ref)
    tol = 1e-12 if precision == 64 else 1e-5
    _say(f"[nye] precision {precision}: per component {np.array2string(comp, precision=2)} whole {whole:.2e}")
    assert np.all(comp <= tol) and whole <= tol


def test_poly_lines_256_full_size_sampled_targets():
    """The axis-basis workload's full size (256 x 256 x 64, periodic x and y,
    15 shells, C = 9) in FP64 and FP32 on sampled cells, with a sparse line
    field (a few source cells with random n, t, b) so the periodic direct sum
    stays cheap."""
    import torch
    from oracle.periodic import stress_direct_periodic
    from paper_1804_01830_amd import binding as B
    w = W.poly_layer_lines()
    rng = np.random.default_rng(61)
    keep = np.zeros((64, 256, 256), dtype=bool)
    for _ in range(7):
        keep[rng.integers(64), rng.integers(256), rng.integers(256)] = True
    keep[0, 0, 0] = keep[63, 255, 255] = True
    n = np.where(keep, rng.uniform(0.5, 1.5, size=keep.shape), 0.0)[None]
    t = rng.normal(size=(1, 3, 64, 256, 256))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    b = rng.uniform(-1, 1, size=(1, 3, 64, 256, 256))
    tg = np.array([[0, 0, 0], [255, 255, 63], [128, 3, 31], [7, 200, 1]]
                  + [[rng.integers(256), rng.integers(256), rng.integers(64)] for _ in range(4)])
    rho_ref = nye_channels(n[0], t[0], b[0])
    ref = stress_direct_periodic(rho_ref, w["d"], AXES, w["mu"], w["nu"], periodic=(True, True), shells=15,
                                 targets=tg)
    for precision, tol in ((64, 1e-12), (32, 1e-5)):
        dt = torch.float32 if precision == 32 else torch.float64
        rho = B.nye_density(_dev(n, dt), _dev(t, dt), _dev(b, dt))
        desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], B.AXIS_LINES, precision=precision,
                           periodic=(True, True))
        plan = B.Plan(desc)
        plan.set_density(rho)
        got = plan.stress(plan.new_output())[0].double().cpu().numpy()[:, tg[:, 2], tg[:, 1], tg[:, 0]]
        plan.close()
        comp, whole = rel_l2(got, ref)
        _say(f"[nye 256] precision {precision}: per component {np.array2string(comp, precision=2)} "
             f"whole {whole:.2e}")
        assert np.all(comp <= tol) and whole <= tol
