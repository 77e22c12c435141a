"""Parity of the free-surface relaxation (Sec. 5, Eq. 14-18) on the device
with the FP64 oracle, through the C ABI.

The explicit iteration is deterministic, so the device state after n steps
is compared with the oracle's after the same n steps: FP64 within 1e-12 of
the largest displacement (relative max error), FP32 within 1e-5 (relative
L2). The total stress after those steps and the update norm are compared the
same way.
"""
import functools
import sys

import numpy as np
import pytest

from oracle.relax import relax, total_stress, update_norm
from paper_1804_01830_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _device(w, precision, steps, dt=0.0):
    import torch
    from paper_1804_01830_amd import binding as B
    r = B.Relax(w["n"], w["d"], w["mu"], w["nu"], precision=precision, dt=dt)
    td = torch.float32 if precision == 32 else torch.float64
    sig = torch.from_numpy(w["sigma"]).to("cuda", dtype=td).contiguous()
    r.set_load(sig)
    r.iterate(steps)
    u = r.displacement()
    tot = r.stress(sig)
    nrm = r.update_norm()
    torch.cuda.synchronize()
    info = r.info()
    out = (u.double().cpu().numpy(), tot.double().cpu().numpy(), nrm, info)
    r.close()
    return out


CASES = {
    "rand-5x7x3": (lambda: W.random_stress((5, 7, 3), seed=1, d=(1.0, 1.5, 0.7)), 30),
    "rand-17x9x6-nu0.2": (lambda: W.random_stress((17, 9, 6), seed=2, d=(1.0, 1.0, 2.0), nu=0.2), 40),
    "rand-70x3x4": (lambda: W.random_stress((70, 3, 4), seed=3, d=(0.5, 1.0, 1.0)), 25),
    "rand-1x1x3": (lambda: W.random_stress((1, 1, 3), seed=4), 10),
    "smooth-64x48x9": (lambda: W.random_stress((64, 48, 9), seed=5, d=(1.0, 1.0, 2.0), smooth=True), 60),
}


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("name", list(CASES))
def test_relaxation_steps_match_the_oracle(name, precision):
    make, steps = CASES[name]
    w = make()
    _say(f"[relax] {name} precision={precision} steps={steps}")
    u_ref = relax(w["sigma"], w["d"], w["mu"], w["nu"], steps)
    s_ref = total_stress(u_ref, w["sigma"], w["d"], w["mu"], w["nu"])
    n_ref = update_norm(u_ref, w["sigma"], w["d"], w["mu"], w["nu"])
    u, s, nrm, info = _device(w, precision, steps)
    assert info.steps == steps
    if precision == 64:
        eu = np.abs(u - u_ref).max() / np.abs(u_ref).max()
        es = np.abs(s - s_ref).max() / np.abs(s_ref).max()
        _say(f"  max rel err u {eu:.2e} sigma {es:.2e} norm {nrm:.6e} vs {n_ref:.6e}")
        assert eu <= 1e-12 and es <= 1e-12 and abs(nrm - n_ref) <= 1e-12 * n_ref
    else:
        eu = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        es = np.linalg.norm(s - s_ref) / np.linalg.norm(s_ref)
        _say(f"  rel L2 u {eu:.2e} sigma {es:.2e} norm {nrm:.6e} vs {n_ref:.6e}")
        assert eu <= 1e-5 and es <= 1e-5 and abs(nrm - n_ref) <= 1e-4 * n_ref


def test_uniform_linear_load_relaxes_to_the_closed_form():
    import torch
    from paper_1804_01830_amd import binding as B
    n, d, mu, nu = (8, 4, 9), (1.0, 1.0, 0.5), 1.0, 0.3
    z = np.arange(n[2]) * d[2]
    rng = np.random.default_rng(3)
    a, b = rng.uniform(-1, 1, 6), rng.uniform(-1, 1, 6)
    sig = np.stack([np.broadcast_to((a[v] + b[v] * z)[:, None, None], (n[2], n[1], n[0])) for v in range(6)])
    r = B.Relax(n, d, mu, nu, precision=64)
    s = torch.from_numpy(np.ascontiguousarray(sig)).cuda()
    r.set_load(s)
    first = r.update_norm()
    steps, final = r.solve(1e-13, 20000, check_every=200)
    assert steps < 20000 and final <= 1e-13 * first              # stopped by the tolerance
    assert steps == r.info().steps and steps % 200 == 0
    tot = r.stress(s).cpu().numpy()
    r.close()
    k = nu / (1 - nu)
    _say(f"[relax closed form] steps {steps}")
    scale = np.abs(sig).max()
    for v in (2, 3, 4):
        assert np.abs(tot[v]).max() < 1e-9 * scale
    assert np.abs(tot[0] - (sig[0] - k * sig[2])).max() < 1e-9 * scale
    assert np.abs(tot[5] - sig[5]).max() < 1e-9 * scale


def test_stress_in_place_and_state_errors():
    import torch
    from paper_1804_01830_amd import binding as B
    w = W.random_stress((6, 5, 4), seed=7)
    r = B.Relax(w["n"], w["d"], w["mu"], w["nu"], precision=64)
    with pytest.raises(B.DDStressError) as e:
        r.iterate(1)
    assert e.value.status == B.E_STATE
    s = torch.from_numpy(w["sigma"]).cuda()
    r.set_load(s)
    r.iterate(5)
    a = r.stress(s)
    b = s.clone()
    r.stress(b, out=b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # a second load restarts from u = 0
    r.set_load(s)
    r.iterate(5)
    assert torch.equal(r.stress(s), a)
    r.close()


@functools.lru_cache(maxsize=None)
def _layer_256():
    w = W.random_stress((256, 256, 64), seed=11, d=(1.0, 1.0, 2.0), nu=0.2, smooth=True)
    return w, relax(w["sigma"], w["d"], w["mu"], w["nu"], 6)


@pytest.mark.parametrize("precision", [64, 32])
def test_layer_256_full_size_steps(precision):
    """256 x 256 x 64 nodes (the periodic layer's grid, dz = 2 dx), smooth load,
    a few steps in the launch configuration the benchmark times, full field."""
    w, u_ref = _layer_256()
    u, s, nrm, _ = _device(w, precision, 6)
    err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    _say(f"[relax 256] precision={precision} rel L2 u {err:.2e}")
    assert err <= (1e-12 if precision == 64 else 1e-5)


@pytest.mark.parametrize("precision", [64, 32])
def test_relaxed_total_stress_is_traction_free_on_both_surfaces(precision):
    """Eq. (16b) on the device: after any number of steps the total sigma_zz,
    sigma_yz, sigma_xz vanish on the first and last node layers (the ghost
    layers carry the discretised condition), while inside they do not."""
    w = W.random_stress((40, 24, 7), seed=12, d=(1.0, 1.0, 2.0), smooth=True)
    _, tot, _, _ = _device(w, precision, 37)
    scale = np.abs(w["sigma"]).max()
    tol = 1e-12 if precision == 64 else 2e-5
    for v in (2, 3, 4):
        for k in (0, 6):
            assert np.abs(tot[v, k]).max() <= tol * scale, (v, k)
    assert np.abs(tot[2, 3]).max() > 1e-3 * scale
