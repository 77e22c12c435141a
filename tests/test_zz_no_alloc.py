"""The allocation-free entry point ddstress_stress_batch_stats_noalloc
(GPU): the stress and the Eq. (20) plane statistics it writes equal, bit for
bit, those of ddstress_stress_batch on a plan whose statistics are set
(ddstress_plan_set_plane_stats, row sums in a plan-owned buffer), on two
calls in a row of which the second evaluates a smaller input; sizes beyond
its static row-sum scratch are refused."""
import ctypes

import numpy as np
import pytest

from paper_1804_01830_amd import workloads as W

pytestmark = pytest.mark.gpu


def _plan(w, precision, batch):
    from paper_1804_01830_amd import binding as B
    return B.Plan(B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=precision, batch=batch))


def _reference(plan, rho, nb):
    """Stress and statistics through the existing route."""
    import torch
    nx, ny, nz = plan.n
    sig = torch.empty((nb, 6, nz, ny, nx), dtype=rho.dtype, device="cuda")
    stats = torch.empty((plan.batch, 6, nz), dtype=torch.float64, device="cuda")
    plan.set_plane_stats(stats)
    plan.stress_batch(rho[:nb].contiguous(), sig, nb)
    torch.cuda.synchronize()
    plan.set_plane_stats(None)
    return sig, stats[:nb].clone()


@pytest.mark.parametrize("n,lines,precision", [((40, 30, 12), 2, 32), ((72, 70, 5), 1, 32), ((33, 20, 9), 2, 64)])
def test_noalloc_matches_the_plan_route_on_two_calls(n, lines, precision):
    import torch
    w = W.random_field(n, n_lines=lines, batch=3, seed=71, d=(1.0, 1.0, 2.0))
    dt = torch.float32 if precision == 32 else torch.float64
    rho = torch.from_numpy(w["rho"]).to("cuda", dtype=dt).contiguous()
    plan = _plan(w, precision, 3)
    print(f"[noalloc] n={n} C={3 * lines} precision={precision} yx_fused={plan.info().yx_fused}", flush=True)
    nx, ny, nz = n
    for nb in (3, 1):                        # the second call evaluates a smaller input
        ref_sig, ref_stats = _reference(plan, rho, nb)
        sig = torch.full((nb, 6, nz, ny, nx), float("nan"), dtype=dt, device="cuda")
        stats = torch.full((nb, 6, nz), float("nan"), dtype=torch.float64, device="cuda")
        plan.stress_batch_stats_noalloc(rho[:nb].contiguous(), sig, nb, stats)
        torch.cuda.synchronize()
        assert torch.equal(sig, ref_sig), nb
        assert torch.equal(stats, ref_stats), nb
    # the statistics are Eq. (20) of the stress written (mean square over each plane)
    ms = (sig.double() ** 2).mean(dim=(3, 4))
    assert torch.allclose(stats, ms, rtol=1e-12, atol=0.0)
    plan.close()


def test_noalloc_after_a_larger_plan_on_the_same_device():
    """The static array is shared by every plan on the device and keeps the
    last call's contents: a small plan after a larger one still gets its own
    statistics."""
    import torch
    big = W.random_field((48, 40, 16), n_lines=1, batch=2, seed=72)
    small = W.random_field((9, 7, 5), n_lines=1, batch=1, seed=73)
    outs = []
    for w, nb in ((big, 2), (small, 1)):
        rho = torch.from_numpy(w["rho"]).to("cuda", dtype=torch.float32).contiguous()
        plan = _plan(w, 32, nb)
        ref_sig, ref_stats = _reference(plan, rho, nb)
        nx, ny, nz = w["n"]
        sig = torch.empty((nb, 6, nz, ny, nx), dtype=torch.float32, device="cuda")
        stats = torch.empty((nb, 6, nz), dtype=torch.float64, device="cuda")
        plan.stress_batch_stats_noalloc(rho, sig, nb, stats)
        torch.cuda.synchronize()
        assert torch.equal(sig, ref_sig) and torch.equal(stats, ref_stats)
        outs.append(stats)
        plan.close()


def test_noalloc_refuses_sizes_beyond_its_scratch():
    """nbatch * 6 * Nz * Ny row sums must fit the 2^21 doubles of scratch."""
    import torch
    from paper_1804_01830_amd import binding as B
    w = W.random_field((4, 512, 128), n_lines=1, batch=6, seed=74)       # 6 * 6 * 128 * 512 > 2^21
    plan = _plan(w, 32, 6)
    rho = torch.zeros((6, 3, 128, 512, 4), dtype=torch.float32, device="cuda")
    sig = torch.empty((6, 6, 128, 512, 4), dtype=torch.float32, device="cuda")
    stats = torch.empty((6, 6, 128), dtype=torch.float64, device="cuda")
    with pytest.raises(B.DDStressError) as e:
        plan.stress_batch_stats_noalloc(rho, sig, 6, stats)
    assert e.value.status == B.E_UNSUPPORTED and "scratch" in str(e.value)
    # one realisation fits (6 * 128 * 512 = 393216 rows)
    ref_sig, ref_stats = _reference(plan, rho, 1)
    plan.stress_batch_stats_noalloc(rho[:1].contiguous(), sig[:1], 1, stats[:1])
    torch.cuda.synchronize()
    assert torch.equal(stats[:1], ref_stats)
    plan.close()
