"""Stress server on the GPU: requests of several shapes arrive while others
run, are batched per shape into slots that share their shape's kernel
spectrum, and overlap on several streams. Each served result must equal the
same density evaluated alone (plan with batch 1, direct launches) bit for bit,
open and periodic shapes alike.
"""
import numpy as np
import pytest

from paper_1804_01830_amd import workloads as W
from paper_1804_01830_amd.serving import GpuExecutor, Request, Server, ShapeKey, poisson_arrivals

pytestmark = pytest.mark.gpu


def _key(w, precision=32):
    return ShapeKey(n=tuple(w["n"]), d=tuple(w["d"]), mu=w["mu"], nu=w["nu"],
                    lines=tuple(tuple(map(float, t)) for t in w["lines"]), precision=precision,
                    periodic=w.get("periodic", (False, False)), pbc_shells=w.get("pbc_shells", 0))


def _periodic(w, shells):
    w = dict(w)
    w["periodic"], w["pbc_shells"] = (True, True), shells
    return w


@pytest.mark.parametrize("precision", [32, 64])
def test_served_results_equal_alone(precision):
    import torch
    from paper_1804_01830_amd import binding as B
    dt = torch.float32 if precision == 32 else torch.float64
    pools = [W.random_field((24, 16, 8), n_lines=2, batch=4, seed=1, d=(1.0, 1.0, 2.0)),
             W.random_field((40, 20, 6), n_lines=1, batch=4, seed=2),
             W.random_field((16, 16, 16), n_lines=2, batch=4, seed=3, d=(2.0, 1.0, 1.0)),
             _periodic(W.random_field((32, 16, 4), n_lines=2, batch=4, seed=4, d=(1.0, 1.0, 2.0)), 3)]
    keys = [_key(w, precision) for w in pools]
    dens = [torch.from_numpy(w["rho"]).to("cuda", dtype=dt) for w in pools]
    rng = np.random.default_rng(9)
    arrivals = poisson_arrivals(3000.0, 24, seed=4)
    ex = GpuExecutor(use_graph=True)
    reqs = []
    for i, t in enumerate(arrivals):
        s = int(rng.integers(len(pools)))
        j = int(rng.integers(4))
        reqs.append(Request(i, keys[s], rho=dens[s][j], arrival=float(t) + ex.clock()))
        reqs[-1].src = (s, j)
    srv = Server(ex, hbm_budget=8 << 30, max_batch=3, max_slots_per_shape=2)
    st = srv.run(reqs, ex.clock)
    torch.cuda.synchronize()
    print(f"[serve] {st}", flush=True)
    assert st["requests"] == len(reqs) and st["mean_batch"] >= 1.0
    alone = {}
    for s, w in enumerate(pools):
        desc = B.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=precision, batch=4,
                           periodic=w.get("periodic", (False, False)), pbc_shells=w.get("pbc_shells", 0))
        plan = B.Plan(desc)
        for j in range(4):
            out = torch.empty((1, 6, *dens[s].shape[2:]), dtype=dt, device="cuda")
            plan.stress_batch(dens[s][j:j + 1].contiguous(), out, 1)
            alone[(s, j)] = out[0]
        torch.cuda.synchronize()
        plan.close()
    for r in reqs:
        assert torch.equal(r.result, alone[r.src]), f"request {r.rid} shape {r.key.n}"
