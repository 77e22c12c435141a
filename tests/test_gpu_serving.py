"""Stress server on the GPU: requests of several shapes arrive while others
run, are batched per shape into slots that share their shape's kernel
spectrum, and overlap on several streams. Every served result is checked
against the FP64 oracle (the direct sum of Eq. 10, or for the periodic shape
the oracle's replica-shell reference of Eq. 12-13) to the tolerances of the
other parity tests, and must equal the same density evaluated alone (plan with
batch 1, direct launches) bit for bit, open and periodic shapes alike. Under a
budget that holds one shape at a time, requests queue, shapes are evicted and
the results are still those of the oracle.
"""
import functools

import numpy as np
import pytest

from gpu_util import rel_l2
from oracle import stress_direct
from oracle.periodic import stress_fft_reference_periodic
from paper_1804_01830_amd import workloads as W
from paper_1804_01830_amd.serving import GpuExecutor, Request, Server, ShapeKey, poisson_arrivals

pytestmark = pytest.mark.gpu

TOL = {64: 1e-12, 32: 1e-5}


def _key(w, precision=32):
    return ShapeKey(n=tuple(w["n"]), d=tuple(w["d"]), mu=w["mu"], nu=w["nu"],
                    lines=tuple(tuple(map(float, t)) for t in w["lines"]), precision=precision,
                    periodic=w.get("periodic", (False, False)), pbc_shells=w.get("pbc_shells", 0))


def _periodic(w, shells):
    w = dict(w)
    w["periodic"], w["pbc_shells"] = (True, True), shells
    return w


def _pools():
    return [W.random_field((24, 16, 8), n_lines=2, batch=4, seed=1, d=(1.0, 1.0, 2.0)),
            W.random_field((40, 20, 6), n_lines=1, batch=4, seed=2),
            W.random_field((16, 16, 16), n_lines=2, batch=4, seed=3, d=(2.0, 1.0, 1.0)),
            _periodic(W.random_field((32, 16, 4), n_lines=2, batch=4, seed=4, d=(1.0, 1.0, 2.0)), 3)]


@functools.lru_cache(maxsize=None)
def _oracle(s, j):
    w = _pools()[s]
    if "periodic" in w:
        return stress_fft_reference_periodic(w["rho"][j], w["d"], w["lines"], w["mu"], w["nu"],
                                             periodic=w["periodic"], shells=w["pbc_shells"])
    return stress_direct(w["rho"][j], w["d"], w["lines"], w["mu"], w["nu"])


def _check_oracle(got, s, j, precision, what):
    comp, whole = rel_l2(np.asarray(got, dtype=np.float64), _oracle(s, j))
    assert np.all(comp <= TOL[precision]) and whole <= TOL[precision], (what, comp, whole)


@pytest.mark.parametrize("precision", [32, 64])
def test_served_results_equal_alone_and_the_oracle(precision):
    import torch
    from paper_1804_01830_amd import binding as B
    dt = torch.float32 if precision == 32 else torch.float64
    pools = _pools()
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
    assert st["latency_clock"] == "device completion events" and all(r.latency > 0 for r in reqs)
    # the device completion precedes the host's poll that noticed it (up to the clock calibration)
    assert all(r.latency <= r.host_latency + ex.ref_error + 1e-4 for r in reqs)
    # every unreleased result is counted against the budget
    assert st["results_held_bytes"] == sum(6 * r.key.cells * dt.itemsize for r in reqs)
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
        _check_oracle(r.result.cpu().numpy(), *r.src, precision, f"request {r.rid} shape {r.key.n}")
    for r in reqs:
        srv.release(r)
    assert srv.results_held == 0


def test_tiny_budget_queues_evicts_and_matches_the_oracle():
    """A budget that fits the largest shape's spectrum, one slot and one
    batch of results: the shapes take turns (requests queue, idle shapes are
    evicted; two small ones may share the budget),
    results are released as they are consumed, the accounted memory never
    exceeds the budget, and every result is the oracle's."""
    import torch
    precision = 32
    pools = _pools()
    keys = [_key(w, precision) for w in pools]
    dens = [torch.from_numpy(w["rho"]).to("cuda", dtype=torch.float32) for w in pools]
    ex = GpuExecutor(use_graph=True)
    max_batch = 2
    need = max(sum(ex.footprint(k, max_batch)) + max_batch * ex.result_bytes(k) for k in keys)
    srv = Server(ex, hbm_budget=need, max_batch=max_batch, max_slots_per_shape=1)
    rng = np.random.default_rng(19)
    reqs = []
    t0 = ex.clock()
    for i in range(16):
        s = i % len(pools)                     # every shape in turn: each arrival needs another shape
        j = int(rng.integers(4))
        reqs.append(Request(i, keys[s], rho=dens[s][j], arrival=t0 + 1e-4 * i))
        reqs[-1].src = (s, j)
    got = {}

    def consume(server, r):
        got[r.rid] = r.result.cpu().numpy()
        server.release(r)

    st = srv.run(reqs, ex.clock, on_complete=consume)
    torch.cuda.synchronize()
    print(f"[serve tiny] budget {need} {st}", flush=True)
    assert st["requests"] == len(reqs) and len(got) == len(reqs)
    assert st["evictions"] >= 3 and st["max_inflight"] < len(pools)     # never all shapes at once
    assert st["hbm_peak_bytes"] <= need and st["results_held_bytes"] == 0
    assert st["latency_clock"] == "device completion events"
    for r in reqs:
        _check_oracle(got[r.rid], *r.src, precision, f"request {r.rid} shape {r.key.n}")
