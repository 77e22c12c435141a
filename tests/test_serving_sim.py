"""Scheduler of the stress server on a simulated executor (no GPU):
batching, admission by HBM budget, eviction, overlap, admit-on-free and the
latency bookkeeping."""
import numpy as np
import pytest

from paper_1804_01830_amd.serving import (Request, Server, ShapeKey, SimExecutor, VirtualClock,
                                          poisson_arrivals)

A = ShapeKey(n=(64, 64, 64), d=(1, 1, 1), mu=1.0, nu=0.3, lines=((0, 0, 1),))
Bk = ShapeKey(n=(128, 128, 32), d=(1, 1, 2), mu=1.0, nu=0.3, lines=((0, 0, 1),))
GB = 1 << 30


def _sim(footprints, lat=lambda k, nb: 1.0 + 0.5 * nb):
    clock = VirtualClock()
    return SimExecutor(footprints, lat, clock), clock


def _run(server, clock, reqs):
    return server.run(reqs, clock, sleep=clock.advance)


def test_one_shape_batches_up_to_max_batch():
    ex, clock = _sim({A: (2 * GB, 1 * GB)})
    srv = Server(ex, hbm_budget=64 * GB, max_batch=4, max_slots_per_shape=1)
    reqs = [Request(i, A, rho=i, arrival=0.0) for i in range(10)]
    st = _run(srv, clock, reqs)
    assert [b for _, b in srv.batches] == [4, 4, 2]
    assert st["requests"] == 10 and all(r.result == r.rid for r in reqs)
    # one slot: batch k starts when batch k-1 completes (3.0 time units for 4 requests)
    starts = sorted({r.start for r in reqs})
    assert starts == [0.0, 3.0, 6.0]
    assert max(r.done for r in reqs) == pytest.approx(8.0)


def test_tiny_budget_serialises_shapes_and_evicts():
    ex, clock = _sim({A: (2 * GB, 1 * GB), Bk: (3 * GB, 1 * GB)})
    srv = Server(ex, hbm_budget=4 * GB, max_batch=2, max_slots_per_shape=1)
    reqs = [Request(i, A if i % 2 == 0 else Bk, rho=i, arrival=0.1 * i) for i in range(8)]
    st = _run(srv, clock, reqs)
    assert st["requests"] == 8
    assert srv.max_inflight == 1 and st["evictions"] >= 1
    assert srv.used <= 4 * GB
    assert ex.live == sum(len(sh["slots"]) for sh in srv.shapes.values())


def test_shapes_overlap_when_memory_allows():
    ex, clock = _sim({A: (2 * GB, 1 * GB), Bk: (3 * GB, 1 * GB)})
    srv = Server(ex, hbm_budget=64 * GB, max_batch=2, max_slots_per_shape=2)
    reqs = [Request(i, A if i % 2 == 0 else Bk, rho=i, arrival=0.0) for i in range(8)]
    _run(srv, clock, reqs)
    assert srv.max_inflight == 4          # two slots per shape, both shapes at once
    assert srv.evictions == 0


def test_requests_are_admitted_when_a_slot_frees():
    ex, clock = _sim({A: (GB, GB)}, lat=lambda k, nb: 2.0)
    srv = Server(ex, hbm_budget=64 * GB, max_batch=8, max_slots_per_shape=1)
    first = Request(0, A, rho=0, arrival=0.0)
    late = [Request(i, A, rho=i, arrival=0.5 + 0.1 * i) for i in range(1, 4)]
    _run(srv, clock, [first] + late)
    assert first.start == 0.0 and first.done == 2.0
    assert all(r.start == 2.0 and r.batch_size == 3 for r in late)      # continuous batching
    assert all(r.done == 4.0 for r in late)


def test_latency_percentiles():
    ex, clock = _sim({A: (GB, GB)}, lat=lambda k, nb: 1.0)
    srv = Server(ex, hbm_budget=64 * GB, max_batch=1, max_slots_per_shape=1)
    reqs = [Request(i, A, rho=i, arrival=0.0) for i in range(100)]
    st = _run(srv, clock, reqs)
    lat = sorted(r.latency for r in reqs)
    assert lat == [float(i + 1) for i in range(100)]
    assert st["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert st["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)


def test_request_larger_than_budget_is_rejected():
    ex, clock = _sim({A: (8 * GB, 1 * GB)})
    srv = Server(ex, hbm_budget=4 * GB)
    with pytest.raises(ValueError):
        srv.submit(Request(0, A, rho=None, arrival=0.0))


def test_poisson_replay_is_deterministic():
    t1 = poisson_arrivals(100.0, 50, seed=5)
    t2 = poisson_arrivals(100.0, 50, seed=5)
    assert np.array_equal(t1, t2) and np.all(np.diff(t1) > 0)
    outs = []
    for _ in range(2):
        ex, clock = _sim({A: (GB, GB), Bk: (GB, GB)})
        srv = Server(ex, hbm_budget=3 * GB, max_batch=3, max_slots_per_shape=1)
        reqs = [Request(i, A if i % 3 else Bk, rho=i, arrival=float(t)) for i, t in enumerate(t1)]
        _run(srv, clock, reqs)
        outs.append([(r.rid, r.start, r.done) for r in reqs])
    assert outs[0] == outs[1]


def test_results_count_against_the_budget_until_released():
    """Each launched batch reserves its results' bytes; released results
    return them. With a budget that holds one batch of results, the second
    batch waits for the first batch's release."""
    ex, clock = _sim({A: (GB, GB)}, lat=lambda k, nb: 1.0)
    ex.result_sizes[A] = GB // 2
    srv = Server(ex, hbm_budget=3 * GB, max_batch=2, max_slots_per_shape=1)
    reqs = [Request(i, A, rho=i, arrival=0.0) for i in range(4)]
    released_at = []

    def consume(server, r):
        assert server.used <= server.budget
        released_at.append(clock())
        server.release(r)

    st = srv.run(reqs, clock, sleep=clock.advance, on_complete=consume)
    assert st["requests"] == 4 and st["results_held_bytes"] == 0
    assert st["hbm_peak_bytes"] == 3 * GB                 # spectrum + slot + one batch of results
    assert [r.start for r in reqs] == [0.0, 0.0, 1.0, 1.0]


def test_unreleased_results_that_block_admission_raise():
    ex, clock = _sim({A: (GB, GB)}, lat=lambda k, nb: 1.0)
    ex.result_sizes[A] = GB
    srv = Server(ex, hbm_budget=3 * GB, max_batch=1, max_slots_per_shape=1)
    reqs = [Request(i, A, rho=i, arrival=0.0) for i in range(2)]
    with pytest.raises(RuntimeError, match="unreleased results"):
        _run(srv, clock, reqs)
