"""Continuous-batching stress server.

Requests (a geometry and one density) arrive over time. The server keeps, per
geometry ("shape"), one kernel spectrum in device memory and a few *slots*:
plans that share that spectrum, each with its own work buffers, stream and
staging buffers for up to ``max_batch`` densities. Whenever a slot is free,
the waiting requests of its shape (oldest first, up to ``max_batch``) are
copied into it and evaluated with one batched call; slots of different
shapes, and several slots of one shape, run concurrently on their own
streams. A new slot (and, for a new shape, its spectrum) is admitted only if
its device footprint fits the HBM budget; shapes with no waiting or running
work are evicted, least recently used first, to make room.

Results count against the budget too: a launched batch reserves the bytes of
its results, and they stay reserved until the caller releases each request
(``Server.release``, typically from the ``on_complete`` callback of ``run``
once the result has been consumed). A server whose budget is held by
unreleased results and that has nothing in flight raises instead of waiting.

The executor is pluggable: ``GpuExecutor`` drives the HIP library through the
binding; tests drive the same scheduler with a simulated executor.
Latency runs from a request's arrival to the completion of its batch. On the
GPU the completion is the device timestamp of an event recorded after the
batch, placed on the host's clock through one reference event whose device and
host times were taken together (so the host's polling delay does not enter).
"""
import collections
import heapq
import itertools
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class ShapeKey:
    """Everything that fixes a plan's kernel spectrum."""
    n: tuple
    d: tuple
    mu: float
    nu: float
    lines: tuple          # tuple of 3-tuples
    precision: int = 32
    near_shells: int = 0
    periodic: tuple = (False, False)     # periodic boundaries along x, y
    pbc_shells: int = 0

    @property
    def cells(self):
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def channels(self):
        return 3 * len(self.lines)


@dataclass
class Request:
    rid: int
    key: ShapeKey
    rho: object                 # (C, Nz, Ny, Nx) device tensor (GPU) or any payload (simulated)
    arrival: float
    start: float = None         # launch time of its batch
    done: float = None
    result: object = None
    batch_size: int = 0
    polled: float = None        # host time at which the server saw the completion
    device_clock: bool = False  # `done` is a device timestamp (on the host's clock)
    held_bytes: int = 0         # result bytes reserved against the budget until released

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival

    @property
    def host_latency(self):
        return None if self.polled is None else self.polled - self.arrival


@dataclass
class Slot:
    key: ShapeKey
    handle: object
    busy: bool = False
    requests: list = field(default_factory=list)
    last_used: float = 0.0


class Server:
    def __init__(self, executor, hbm_budget, max_batch=4, max_slots_per_shape=2):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.max_slots = int(max_slots_per_shape)
        self.pending = collections.OrderedDict()      # key -> deque of requests
        self.shapes = {}                               # key -> dict(cached=, slots=[...], last_used=)
        self.used = 0
        self.peak_used = 0
        self.results_held = 0                          # bytes of unreleased results
        self.completed = []
        self.batches = []                              # (key, size) of every launch
        self.max_inflight = 0
        self.evictions = 0

    # ---- bookkeeping -------------------------------------------------------
    def submit(self, req):
        if req.key not in self.shapes:
            cached, slot_bytes = self.ex.footprint(req.key, self.max_batch)
            if cached + slot_bytes + self.ex.result_bytes(req.key) > self.budget:
                raise ValueError(f"request {req.rid}: shape {req.key.n} needs {cached + slot_bytes} bytes, "
                                 f"more than the HBM budget {self.budget}")
        self.pending.setdefault(req.key, collections.deque()).append(req)

    def release(self, req):
        """Return a completed request's result bytes to the budget (the
        result itself is dropped)."""
        if req.held_bytes:
            self.used -= req.held_bytes
            self.results_held -= req.held_bytes
            req.held_bytes = 0
        req.result = None

    def inflight(self):
        return sum(1 for sh in self.shapes.values() for s in sh["slots"] if s.busy)

    def idle(self):
        return not any(self.pending.values()) and self.inflight() == 0

    def _note_used(self):
        self.peak_used = max(self.peak_used, self.used)

    def _evict_for(self, need, protect):
        """Free idle shapes (no pending, no running work), LRU first, until
        `need` more bytes fit. Returns True if they fit."""
        while self.used + need > self.budget:
            victims = [(sh["last_used"], k) for k, sh in self.shapes.items()
                       if k != protect and not any(s.busy for s in sh["slots"]) and not self.pending.get(k)]
            if not victims:
                return False
            _, k = min(victims, key=lambda v: v[0])
            sh = self.shapes.pop(k)
            for s in sh["slots"]:
                self.ex.close_slot(s.handle)
            self.ex.close_shape(k)
            self.used -= sh["cached"] + sum(sh["slot_bytes"] for _ in sh["slots"])
            self.evictions += 1
        return True

    def _free_slot(self, key, now, extra=0):
        """A free slot of `key`, admitting a new slot (and the shape's
        spectrum) if the budget allows, with room for `extra` more bytes
        (the batch's results); None if the request must wait."""
        sh = self.shapes.get(key)
        if sh is not None:
            for s in sh["slots"]:
                if not s.busy:
                    return s if self._evict_for(extra, key) else None
            if len(sh["slots"]) >= self.max_slots:
                return None
            need = sh["slot_bytes"]
        else:
            cached, slot_bytes = self.ex.footprint(key, self.max_batch)
            need = cached + slot_bytes
        if not self._evict_for(need + extra, key):
            return None
        if sh is None:
            cached, slot_bytes = self.ex.footprint(key, self.max_batch)
            self.ex.open_shape(key)
            sh = self.shapes[key] = dict(cached=cached, slot_bytes=slot_bytes, slots=[], last_used=now)
            self.used += cached
        slot = Slot(key=key, handle=self.ex.new_slot(key, self.max_batch))
        sh["slots"].append(slot)
        self.used += sh["slot_bytes"]
        self._note_used()
        return slot

    # ---- one scheduling round ------------------------------------------------
    def step(self, now):
        """One scheduling round; returns the requests completed in it."""
        done = []
        for key, sh in self.shapes.items():
            for s in sh["slots"]:
                if s.busy and self.ex.poll(s.handle):
                    t_done = self.ex.finish(s.handle, s.requests)
                    for r in s.requests:
                        r.done = t_done if t_done is not None else now
                        r.polled = now
                        self.completed.append(r)
                        done.append(r)
                    s.busy = False
                    s.requests = []
        # admission and launches, oldest waiting request first
        order = sorted(((q[0].arrival, q[0].rid), k) for k, q in self.pending.items() if q)
        for _, key in order:
            q = self.pending[key]
            while q:
                nb = min(self.max_batch, len(q))
                res_bytes = nb * self.ex.result_bytes(key)
                slot = self._free_slot(key, now, extra=res_bytes)
                if slot is None:
                    break
                batch = [q.popleft() for _ in range(nb)]
                for r in batch:                       # reserved until released
                    r.held_bytes = self.ex.result_bytes(key)
                self.used += res_bytes
                self.results_held += res_bytes
                self._note_used()
                for r in batch:
                    r.start = now
                    r.batch_size = len(batch)
                slot.busy = True
                slot.requests = batch
                slot.last_used = now
                self.shapes[key]["last_used"] = now
                self.ex.launch(slot.handle, batch)
                self.batches.append((key, len(batch)))
        self.max_inflight = max(self.max_inflight, self.inflight())
        if self.inflight() == 0 and any(self.pending.values()) and not done:
            # nothing runs and nothing could be admitted: only releases can help
            waiting = sum(len(q) for q in self.pending.values())
            raise RuntimeError(f"{waiting} requests wait but the budget ({self.budget} bytes) is held by "
                               f"{self.results_held} bytes of unreleased results; release completed requests")
        return done

    # ---- drivers -------------------------------------------------------------
    def run(self, requests, clock, sleep=None, idle_wait=0.0, on_complete=None):
        """Feed `requests` (sorted by arrival) as `clock()` passes their
        arrival times; returns when all are complete. `on_complete(server,
        request)` is called once per completed request (it may consume the
        result and release the request)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        if hasattr(clock, "at"):
            for r in reqs:
                clock.at(r.arrival)
        i = 0
        while i < len(reqs) or not self.idle():
            now = clock()
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            done = self.step(now)
            while done and on_complete is not None:
                for r in done:
                    on_complete(self, r)
                done = self.step(now)        # admit what the releases made room for, at once
            if sleep is not None:
                sleep(idle_wait)
        return self.stats()

    def stats(self):
        lat = np.array([r.latency for r in self.completed], dtype=np.float64)
        host = np.array([r.host_latency for r in self.completed], dtype=np.float64)
        cells = sum(r.key.cells for r in self.completed)
        t0 = min((r.arrival for r in self.completed), default=0.0)
        t1 = max((r.done for r in self.completed), default=0.0)
        makespan = t1 - t0
        sizes = [b for _, b in self.batches]
        device = bool(self.completed) and all(r.device_clock for r in self.completed)
        return {
            "requests": len(self.completed),
            "latency_clock": "device completion events" if device else "host clock",
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
            "mean_ms": float(lat.mean() * 1e3) if len(lat) else None,
            "host_p50_ms": float(np.percentile(host, 50) * 1e3) if len(host) else None,
            "host_p99_ms": float(np.percentile(host, 99) * 1e3) if len(host) else None,
            "cells_per_s": cells / makespan if makespan and makespan > 0 else None,
            "makespan_s": makespan,
            "batches": len(sizes),
            "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
            "max_inflight": self.max_inflight,
            "evictions": self.evictions,
            "hbm_used_bytes": self.used,
            "hbm_peak_bytes": self.peak_used,
            "results_held_bytes": self.results_held,
        }


def poisson_arrivals(rate, count, seed, t0=0.0):
    """Arrival times of a Poisson process of `rate` per second."""
    rng = np.random.default_rng(seed)
    return t0 + np.cumsum(rng.exponential(1.0 / rate, size=count))


class GpuExecutor:
    """Executor on the HIP library: one base plan (owner of the kernel
    spectrum) per shape and, per slot, a plan sharing that spectrum with its
    own stream, staging buffers and completion event. Slots use graph replay
    (their buffers never move)."""

    def __init__(self, use_graph=True, tune=False):
        import torch
        from . import binding
        self.torch = torch
        self.B = binding
        self.use_graph = use_graph
        self.tune = tune
        self.base = {}
        self.t0 = time.perf_counter()
        self.calibrate()

    def calibrate(self, samples=8):
        """Reference event for placing device timestamps on the host clock:
        recorded on an idle device between two host readings; the pair with
        the shortest gap is kept and the event taken at its midpoint (error
        below half that gap, tens of microseconds)."""
        torch = self.torch
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        best = None
        for _ in range(samples):
            ev = torch.cuda.Event(enable_timing=True)
            h0 = self.clock()
            ev.record(stream)
            ev.synchronize()
            h1 = self.clock()
            if best is None or h1 - h0 < best[2] - best[1]:
                best = (ev, h0, h1)
        self.ref_event, self.ref_host = best[0], 0.5 * (best[1] + best[2])
        self.ref_error = 0.5 * (best[2] - best[1])

    def device_time(self, ev):
        """Host-clock time (s) at which the completed event `ev` executed."""
        return self.ref_host + self.ref_event.elapsed_time(ev) * 1e-3

    def result_bytes(self, key):
        nx, ny, nz = key.n
        return 6 * nx * ny * nz * (4 if key.precision == 32 else 8)

    def _desc(self, key, batch):
        return self.B.make_desc(key.n, key.d, key.mu, key.nu, key.lines, precision=key.precision, batch=batch,
                                near_shells=key.near_shells, periodic=key.periodic, pbc_shells=key.pbc_shells)

    def footprint(self, key, batch):
        """(bytes per shape, bytes per slot): the shape's base plan holds the
        kernel spectrum and its own batch-1 work buffers; a slot holds a
        shared plan's work buffers and its density and stress staging."""
        cached, work, _ = self.B.footprint(self._desc(key, batch))
        _, base_work, _ = self.B.footprint(self._desc(key, 1))
        nx, ny, nz = key.n
        elem = 4 if key.precision == 32 else 8
        staging = batch * (key.channels + 6) * nx * ny * nz * elem
        return cached + base_work, work + staging

    def open_shape(self, key):
        desc = self._desc(key, 1)
        if self.tune:
            from . import tuning
            self.base[key] = tuning.tuned_plan(desc)
        else:
            self.base[key] = self.B.Plan(desc)

    def close_shape(self, key):
        self.base.pop(key).close()

    def new_slot(self, key, batch):
        torch = self.torch
        plan = self.base[key].share(batch)
        plan.set_graph(self.use_graph)
        nx, ny, nz = key.n
        dt = torch.float32 if key.precision == 32 else torch.float64
        return dict(plan=plan, stream=torch.cuda.Stream(), event=None, key=key, batch=batch,
                    rho=torch.empty((batch, key.channels, nz, ny, nx), dtype=dt, device="cuda"),
                    out=torch.empty((batch, 6, nz, ny, nx), dtype=dt, device="cuda"))

    def close_slot(self, slot):
        slot["plan"].close()

    def launch(self, slot, requests):
        torch = self.torch
        s = slot["stream"]
        s.wait_stream(torch.cuda.current_stream())     # request densities were written on the current stream
        with torch.cuda.stream(s):
            for i, r in enumerate(requests):
                slot["rho"][i].copy_(r.rho, non_blocking=True)
                r.rho.record_stream(s)                 # the caller may drop it before the copy runs
            nb = len(requests)
            slot["plan"].stress_batch(slot["rho"][:nb], slot["out"][:nb], nb, stream=s)
            for i, r in enumerate(requests):
                r.result = slot["out"][i].clone()      # allocated on s; counted by the server until released
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        slot["event"] = ev

    def poll(self, slot):
        return slot["event"] is not None and slot["event"].query()

    def finish(self, slot, requests):
        ev = slot["event"]
        slot["event"] = None
        for r in requests:
            r.device_clock = True
        return self.device_time(ev)

    def clock(self):
        return time.perf_counter() - self.t0


class SimExecutor:
    """Simulated executor for scheduler tests: a launch completes
    `latency(key, nb)` after it starts, on a virtual clock; payloads are
    echoed as results."""

    def __init__(self, footprints, latency, clock, result_sizes=None):
        self.fp = footprints          # key -> (cached, slot_bytes)
        self.result_sizes = result_sizes or {}    # key -> bytes of one result
        self.lat = latency
        self.clock = clock
        self.opened = []
        self.closed = []
        self.live = 0
        self._ids = itertools.count()

    def footprint(self, key, batch):
        return self.fp[key]

    def result_bytes(self, key):
        return self.result_sizes.get(key, 0)

    def open_shape(self, key):
        self.opened.append(key)

    def close_shape(self, key):
        self.closed.append(key)

    def new_slot(self, key, batch):
        self.live += 1
        return {"key": key, "until": None, "id": next(self._ids)}

    def close_slot(self, slot):
        self.live -= 1

    def launch(self, slot, requests):
        slot["until"] = self.clock() + self.lat(slot["key"], len(requests))
        if hasattr(self.clock, "at"):
            self.clock.at(slot["until"])
        for r in requests:
            r.result = r.rho

    def poll(self, slot):
        return slot["until"] is not None and self.clock() >= slot["until"]

    def finish(self, slot, requests):
        t = slot["until"]
        slot["until"] = None
        return t


class VirtualClock:
    """Event-driven clock for simulations: advances to the next arrival or
    completion each time it is read after a sleep."""

    def __init__(self):
        self.now = 0.0
        self._events = []

    def __call__(self):
        return self.now

    def at(self, t):
        heapq.heappush(self._events, t)

    def advance(self, _=None):
        while self._events and self._events[0] <= self.now:
            heapq.heappop(self._events)
        self.now = heapq.heappop(self._events) if self._events else self.now + 1e-3
