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

The executor is pluggable: ``GpuExecutor`` drives the HIP library through the
binding; tests drive the same scheduler with a simulated executor.
Latency is measured from a request's arrival to the completion of its batch.
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

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


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
        self.completed = []
        self.batches = []                              # (key, size) of every launch
        self.max_inflight = 0
        self.evictions = 0

    # ---- bookkeeping -------------------------------------------------------
    def submit(self, req):
        if req.key not in self.shapes:
            cached, slot_bytes = self.ex.footprint(req.key, self.max_batch)
            if cached + slot_bytes > self.budget:
                raise ValueError(f"request {req.rid}: shape {req.key.n} needs {cached + slot_bytes} bytes, "
                                 f"more than the HBM budget {self.budget}")
        self.pending.setdefault(req.key, collections.deque()).append(req)

    def inflight(self):
        return sum(1 for sh in self.shapes.values() for s in sh["slots"] if s.busy)

    def idle(self):
        return not any(self.pending.values()) and self.inflight() == 0

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

    def _free_slot(self, key, now):
        """A free slot of `key`, admitting a new slot (and the shape's
        spectrum) if the budget allows; None if the request must wait."""
        sh = self.shapes.get(key)
        if sh is not None:
            for s in sh["slots"]:
                if not s.busy:
                    return s
            if len(sh["slots"]) >= self.max_slots:
                return None
            need = sh["slot_bytes"]
        else:
            cached, slot_bytes = self.ex.footprint(key, self.max_batch)
            need = cached + slot_bytes
        if not self._evict_for(need, key):
            return None
        if sh is None:
            cached, slot_bytes = self.ex.footprint(key, self.max_batch)
            self.ex.open_shape(key)
            sh = self.shapes[key] = dict(cached=cached, slot_bytes=slot_bytes, slots=[], last_used=now)
            self.used += cached
        slot = Slot(key=key, handle=self.ex.new_slot(key, self.max_batch))
        sh["slots"].append(slot)
        self.used += sh["slot_bytes"]
        return slot

    # ---- one scheduling round ------------------------------------------------
    def step(self, now):
        # completions
        for key, sh in self.shapes.items():
            for s in sh["slots"]:
                if s.busy and self.ex.poll(s.handle):
                    t_done = self.ex.finish(s.handle, s.requests)
                    for r in s.requests:
                        r.done = t_done if t_done is not None else now
                        self.completed.append(r)
                    s.busy = False
                    s.requests = []
        # admission and launches, oldest waiting request first
        order = sorted(((q[0].arrival, q[0].rid), k) for k, q in self.pending.items() if q)
        for _, key in order:
            q = self.pending[key]
            while q:
                slot = self._free_slot(key, now)
                if slot is None:
                    break
                batch = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
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

    # ---- drivers -------------------------------------------------------------
    def run(self, requests, clock, sleep=None, idle_wait=0.0):
        """Feed `requests` (sorted by arrival) as `clock()` passes their
        arrival times; returns when all are complete."""
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
            self.step(now)
            if sleep is not None:
                sleep(idle_wait)
        return self.stats()

    def stats(self):
        lat = np.array([r.latency for r in self.completed], dtype=np.float64)
        cells = sum(r.key.cells for r in self.completed)
        t0 = min((r.arrival for r in self.completed), default=0.0)
        t1 = max((r.done for r in self.completed), default=0.0)
        sizes = [b for _, b in self.batches]
        return {
            "requests": len(self.completed),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
            "mean_ms": float(lat.mean() * 1e3) if len(lat) else None,
            "cells_per_s": cells / (t1 - t0) if t1 > t0 else None,
            "makespan_s": t1 - t0,
            "batches": len(sizes),
            "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
            "max_inflight": self.max_inflight,
            "evictions": self.evictions,
            "hbm_used_bytes": self.used,
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

    def _desc(self, key, batch):
        return self.B.make_desc(key.n, key.d, key.mu, key.nu, key.lines, precision=key.precision, batch=batch,
                                near_shells=key.near_shells, periodic=key.periodic, pbc_shells=key.pbc_shells)

    def footprint(self, key, batch):
        cached, work, _ = self.B.footprint(self._desc(key, batch))
        nx, ny, nz = key.n
        elem = 4 if key.precision == 32 else 8
        staging = batch * (key.channels + 6) * nx * ny * nz * elem
        return cached, work + staging

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
            nb = len(requests)
            slot["plan"].stress_batch(slot["rho"][:nb], slot["out"][:nb], nb, stream=s)
            for i, r in enumerate(requests):
                r.result = slot["out"][i].clone()
            ev = torch.cuda.Event()
            ev.record(s)
        slot["event"] = ev

    def poll(self, slot):
        return slot["event"] is not None and slot["event"].query()

    def finish(self, slot, requests):
        slot["event"] = None
        return self.clock()

    def clock(self):
        return time.perf_counter() - self.t0


class SimExecutor:
    """Simulated executor for scheduler tests: a launch completes
    `latency(key, nb)` after it starts, on a virtual clock; payloads are
    echoed as results."""

    def __init__(self, footprints, latency, clock):
        self.fp = footprints          # key -> (cached, slot_bytes)
        self.lat = latency
        self.clock = clock
        self.opened = []
        self.closed = []
        self.live = 0
        self._ids = itertools.count()

    def footprint(self, key, batch):
        return self.fp[key]

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
