#!/usr/bin/env python3
"""Benchmark of the stress evaluation (one GPU).

A step is one full evaluation of the six stress components of every cell:
density hand-over (device-resident, borrowed) and the five passes of the
zero-padded FFT convolution with the plan's kernel spectrum. The plan (kernel
coefficients and their FP64 transform) is built once per geometry before the
timed region, as the method prescribes (Sec. 2.3).

Default workload: a 128 x 128 x 32 disk of mixed dislocations (t = e_z,
per-cell random in-plane angle, b = (cos phi, sin phi, 1)/sqrt 2), cells
dx = dy = 1, dz = 2, radial Gaussian density with 10 % noise; FP32 transforms
with an FP64 kernel precompute, compared with the plain FP64 path.

Prints one JSON line. ``--gpus`` above 1 is rejected: the benchmark runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid cells/s full σ_ij eval, FP32-batched vs FP64 plain at 1e-5 err; p50/p99"
HBM_PEAK_GBS = 8000.0


def make_workload(name, batch=1):
    """The named workload; for the disk workloads, `batch` realisations of the
    same recipe with consecutive noise seeds (realisation 0 is the base seed)."""
    import numpy as np
    from paper_1804_01830_amd import workloads as W
    if name == "disk-mixed-128":
        parts = [W.disk_mixed(seed=2 + i) for i in range(batch)]
        w = dict(parts[0])
        w["rho"] = np.concatenate([p["rho"] for p in parts], axis=0)
        return w
    if name == "disk-edge-32":
        return W.disk_edge()
    if name == "poly-256":
        return W.poly_layer()
    if name == "poly-pbc-256":          # periodic boundaries in the layer plane, 15 replica shells
        w = W.poly_layer(periodic=True)
        w["periodic"] = (True, True)
        return w
    if name == "sweep-64":
        return W.poly_sweep()
    if name == "poly-lines-256":        # per-grain line directions, axis-basis channels (C = 9), periodic
        w = W.poly_layer_lines()
        w["periodic"] = (True, True)
        return w
    raise SystemExit(f"unknown workload {name}")


def sweep_grain_law(w, plan, out):
    """Sec. 6.5 on the sweep: the in-plane standard deviation of sigma_xx
    (root of the Eq. 20 mean square over the interior half of the layers,
    averaged over the realisations of each grain size) against the grain
    size, for the height-dependent density of the workload and for the same
    grain maps with a height-independent density; log-log slopes."""
    import numpy as np
    import torch
    from paper_1804_01830_amd import binding as Bd
    from paper_1804_01830_amd import workloads as W
    grains = (4, 8, 16, 32)
    per = w["rho"].shape[0] // len(grains)
    nz = w["n"][2]
    lo, hi = nz // 4, nz - nz // 4

    def s_xx(rho_np):
        rho = torch.from_numpy(rho_np).to("cuda", dtype=torch.float32).contiguous()
        plan.set_density(rho)
        plan.stress(out)
        ms = Bd.plane_mean_square(out)[:, 0, lo:hi].mean(dim=1).sqrt().cpu().numpy()
        return [float(ms[g * per:(g + 1) * per].mean()) for g in range(len(grains))]

    hd = s_xx(w["rho"])
    flat = W.poly_sweep(*w["n"], z_decay=1e30)
    hom = s_xx(flat["rho"])
    slope = lambda v: float(np.polyfit(np.log(grains), np.log(v), 1)[0])
    return {"grain_sizes": list(grains), "realisations_per_size": per,
            "s_xx_height_dependent": [round(v, 5) for v in hd], "slope_height_dependent": round(slope(hd), 3),
            "s_xx_height_independent": [round(v, 5) for v in hom], "slope_height_independent": round(slope(hom), 3)}


def device_density(w, nb, dt):
    """The first nb densities on the device: the workload's channels, or for
    per-cell line fields the axis-basis channels built by the library
    (returns the tensor and the milliseconds of that conversion)."""
    import torch
    from paper_1804_01830_amd import binding as Bd
    if "density" not in w:
        return torch.from_numpy(w["rho"][:nb]).to("cuda", dtype=dt).contiguous(), None
    n, t, b = (torch.from_numpy(w[k][:nb]).to("cuda", dtype=dt).contiguous() for k in ("density", "t", "b"))
    rho = Bd.nye_density(n, t, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        Bd.nye_density(n, t, b, rho=rho)
    e1.record()
    torch.cuda.synchronize()
    return rho, e0.elapsed_time(e1) / 10


def z_pass_bytes(info, n, C, B, elem):
    """Algorithmic HBM bytes of one fused z launch: per (kx, ky) column it
    reads the C*B density columns (Nz complex values each) and writes 6*B
    stress columns (Nz complex each), (Px/2 + 1) * Py columns; the kernel
    spectrum is read once: 6*C reals for each stored (kx, ky, kz), where a
    mirror symmetry stores ky <= Py/2 (kz <= Pz/2) only."""
    Px, Py, Pz = info.padded
    Nz = n[2]
    M1 = Px // 2 + 1
    cols = M1 * Py
    nky = Py // 2 + 1 if info.mirror_y else Py
    nkz = Pz // 2 + 1 if info.mirror_z else Pz
    return elem * (cols * (2 * C * B * Nz + 2 * 6 * B * Nz) + 6 * C * M1 * nky * nkz)


def path_bytes(info, n, C, B, elem):
    """Algorithmic HBM bytes of the whole path for one call: five passes, or
    fewer where the plan fuses the x and y passes (the intermediate plane then
    stays in LDS and is not counted)."""
    Px, Py, Pz = info.padded
    Nx, Ny, Nz = n
    M1 = Px // 2 + 1
    cx = 2 * M1                       # reals per complex x-spectrum row
    if info.xy_fused:                 # density reals in, y spectra out
        fwd = elem * B * C * Nz * (Ny * Nx + M1 * 2 * Py)
    else:
        fwd = elem * B * C * Nz * Ny * (Nx + cx) + elem * B * C * Nz * M1 * 2 * (Ny + Py)
    z = z_pass_bytes(info, n, C, B, elem)
    if info.yx_fused:                 # z output in, stress reals out
        inv = elem * B * 6 * Nz * (M1 * 2 * Py + Ny * Nx)
    else:
        inv = elem * B * 6 * Nz * M1 * 2 * (Py + Ny) + elem * B * 6 * Nz * Ny * (cx + Nx)
    return fwd + z + inv


def b_pass_bytes(C, B, elem):
    """Bytes per cell of the plain five-pass model, s (13 C + 24 C / B + 78):
    forward passes, the kernel spectrum read once per batch, inverse passes.
    value x b_pass_bytes / 8 TB/s is the fraction of the HBM roofline that
    model allows (fused planes move fewer bytes than it counts)."""
    return elem * (13 * C + 24 * C / B + 78)


def five_pass_z_bytes(C, B, cells, elem):
    """Algorithmic HBM bytes of one fused z launch by the five-pass model:
    per cell and realisation it reads the C density columns (4C reals: the
    half spectrum of the padded x-y plane holds about 2N complex values per
    channel) and writes the six stress columns (24 reals), and the kernel
    spectrum, 6C reals at every one of the ~4N non-redundant wavevectors, is
    read once per launch: s (4C + 24C/B + 24) per cell, over B cells per
    grid cell. The mirror-compressed spectrum the plans store is smaller;
    z_pass_bytes counts that."""
    return elem * (4 * C + 24 * C / B + 24) * B * cells


def time_steps(plan, rho, out, steps, warmup, graph=False):
    """The headline timing: `warmup` untimed steps, then exactly `steps`
    steps (density hand-over and stress call) between two synchronisations
    (wall clock) and two events on the stream (device time). No per-pass or
    per-step events are recorded inside."""
    import torch
    from paper_1804_01830_amd import binding as Bd
    stream = torch.cuda.current_stream()
    plan.set_graph(graph)
    for _ in range(warmup):
        plan.set_density(rho, Bd.DEVICE_BORROW)
        plan.stress(out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.set_density(rho, Bd.DEVICE_BORROW)
        plan.stress(out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.set_graph(False)
    return wall, e0.elapsed_time(e1)


def time_latency(plan, rho, out, reps, graph=False):
    """Device time of `reps` single evaluations, each between its own pair
    of events (p50 / p99 of one evaluation); sorted milliseconds."""
    import torch
    from paper_1804_01830_amd import binding as Bd
    stream = torch.cuda.current_stream()
    plan.set_graph(graph)
    plan.set_density(rho, Bd.DEVICE_BORROW)
    plan.stress(out)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    torch.cuda.synchronize()
    for i in range(reps):
        starts[i].record(stream)
        plan.set_density(rho, Bd.DEVICE_BORROW)
        plan.stress(out)
        ends[i].record(stream)
    torch.cuda.synchronize()
    plan.set_graph(False)
    return sorted(a.elapsed_time(b) for a, b in zip(starts, ends))


def time_host_io(plan, rho, steps, warmup):
    """Host-to-host steps: density from pinned host memory, stress back to
    pinned host memory (PCIe both ways), one synchronisation per step."""
    import torch
    from paper_1804_01830_amd import binding as Bd
    rho_h = rho.cpu().pin_memory()
    out_h = torch.empty(tuple(plan.new_output().shape), dtype=rho.dtype).pin_memory()
    for _ in range(warmup):
        plan.set_density(rho_h, Bd.HOST)
        plan.stress(out_h, where=Bd.HOST)
    torch.cuda.synchronize()
    per = []
    for _ in range(steps):
        t = time.perf_counter()
        plan.set_density(rho_h, Bd.HOST)
        plan.stress(out_h, where=Bd.HOST)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - t)
    per.sort()
    return sum(per), per, rho_h.numel() * rho_h.element_size() + out_h.numel() * out_h.element_size()


def pct(sorted_vals, q):
    k = min(len(sorted_vals) - 1, max(0, int(round(q / 100.0 * (len(sorted_vals) - 1)))))
    return sorted_vals[k]


def _oracle_targets(args):
    rho, d, lines, mu, nu, tg = args
    from oracle import stress_direct
    return stress_direct(rho, d, lines, mu, nu, targets=tg)


def rel_l2_targets(got, ref):
    """Relative L2 error per Voigt component over the sampled cells (a
    component with a negligible reference norm is measured against the whole
    norm) and over the whole tensor."""
    import numpy as np
    whole = np.linalg.norm(ref)
    comp = [np.linalg.norm(got[v] - ref[v]) / max(np.linalg.norm(ref[v]), 1e-3 * whole) for v in range(6)]
    return comp, np.linalg.norm(got - ref) / whole


def cpu_baseline(w, seconds):
    """Time the FP64 oracle (direct sum over all cells) on a bounded sample of
    target cells on the host cores. Runs before the GPU is touched (the worker
    pool forks). Returns the baseline record, the targets and their values."""
    import multiprocessing as mp
    import numpy as np
    nx, ny, nz = w["n"]
    rng = np.random.default_rng(12345)
    cores = max(1, min(16, os.cpu_count() or 1))
    # calibrate: one target on one core
    tg0 = np.array([[nx // 2, ny // 2, nz // 2]])
    t = time.perf_counter()
    _oracle_targets((w["rho"][0], w["d"], w["lines"], w["mu"], w["nu"], tg0))
    one = time.perf_counter() - t
    n_tg = int(max(cores, min(512, seconds * cores / max(one, 1e-3))))
    n_tg = max(cores, (n_tg // cores) * cores)
    tg = np.stack([rng.integers(0, nx, n_tg), rng.integers(0, ny, n_tg), rng.integers(0, nz, n_tg)], axis=1)
    chunks = np.array_split(tg, cores)
    ctx = mp.get_context("fork")
    t = time.perf_counter()
    with ctx.Pool(cores) as pool:
        parts = pool.map(_oracle_targets, [(w["rho"][0], w["d"], w["lines"], w["mu"], w["nu"], c) for c in chunks])
    el = time.perf_counter() - t
    ref = np.concatenate(parts, axis=1)
    base = {"value": round(n_tg / el, 3), "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_tg} random target cells of the {nx}x{ny}x{nz} grid, each a full FP64 direct sum "
                      f"over all {nx * ny * nz} source cells (Eq. 10), {cores} worker processes, {el:.1f} s"}
    return base, tg, ref


def cpu_baseline_periodic(w, seconds, shells=15):
    """The periodic oracle (replica-shell kernel, Eq. 13, and the direct sum of
    Eq. 12) timed on a bounded sample: a few target cells, each summed over a
    random subset of source cells with the workload's channels (all other
    cells zeroed), on one host core; scaled to full sums over every source
    cell. Returns the baseline record."""
    import numpy as np
    from oracle.periodic import stress_direct_periodic
    nx, ny, nz = w["n"]
    cells = nx * ny * nz
    rng = np.random.default_rng(2024)
    if "density" in w:
        from oracle.nye import nye_channels
        full = None
    else:
        full = w["rho"][0]
    tg = np.stack([rng.integers(0, nx, 2), rng.integers(0, ny, 2), rng.integers(0, nz, 2)], axis=1)

    def run(ns):
        flat = rng.choice(cells, size=ns, replace=False)
        k, j, i = np.unravel_index(flat, (nz, ny, nx))
        if full is None:
            ch = nye_channels(w["density"][0][k, j, i], w["t"][0][:, k, j, i], w["b"][0][:, k, j, i])
            C = 9
        else:
            ch = full[:, k, j, i]
            C = full.shape[0]
        rho = np.zeros((C, nz, ny, nx))
        rho[:, k, j, i] = ch
        t0 = time.perf_counter()
        stress_direct_periodic(rho, w["d"], w["lines"], w["mu"], w["nu"], periodic=(True, True), shells=shells,
                               targets=tg)
        return time.perf_counter() - t0

    # the oracle's cost is a fixed part per call (one numpy pass per replica) plus a part per source cell;
    # two small runs give both, a third run of about `seconds` measures the per-source part
    t1, t2 = run(64), run(512)
    per_src = max((t2 - t1) / 448.0, 1e-9)
    fixed = max(t1 - 64 * per_src, 0.0)
    ns = int(max(512, min(cells, (seconds - fixed) / per_src)))
    el = run(ns)
    per_src = max((el - fixed) / ns, 1e-12)
    per_target = (fixed + per_src * cells) / len(tg)
    return {"value": float(f"{1.0 / per_target:.4g}"), "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(tg)} target cells, each summed over {ns} random source cells of the {nx}x{ny}x{nz} "
                      f"grid with {shells} replica shells (Eq. 12-13), {el:.1f} s on one core; the per-source cost "
                      f"(after the fixed per-call part, fitted from runs over 64 and 512 sources) scaled to full "
                      f"sums over all {cells} source cells"}


def cpu_baseline_relax(n, d, mu, nu, seconds):
    """The relaxation oracle (explicit steps of Eq. 17) timed on the host for
    the full node grid on a synthetic load of the same shape; node-steps/s."""
    from oracle.relax import relax
    from paper_1804_01830_amd import workloads as W
    load = W.random_stress(n, seed=77, d=d, mu=mu, nu=nu, smooth=True)["sigma"]
    t0 = time.perf_counter()
    relax(load, d, mu, nu, 1)
    one = time.perf_counter() - t0
    steps = int(max(1, min(50, seconds / max(one, 1e-3))))
    t0 = time.perf_counter()
    relax(load, d, mu, nu, steps)
    el = time.perf_counter() - t0
    nodes = n[0] * n[1] * n[2]
    return {"value": round(nodes * steps / el, 1), "unit": "node-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} explicit steps (and their set-up) of the {n[0]}x{n[1]}x{n[2]} node grid on a "
                      f"synthetic smooth load, {el:.1f} s on one core"}


def errors_at(tg, ref, gpu32, gpu64):
    sel32 = gpu32[:, tg[:, 2], tg[:, 1], tg[:, 0]]
    sel64 = gpu64[:, tg[:, 2], tg[:, 1], tg[:, 0]]
    e32, w32 = rel_l2_targets(sel32, ref)
    e64, w64 = rel_l2_targets(sel64, ref)
    return {"fp32_rel_l2_per_component": [float("%.3e" % x) for x in e32], "fp32_rel_l2": float("%.3e" % w32),
            "fp64_rel_l2_per_component": [float("%.3e" % x) for x in e64], "fp64_rel_l2": float("%.3e" % w64),
            "targets": int(len(tg))}


SERVE_SHAPES = ((64, 64, 64), (128, 128, 32), (256, 256, 64), (256, 256, 128))


def serve_bench(args):
    """Serving stream: Poisson arrivals of stress requests on grids drawn from
    SERVE_SHAPES with polycrystal densities (grain size 16 cells), admitted by
    HBM footprint, batched per shape; reports p50/p99 latency and cells/s at
    the saturated rate and at a fraction of it."""
    import numpy as np
    import torch
    from paper_1804_01830_amd import workloads as W
    from paper_1804_01830_amd.serving import GpuExecutor, Request, Server, ShapeKey, poisson_arrivals
    torch.cuda.set_device(0)
    pools, keys = [], []
    for n in SERVE_SHAPES:
        w = W.poly_layer(*n, batch_seeds=list(range(args.serve_pool)))
        keys.append(ShapeKey(n=tuple(n), d=tuple(w["d"]), mu=w["mu"], nu=w["nu"],
                             lines=tuple(tuple(map(float, t)) for t in w["lines"]), precision=32))
        pools.append(torch.from_numpy(w["rho"]).to("cuda", dtype=torch.float32))
        print(f"[serve] pool {n}: {args.serve_pool} densities", file=sys.stderr, flush=True)
    ex = GpuExecutor(use_graph=True, tune=not args.no_tune)
    srv = Server(ex, hbm_budget=int(args.serve_budget_gb * (1 << 30)), max_batch=args.serve_batch,
                 max_slots_per_shape=2)
    rng = np.random.default_rng(5)

    def make(count, rate):
        arr = np.zeros(count) if rate is None else poisson_arrivals(rate, count, seed=5)
        t0 = ex.clock()
        out = []
        for i, t in enumerate(arr):
            s = int(rng.integers(len(keys)))
            out.append(Request(i, keys[s], rho=pools[s][int(rng.integers(args.serve_pool))], arrival=t0 + float(t)))
        return out

    def consume(server, r):        # the benchmark drops each result once it is complete
        server.release(r)

    # warm-up: one request per shape builds the plans (and tunings)
    srv.run([Request(i, k, rho=pools[i][0], arrival=ex.clock()) for i, k in enumerate(keys)], ex.clock,
            on_complete=consume)
    torch.cuda.synchronize()
    results = {}
    srv.completed, srv.batches = [], []
    sat = srv.run(make(args.serve_requests, None), ex.clock, on_complete=consume)
    torch.cuda.synchronize()
    results["saturated"] = sat
    rate_sat = sat["requests"] / sat["makespan_s"]
    for frac in (0.5, 0.9):
        srv.completed, srv.batches = [], []
        st = srv.run(make(args.serve_requests, frac * rate_sat), ex.clock, on_complete=consume)
        torch.cuda.synchronize()
        st["offered_rate_per_s"] = frac * rate_sat
        results[f"{frac:.2f}x"] = st
    line = {"metric": "served stress requests: p50/p99 latency (device events, arrival to completion) and cells/s",
            "unit": "cells/s",
            "value": round(sat["cells_per_s"], 1), "higher_is_better": True, "n_gpus": 1, "dtype": "f32",
            "data": "synthetic (seeded)",
            "config": {"workload": "serve-poly-mix", "shapes": [list(n) for n in SERVE_SHAPES],
                       "max_batch": args.serve_batch, "hbm_budget_gb": args.serve_budget_gb,
                       "requests_per_run": args.serve_requests},
            "runs": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                     for k, v in results.items()}}
    print(json.dumps(line), flush=True)


def relax_step_bytes(n, elem):
    """Algorithmic HBM bytes of one explicit relaxation step: every node reads
    its three displacement components and three force components and writes
    three displacement components (neighbours come from caches); the two
    ghost layers add 3 * 2 * Nx * Ny writes and their reads."""
    nx, ny, nz = n
    return elem * (9 * nx * ny * nz + 2 * 3 * 2 * nx * ny)


def relax_bench(args):
    """Free-surface relaxation (Sec. 5) of the periodic layer's dislocation
    stress: the stress plan evaluates sigma^dis once, then K explicit steps
    are timed; also the steps needed to bring the update norm below 1e-6 of
    its first value on the same load."""
    import numpy as np
    import torch
    from paper_1804_01830_amd import binding as Bd
    w = make_workload("poly-pbc-256")
    nx, ny, nz = w["n"]
    nodes = nx * ny * nz
    base = None
    if not args.no_cpu_baseline:
        base = cpu_baseline_relax(w["n"], w["d"], w["mu"], w["nu"], args.cpu_seconds)
        print(f"[relax] cpu baseline: {base['sample']}", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    res = {}
    for prec in (32, 64):
        dt = torch.float32 if prec == 32 else torch.float64
        desc = Bd.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=prec, periodic=(True, True))
        plan = Bd.Plan(desc)
        rho = torch.from_numpy(w["rho"]).to("cuda", dtype=dt).contiguous()
        plan.set_density(rho)
        sig = plan.new_output()
        plan.stress(sig)
        sig = sig[0].contiguous()
        torch.cuda.synchronize()
        plan.close()
        r = Bd.Relax(w["n"], w["d"], w["mu"], w["nu"], precision=prec)
        r.set_load(sig)
        r.iterate(args.warmup)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        steps = args.relax_steps
        t0.record(stream)
        r.iterate(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        # convergence on the same load, from u = 0
        r.set_load(sig)
        first = r.update_norm()
        conv, taken = None, 0
        while taken < args.relax_max_steps:
            r.iterate(1000)
            taken += 1000
            nrm = r.update_norm()
            if nrm <= 1e-6 * first:
                conv = taken
                break
        info = r.info()
        r.close()
        res[prec] = dict(ms=ms, steps=steps, dt=info.dt, first=first, last=nrm, conv=conv, taken=taken)
        print(f"[relax] precision {prec}: {ms / steps * 1e3:.2f} us/step, update norm {first:.3e} -> {nrm:.3e} "
              f"after {taken} steps", file=sys.stderr, flush=True)
    r32, r64 = res[32], res[64]
    per32 = r32["ms"] / r32["steps"] * 1e-3
    per64 = r64["ms"] / r64["steps"] * 1e-3
    b32 = relax_step_bytes(w["n"], 4)
    line = {
        "metric": "free-surface relaxation: node-steps/s (explicit Navier-Cauchy steps, Eq. 17)",
        "value": round(nodes / per32, 1), "unit": "node-steps/s", "n_gpus": 1, "steps": r32["steps"],
        "warmup": args.warmup, "ms_per_step": round(per32 * 1e3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded)",
        "config": {"workload": "relax-" + w["name"], "grid": [nx, ny, nz], "cell": list(w["d"]), "nu": w["nu"],
                   "load": "dislocation stress of the periodic layer (stress plan, 15 shells)",
                   "boundary": "periodic x, y; traction-free top and bottom"},
        "fp64": {"value": round(nodes / per64, 1), "ms_per_step": round(per64 * 1e3, 5)},
        "roofline": {"bound": "hbm", "achieved": round(b32 / per32 / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(b32 / per32 / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_relax_march + k_relax_ghost (one step; events around K steps)",
                     "algorithmic_bytes_per_launch": int(b32)},
        "convergence": {str(p): {"dt": res[p]["dt"], "update_norm_first": res[p]["first"],
                                 "update_norm_last": res[p]["last"], "steps_to_1e-6": res[p]["conv"],
                                 "steps_run": res[p]["taken"]} for p in (32, 64)},
    }
    if base is not None:
        line["cpu_baseline"] = base
    from paper_1804_01830_amd import profiling as Pf
    tr = Pf.stored_traffic(os.path.join(ROOT, "profiles"), line["config"]["workload"], 1, "k_relax_march",
                           sources=Pf.RELAX_SOURCES)
    if tr is not None:
        line["roofline"]["traffic"] = int(tr)
        line["roofline"]["traffic_vs_algorithmic"] = round(tr / b32, 3)
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calib_copy_bytes"] = 4 * n
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="disk-mixed-128")
    ap.add_argument("--batch", type=int, default=8,
                    help="realisations per FP32 call for the disk-mixed workload (the FP64 plain path "
                         "always evaluates the single base grid)")
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--latency-reps", type=int, default=200,
                    help="single evaluations with an event pair each, for p50 / p99 (at least --steps)")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="skip the 256x256x64 layer and the 64-realisation sweep after the default workload")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="default launch shapes for the FP32 plan")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a device buffer of this many MiB once (a plain copy kernel of "
                         "known size, for scaling hardware traffic counters)")
    ap.add_argument("--serve", action="store_true", help="run the serving benchmark instead")
    ap.add_argument("--relax", action="store_true",
                    help="run the free-surface relaxation benchmark on the periodic layer instead")
    ap.add_argument("--relax-steps", type=int, default=2000)
    ap.add_argument("--relax-max-steps", type=int, default=100000)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-pool", type=int, default=4)
    ap.add_argument("--serve-batch", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the stress evaluation of one grid (or one batch of grids) "
              "is not sharded across GPUs; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    if args.relax:
        relax_bench(args)
        return

    w = make_workload(args.workload, args.batch)
    if "density" in w:
        import numpy as np
        from paper_1804_01830_amd.binding import AXIS_LINES
        w["lines"] = np.array(AXIS_LINES)
        B, C = w["density"].shape[0], 9
    else:
        B, C = w["rho"].shape[0], w["rho"].shape[1]
    nx, ny, nz = w["n"]
    cells = B * nx * ny * nz
    plain_one = args.workload == "disk-mixed-128"     # FP64 plain: the single base grid
    print(f"[bench] workload {w['name']} B={B} C={C} cells={cells}", file=sys.stderr, flush=True)
    base = None
    periodic = tuple(w.get("periodic", (False, False)))
    if any(periodic) and not args.no_cpu_baseline:
        # the oracle's periodic sum costs (2 n_sh + 1)^2 open sums per target: a sampled, scaled timing
        base = cpu_baseline_periodic(w, args.cpu_seconds)
        print(f"[bench] cpu baseline: {base['sample']}", file=sys.stderr, flush=True)
    elif not args.no_cpu_baseline and (B == 1 or plain_one):
        base, tg, ref = cpu_baseline(w, args.cpu_seconds)
        print(f"[bench] cpu baseline: {base['sample']}", file=sys.stderr, flush=True)

    import torch
    torch.cuda.set_device(0)
    extras = args.workload == "disk-mixed-128"
    keep = (0,) if (B == 1 or plain_one) else ()
    r32 = measure(w, 32, B, args, periodic, tune=not args.no_tune, graph=True, host_io=extras, stats=extras,
                  keep_out=keep, grain_law=args.workload == "sweep-64")
    r64 = measure(w, 64, 1 if plain_one else B, args, periodic, tune=False, keep_out=keep)
    line = {
        "metric": METRIC, "value": round(r32["value"], 1), "unit": "cells/s", "n_gpus": 1,
        "steps": r32["steps"], "warmup": args.warmup, "ms_per_step": round(r32["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded)",
        "config": {"workload": w["name"], "grid": list(w["n"]), "cell": list(w["d"]), "channels": C,
                   "batch": B, "cells_per_step": cells, "precision": "fp32 transforms and contraction, "
                   "fp64 kernel coefficients and transform", "parallelism": "single GPU",
                   "boundary": "periodic in x and y, 15 replica shells" if any(periodic) else "open"},
    }
    line.update(summary(r32, r64, w, C, B, periodic))
    if r32.get("grain_law") is not None:
        line["grain_law"] = r32["grain_law"]
    if r32.get("nye_ms") is not None:
        line["axis_basis_channels"] = {
            "what": "rho[3l+g] = n t_l b_g from per-cell line fields (ddstress_nye_density), outside the step",
            "ms": round(r32["nye_ms"], 5),
            "gbs": round(B * (7 + 9) * nx * ny * nz * 4 / (r32["nye_ms"] * 1e-3) / 1e9, 1)}
    if base is not None:
        line["cpu_baseline"] = base
        if not any(periodic):
            line["error_vs_oracle"] = errors_at(tg, ref, r32["out"][0], r64["out"][0])
    r32.clear()
    r64.clear()
    if extras and not args.no_extra_configs:
        line["configs"] = {}
        for name in ("poly-256", "sweep-64"):
            line["configs"][name] = sub_config(name, args)
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calib_copy_bytes"] = 4 * n
    print(json.dumps(line), flush=True)


def measure(w, prec, Bp, args, periodic, tune, graph=False, host_io=False, stats=False, keep_out=(),
            grain_law=False):
    """Plan (tuned in FP32), then: the headline loop (exactly args.steps steps,
    no events inside), the latency loop (max(200, steps) single evaluations
    with an event pair each), each pass timed alone (ddstress_plan_time_passes),
    and on request graph replay, host-to-host steps and the plane statistics."""
    import torch
    from paper_1804_01830_amd import binding as Bd
    from paper_1804_01830_amd import tuning as Tn
    nx, ny, nz = w["n"]
    desc = Bd.make_desc(w["n"], w["d"], w["mu"], w["nu"], w["lines"], precision=prec, batch=Bp, periodic=periodic)
    t = time.perf_counter()
    tuning = Tn.get_tuning(desc) if tune else None
    plan = Bd.Plan(desc, tuning=tuning)
    plan_s = time.perf_counter() - t
    dt = torch.float32 if prec == 32 else torch.float64
    rho, nye_ms = device_density(w, Bp, dt)
    out = plan.new_output()
    steps = args.steps if prec == 32 else (args.fp64_steps or args.steps)
    # the latency loop first: the headline's steps then run on a device that
    # has been busy for a while (its clocks settled), as in steady use
    lat = time_latency(plan, rho, out, max(args.latency_reps, steps))
    wall, dev_ms = time_steps(plan, rho, out, steps, args.warmup)
    plan.set_density(rho, Bd.DEVICE_BORROW)
    passes = plan.time_passes(out, max(20, min(steps, 100)))
    r = dict(info=plan.info(), steps=steps, ms_per_step=wall / steps * 1e3, device_ms_per_step=dev_ms / steps,
             lat=lat, passes=passes, plan_s=plan_s, nye_ms=nye_ms, cells=Bp * nx * ny * nz,
             tune=Tn.to_dict(tuning) if tuning is not None else None)
    r["value"] = r["cells"] / (r["ms_per_step"] * 1e-3)
    if graph:
        gw, gdev = time_steps(plan, rho, out, steps, args.warmup, graph=True)
        r["graph"] = dict(ms=gw / steps * 1e3, dev_ms=gdev / steps,
                          lat=time_latency(plan, rho, out, max(args.latency_reps, steps), graph=True))
    if host_io:
        hw, hper, hbytes = time_host_io(plan, rho, min(steps, 50), min(args.warmup, 5))
        r["host"] = dict(wall=hw, per=hper, bytes=hbytes, steps=min(steps, 50))
    if stats:
        # Eq. (20) plane statistics of the stress just computed (one read of sigma)
        stream = torch.cuda.current_stream()
        ms_out = Bd.plane_mean_square(out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            Bd.plane_mean_square(out, ms_out)
        e1.record(stream)
        torch.cuda.synchronize()
        r["stats_ms"] = e0.elapsed_time(e1) / 20
        # the same statistics fused into the stress call (inverse x epilogue),
        # against the same loop without them
        k = min(steps, 100)
        pw, _ = time_steps(plan, rho, out, k, min(args.warmup, 10))
        plan.set_plane_stats(ms_out)
        fw, _ = time_steps(plan, rho, out, k, min(args.warmup, 10))
        plan.set_plane_stats(None)
        r["fused_ms"], r["plain_ms"] = fw / k * 1e3, pw / k * 1e3
    if grain_law:
        r["grain_law"] = sweep_grain_law(w, plan, out)
    if keep_out:          # the stress of these realisations, for the error against the oracle
        plan.set_density(rho, Bd.DEVICE_BORROW)
        plan.stress(out)
        torch.cuda.synchronize()
        r["out"] = {i: out[i].double().cpu().numpy() for i in keep_out}
    plan.close()
    del rho, out
    torch.cuda.empty_cache()
    print(f"[bench] {w['name']} precision {prec} B={Bp}: {r['ms_per_step']:.4f} ms/step "
          f"(device {r['device_ms_per_step']:.4f}), p50 {pct(lat, 50):.4f} p99 {pct(lat, 99):.4f} ms, plan "
          f"{plan_s:.2f} s, passes(ms/launch) " + ", ".join(f"{k}={v:.4f}" for k, v in passes.items()),
          file=sys.stderr, flush=True)
    return r


def summary(r32, r64, w, C, B, periodic):
    """The fields of a bench line (or sub-object) from the FP32 and FP64 runs."""
    info = r32["info"]
    elem = 4
    nx, ny, nz = w["n"]
    cells = B * nx * ny * nz
    z_ms = r32["passes"]["z_fused"]
    wave = info.z_groups == 1 and info.ez == 8 and info.padded[2] == 64 and info.precision == 32
    kname = "k_z_grouped" if info.z_groups > 1 else ("k_z_wave" if wave else "k_z_serial")
    zmir = z_pass_bytes(info, w["n"], C, B, elem)
    from paper_1804_01830_amd import profiling as Pf
    traffic = Pf.stored_traffic(os.path.join(ROOT, "profiles"), w["name"], B, kname)
    if any(periodic):
        # the five-pass model assumes padded x and y: the periodic plans transform Nx x Ny planes
        zalg, basis = zmir, "algorithmic bytes of the transforms the plan runs (mirror-compressed spectrum)"
    else:
        zalg = five_pass_z_bytes(C, B, nx * ny * nz, elem)
        basis = "five-pass model: s (4C + 24C/B + 24) per cell (full spectrum read once per launch)"
    achieved = zalg / (z_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(traffic),
                "traffic_vs_algorithmic": None if traffic is None else round(traffic / zalg, 3),
                "kernel": kname, "kernel_does": "forward z FFT, 6 x C contraction with the kernel spectrum, "
                                                "inverse z FFT (fused)",
                "algorithmic_bytes_per_launch": int(zalg), "algorithmic_basis": basis,
                "mirror_aware_bytes_per_launch": int(zmir),
                "mirror_aware_frac": round(zmir / (z_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "avg_launch_ms": round(z_ms, 5),
                "avg_launch_timing": "ddstress_plan_time_passes: launches back to back between two HIP events "
                                     "on the library's stream"}
    ms32 = r32["ms_per_step"]
    pbytes = path_bytes(info, w["n"], C, B, elem)
    out = {
        "p50_ms": round(pct(r32["lat"], 50), 5), "p99_ms": round(pct(r32["lat"], 99), 5),
        "latency_reps": len(r32["lat"]),
        "device_ms_per_step": round(r32["device_ms_per_step"], 5),
        "fp64_plain": {"value": round(r64["value"], 1), "ms_per_step": round(r64["ms_per_step"], 5),
                       "steps": r64["steps"], "batch": r64["info"].batch,
                       "p50_ms": round(pct(r64["lat"], 50), 5), "p99_ms": round(pct(r64["lat"], 99), 5),
                       "pass_ms": {k: round(v, 5) for k, v in r64["passes"].items()}},
        "speedup_fp32_vs_fp64": round(r32["value"] / r64["value"], 3),
        "tuning": r32["tune"],
        "pass_ms": {k: round(v, 5) for k, v in r32["passes"].items()},
        "path_algorithmic_gbs": round(pbytes / (ms32 * 1e-3) / 1e9, 1),
        "path_frac": round(pbytes / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "plan_build_s": {"fp32": round(r32["plan_s"], 3), "fp64": round(r64["plan_s"], 3)},
        "roofline": roofline,
        "plan_info": {"padded": list(info.padded), "tile_z": info.tile_z, "ez": info.ez,
                      "z_groups": info.z_groups, "mirror_y": info.mirror_y, "mirror_z": info.mirror_z,
                      "xy_fused": info.xy_fused, "yx_fused": info.yx_fused,
                      "rows_x": info.rows_x, "tile_y": info.tile_y, "ex": info.ex, "ey": info.ey},
    }
    if not any(periodic):
        out["b_pass_frac"] = round(r32["value"] * b_pass_bytes(C, B, elem) / (HBM_PEAK_GBS * 1e9), 4)
    if "graph" in r32:
        g = r32["graph"]
        out["graph_replay"] = {"value": round(cells / (g["ms"] * 1e-3), 1), "ms_per_step": round(g["ms"], 5),
                               "p50_ms": round(pct(g["lat"], 50), 5), "p99_ms": round(pct(g["lat"], 99), 5)}
    if "host" in r32:
        h = r32["host"]
        out["host_to_host"] = {"value": round(cells / (h["wall"] / h["steps"]), 1),
                               "ms_per_step": round(h["wall"] / h["steps"] * 1e3, 5),
                               "p50_ms": round(pct(h["per"], 50) * 1e3, 5),
                               "pcie_bytes_per_step": h["bytes"],
                               "note": "density from and stress to pinned host memory; not the headline value"}
    if "stats_ms" in r32:
        out["plane_stats"] = {"what": "Eq. 20 mean square per plane of the FP32 stress (ddstress_plane_mean_square)",
                              "ms": round(r32["stats_ms"], 5),
                              "gbs": round(B * 6 * nx * ny * nz * 4 / (r32["stats_ms"] * 1e-3) / 1e9, 1),
                              "fused_ms_per_step": round(r32["fused_ms"], 5),
                              "plain_ms_per_step": round(r32["plain_ms"], 5),
                              "fused_note": "stress call with the statistics in the inverse x pass "
                                            "(ddstress_plan_set_plane_stats), and the same loop without them"}
    return out


GOLDEN = {"poly-256": ("poly_layer_256x256x64",), "sweep-64": ("poly_sweep_128x128x32_b0", "poly_sweep_128x128x32_b63")}


def sub_config(name, args):
    """One more workload timed like the headline (FP32 batched and tuned, FP64
    plain with one realisation), with its error on the stored oracle values of
    tests/golden (written by the oracle alone)."""
    import numpy as np
    w = make_workload(name)
    B, C = w["rho"].shape[0], w["rho"].shape[1]
    nx, ny, nz = w["n"]
    print(f"[bench] sub-config {w['name']} B={B} C={C}", file=sys.stderr, flush=True)
    goldens = []
    for gname in GOLDEN[name]:
        with open(os.path.join(ROOT, "tests", "golden", gname + ".json")) as f:
            goldens.append(json.load(f))
    r32 = measure(w, 32, B, args, (False, False), tune=not args.no_tune,
                  keep_out=tuple(g["batch_index"] for g in goldens))
    r64 = measure(w, 64, 1, args, (False, False), tune=False, keep_out=(0,))
    sub = {"workload": w["name"], "value": round(r32["value"], 1), "unit": "cells/s",
           "ms_per_step": round(r32["ms_per_step"], 5), "steps": r32["steps"], "batch": B, "channels": C,
           "grid": list(w["n"]), "cells_per_step": B * nx * ny * nz}
    sub.update(summary(r32, r64, w, C, B, (False, False)))
    errs = {}
    for gname, g in zip(GOLDEN[name], goldens):
        tg = np.array(g["targets"])
        ref = np.array(g["sigma_voigt"]).T
        bi = g["batch_index"]
        e32, w32 = rel_l2_targets(r32["out"][bi][:, tg[:, 2], tg[:, 1], tg[:, 0]], ref)
        rec = {"realisation": bi, "targets": len(tg), "fp32_rel_l2_per_component": [float("%.3e" % x) for x in e32],
               "fp32_rel_l2": float("%.3e" % w32)}
        if bi == 0:
            e64, w64 = rel_l2_targets(r64["out"][0][:, tg[:, 2], tg[:, 1], tg[:, 0]], ref)
            rec.update({"fp64_rel_l2_per_component": [float("%.3e" % x) for x in e64], "fp64_rel_l2": float("%.3e" % w64)})
        errs[gname] = rec
    sub["error_vs_oracle"] = {"oracle": "stored FP64 direct-sum values (tests/golden, written by the oracle only)",
                              "fixtures": errs}
    return sub


if __name__ == "__main__":
    main()
