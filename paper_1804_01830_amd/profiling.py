"""Summaries of rocprofv3 output for the fused z pass and the whole path.

Two reports, each a short markdown file that records the command it came from:

* ``trace``: the kernel statistics of ``rocprofv3 --kernel-trace --stats
  --output-format csv`` (calls, total and average duration per kernel).
* ``traffic``: HBM bytes per launch of the fused z kernel from two counter
  runs, ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, of a ``bench.py``
  command with ``--calib-copy-mib M``. The counters are scaled by what they
  read for that plain device copy of M MiB (M MiB read, M MiB written), and
  only the launches with the block and grid of the benchmarked plan are used
  (an autotuning run launches other shapes too). The report carries a digest
  of the device sources; ``bench.py`` reports the traffic only while the
  digest matches the sources it runs.

Usage::

    python -m paper_1804_01830_amd.profiling trace <dir> <title> <command> > report.md
    python -m paper_1804_01830_amd.profiling traffic <fetch_dir> <write_dir> <bench_json_line_file> \\
        <copy_mib> <title> <command> > report.md
    python -m paper_1804_01830_amd.profiling relax-traffic <fetch_dir> <write_dir> <bench_json_line_file> \\
        <copy_mib> <title> <command> > report.md
    python -m paper_1804_01830_amd.profiling kernels <fetch_dir> <write_dir> <copy_mib> <title> <command> > report.md
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEVICE_SOURCES = ("csrc/passes.hip", "csrc/zfused.hpp", "csrc/z_serial_f32.hip", "csrc/z_serial_f64.hip",
                  "csrc/z_grouped_f32.hip", "csrc/z_grouped_f64.hip", "csrc/fft_device.hpp",
                  "csrc/ddstress_internal.hpp")
RELAX_SOURCES = ("csrc/relax.hip", "csrc/fft_device.hpp", "csrc/ddstress_internal.hpp")


def source_digest(sources=DEVICE_SOURCES):
    """sha256 over device sources (default: those of the five passes)."""
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _csv(directory, suffix):
    paths = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not paths:
        raise SystemExit(f"no *{suffix} under {directory}")
    with open(paths[0], newline="") as f:
        return list(csv.DictReader(f))


def short_name(name):
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0]


def trace_report(directory, title, command):
    rows = _csv(directory, "kernel_stats.csv")
    out = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", "```", command, "```", "",
           "`rocprofv3 --kernel-trace --stats` kernel statistics (durations in microseconds):", "",
           "| kernel | calls | total us | average us | min us | max us | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.3f} | {float(r['MinNs']) / 1e3:.3f} | "
                   f"{float(r['MaxNs']) / 1e3:.3f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out) + "\n"


def _z_shape(line):
    """Block size and grid (threads) of the benchmarked plan's fused z launches."""
    cfg, tune = line["config"], line.get("tuning") or {}
    nx, ny, nz = cfg["grid"]
    info = line["plan_info"]
    pz = info["padded"][2]
    groups = info["z_groups"]
    tk = info["tile_z"]
    e = min(pz, info["ez"])
    threads = groups * tk * (pz // e)
    if groups == 1 and e == 8 and pz == 64:       # the wave form: one wave per realisation, up to four a block
        b = cfg["batch"]
        threads = 64 * (4 if b >= 4 else (2 if b >= 2 else 1))
    m1 = info["padded"][0] // 2 + 1
    py = info["padded"][1]
    tiles = (m1 + tk - 1) // tk
    if cfg["batch"] >= 4 and m1 > tk and (m1 - 1) % tk == 0:   # the Nyquist strip (plans of 4 or more)
        blocks = (tiles - 1) * py + (py // 2 + tk) // tk * cfg["batch"]
    else:
        blocks = tiles * py
    return threads, blocks * threads


def traffic(fetch_dir, write_dir, line, copy_mib):
    block, grid = _z_shape(line)
    result = {}
    for counter, directory in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _csv(directory, "counter_collection.csv") if r["Counter_Name"] == counter]
        z = [float(r["Counter_Value"]) for r in rows
             if re.search(r"k_z_(serial|grouped|wave)<", r["Kernel_Name"])
             and int(r["Workgroup_Size"]) == block and int(r["Grid_Size"]) == grid]
        other = [float(r["Counter_Value"]) for r in rows if "dds::" not in r["Kernel_Name"]]
        if not z or not other:
            raise SystemExit(f"{counter}: no matching z launches ({block} x {grid}) or no copy kernel")
        copy_kib = max(other)                     # the calibration copy is the largest other transfer
        factor = copy_mib * 1024.0 / copy_kib
        kib = sorted(z)[len(z) // 2]
        result[counter] = dict(launches=len(z), median_kib=kib, copy_kib=copy_kib, factor=factor,
                               bytes=kib * 1024.0 * factor)
    return result


def traffic_report(fetch_dir, write_dir, line_file, copy_mib, title, command):
    line = None
    with open(line_file) as f:
        for text in f:
            text = text.strip()
            if text.startswith("{") and '"metric"' in text:
                line = json.loads(text)
    if line is None:
        raise SystemExit(f"no bench JSON line in {line_file}")
    t = traffic(fetch_dir, write_dir, line, copy_mib)
    roof = line["roofline"]
    alg = roof["algorithmic_bytes_per_launch"]
    total = t["FETCH_SIZE"]["bytes"] + t["WRITE_SIZE"]["bytes"]
    out = [f"# {title}", "", "Commands (from the repository root, one MI355X; one counter per run):", "", "```",
           command.replace("{COUNTER}", "FETCH_SIZE"), command.replace("{COUNTER}", "WRITE_SIZE"), "```", "",
           f"Kernel: `{roof['kernel']}`, launch shape {_z_shape(line)[0]} threads per block.", "",
           "| counter | launches | median KiB per launch | copy kernel KiB | scale | bytes per launch |",
           "|---|---:|---:|---:|---:|---:|"]
    for k in ("FETCH_SIZE", "WRITE_SIZE"):
        r = t[k]
        out.append(f"| {k} | {r['launches']} | {r['median_kib']:.1f} | {r['copy_kib']:.1f} | "
                   f"{r['factor']:.3f} | {r['bytes']:.4g} |")
    out += ["", f"Scale: {copy_mib} MiB plain device copy (reads and writes {copy_mib} MiB).",
            f"Algorithmic bytes per launch: {alg:.4g}; measured HBM traffic {total:.4g} "
            f"({total / alg:.3f} x algorithmic).", "",
            "```", f"source_sha256: {source_digest()}", f"workload: {line['config']['workload']}",
            f"batch: {line['config']['batch']}", f"kernel: {roof['kernel']}",
            f"traffic_bytes_per_launch: {total:.6g}", "```"]
    return "\n".join(out) + "\n"


def kernel_traffic(fetch_dir, write_dir, name_regex, copy_mib):
    """Median FETCH_SIZE and WRITE_SIZE bytes per launch of the kernels whose
    name matches `name_regex`, scaled by the plain copy of `copy_mib` MiB."""
    result = {}
    for counter, directory in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _csv(directory, "counter_collection.csv") if r["Counter_Name"] == counter]
        k = [float(r["Counter_Value"]) for r in rows if re.search(name_regex, r["Kernel_Name"])]
        other = [float(r["Counter_Value"]) for r in rows if "dds::" not in r["Kernel_Name"]]
        if not k or not other:
            raise SystemExit(f"{counter}: no launches matching {name_regex!r} or no copy kernel")
        copy_kib = max(other)
        factor = copy_mib * 1024.0 / copy_kib
        kib = sorted(k)[len(k) // 2]
        result[counter] = dict(launches=len(k), median_kib=kib, copy_kib=copy_kib, factor=factor,
                               bytes=kib * 1024.0 * factor)
    return result


def relax_traffic_report(fetch_dir, write_dir, line_file, copy_mib, title, command):
    """Traffic report of the FP32 relaxation step (`bench.py --relax`)."""
    line = None
    with open(line_file) as f:
        for text in f:
            text = text.strip()
            if text.startswith("{") and '"metric"' in text:
                line = json.loads(text)
    if line is None:
        raise SystemExit(f"no bench JSON line in {line_file}")
    t = kernel_traffic(fetch_dir, write_dir, r"k_relax_march<float", copy_mib)
    alg = line["roofline"]["algorithmic_bytes_per_launch"]
    total = t["FETCH_SIZE"]["bytes"] + t["WRITE_SIZE"]["bytes"]
    out = [f"# {title}", "", "Commands (from the repository root, one MI355X; one counter per run):", "", "```",
           command.replace("{COUNTER}", "FETCH_SIZE"), command.replace("{COUNTER}", "WRITE_SIZE"), "```", "",
           "Kernel: `k_relax_march<float, ...>` (one explicit step of the FP32 relaxation).", "",
           "| counter | launches | median KiB per launch | copy kernel KiB | scale | bytes per launch |",
           "|---|---:|---:|---:|---:|---:|"]
    for k in ("FETCH_SIZE", "WRITE_SIZE"):
        r = t[k]
        out.append(f"| {k} | {r['launches']} | {r['median_kib']:.1f} | {r['copy_kib']:.1f} | "
                   f"{r['factor']:.3f} | {r['bytes']:.4g} |")
    out += ["", f"Scale: {copy_mib} MiB plain device copy (reads and writes {copy_mib} MiB).",
            f"Algorithmic bytes per step (u and f read, u written, the ghost layers): {alg:.4g}; measured HBM "
            f"traffic of the step kernel {total:.4g} ({total / alg:.3f} x algorithmic).", "",
            "```", f"source_sha256: {source_digest(RELAX_SOURCES)}", f"workload: {line['config']['workload']}",
            "batch: 1", "kernel: k_relax_march", f"traffic_bytes_per_launch: {total:.6g}", "```"]
    return "\n".join(out) + "\n"


def kernels_report(fetch_dir, write_dir, copy_mib, title, command, min_launches=4):
    """Median FETCH_SIZE and WRITE_SIZE bytes per launch of every library
    kernel shape (name, block, grid) with at least `min_launches` launches,
    scaled by the plain copy of `copy_mib` MiB."""
    def load(directory, counter):
        out = {}
        for r in _csv(directory, "counter_collection.csv"):
            if r["Counter_Name"] == counter:
                out.setdefault((short_name(r["Kernel_Name"]), int(r["Workgroup_Size"]), int(r["Grid_Size"])),
                               []).append(float(r["Counter_Value"]))
        return out
    f, w = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy_f = max(v for k, vs in f.items() if "dds::" not in k[0] for v in vs)
    copy_w = max(v for k, vs in w.items() if "dds::" not in k[0] for v in vs)
    sf, sw = copy_mib * 1024.0 / copy_f, copy_mib * 1024.0 / copy_w
    med = lambda vs: sorted(vs)[len(vs) // 2]
    out = [f"# {title}", "", "Commands (from the repository root, one MI355X; one counter per run):", "", "```",
           command.replace("{COUNTER}", "FETCH_SIZE"), command.replace("{COUNTER}", "WRITE_SIZE"), "```", "",
           f"Median HBM bytes per launch: counter KiB x 1024 x scale, the scale from a {copy_mib} MiB plain device "
           f"copy (FETCH_SIZE x {sf:.3f}, WRITE_SIZE x {sw:.3f}).", "",
           "| kernel | block | grid | launches | fetch MB | write MB |", "|---|---:|---:|---:|---:|---:|"]
    for k in sorted(f, key=lambda k: -med(f[k])):
        if "dds::" not in k[0] or len(f[k]) < min_launches:
            continue
        out.append(f"| `{k[0]}` | {k[1]} | {k[2]} | {len(f[k])} | {med(f[k]) * 1024 * sf / 1e6:.1f} | "
                   f"{med(w.get(k, [0.0])) * 1024 * sw / 1e6:.1f} |")
    return "\n".join(out) + "\n"


def counters_report(dirs, title, commands, notes=(), min_launches=4):
    """Median value per launch of every counter collected in the rocprofv3
    `--pmc` runs under `dirs`, for every library kernel shape (name, block,
    grid) with at least `min_launches` launches."""
    vals, names = {}, []
    for directory in dirs:
        for r in _csv(directory, "counter_collection.csv"):
            if "dds::" not in r["Kernel_Name"]:
                continue
            key = (short_name(r["Kernel_Name"]), int(r["Workgroup_Size"]), int(r["Grid_Size"]))
            c = r["Counter_Name"]
            if c not in names:
                names.append(c)
            vals.setdefault(key, {}).setdefault(c, []).append(float(r["Counter_Value"]))
    med = lambda vs: sorted(vs)[len(vs) // 2]
    out = [f"# {title}", "", "Commands (from the repository root, one MI355X):", "", "```", *commands, "```", "",
           *notes, "", "| kernel | block | grid | launches | " + " | ".join(names) + " |",
           "|---|---:|---:|---:|" + "---:|" * len(names)]
    rows = [(k, v) for k, v in vals.items() if len(next(iter(v.values()))) >= min_launches]
    for k, v in sorted(rows, key=lambda kv: kv[0]):
        cells = [f"{med(v[c]):.4g}" if c in v else "" for c in names]
        out.append(f"| `{k[0]}` | {k[1]} | {k[2]} | {len(next(iter(v.values())))} | " + " | ".join(cells) + " |")
    return "\n".join(out) + "\n"


def stored_traffic(profiles_dir, workload, batch, kernel, sources=DEVICE_SOURCES):
    """HBM bytes per launch from a traffic report in `profiles_dir` for this
    workload, batch and kernel, or None when there is none or the device
    sources have changed since it was taken."""
    digest = source_digest(sources)
    for path in sorted(glob.glob(os.path.join(profiles_dir, "*.md"))):
        with open(path) as f:
            text = f.read()
        fields = dict(re.findall(r"^(source_sha256|workload|batch|kernel|traffic_bytes_per_launch): (.+)$",
                                 text, re.M))
        if (fields.get("source_sha256") == digest and fields.get("workload") == workload
                and fields.get("batch") == str(batch) and fields.get("kernel") == kernel):
            return float(fields["traffic_bytes_per_launch"])
    return None


def main(argv):
    if len(argv) >= 4 and argv[0] == "trace":
        sys.stdout.write(trace_report(argv[1], argv[2], argv[3]))
    elif len(argv) >= 7 and argv[0] == "traffic":
        sys.stdout.write(traffic_report(argv[1], argv[2], argv[3], int(argv[4]), argv[5], argv[6]))
    elif len(argv) >= 6 and argv[0] == "kernels":
        sys.stdout.write(kernels_report(argv[1], argv[2], int(argv[3]), argv[4], argv[5]))
    elif len(argv) >= 7 and argv[0] == "relax-traffic":
        sys.stdout.write(relax_traffic_report(argv[1], argv[2], argv[3], int(argv[4]), argv[5], argv[6]))
    else:
        sys.stderr.write(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
