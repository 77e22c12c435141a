"""Autotuning cache: launch shapes chosen by ``ddstress_autotune`` per
(device, grid, precision, channels, batch), kept in a JSON file.

The cache file is ``$DDSTRESS_TUNE_CACHE`` or ``~/.cache/ddstress/tuning.json``.
Tile choices do not change the arithmetic, so a tuned plan gives the same
bits as a default one.
"""
import json
import os
import tempfile

from . import binding as B


def cache_path():
    return os.environ.get("DDSTRESS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ddstress", "tuning.json"))


# Part of every key: entries written for other launch-shape fields are not reused.
LAYOUT = "z4"


def device_tag():
    """Architecture and compute-unit count of the current device (the marketing
    name can read differently under a profiler)."""
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch.split(':')[0]}-{p.multi_processor_count}cu"


def shape_key(desc, device_name=""):
    """Cache key: the transform lengths follow from the grid and the periodic
    axes, the launch shapes from those, the precision, channels and batch."""
    n = "x".join(str(v) for v in desc.n)
    per = "".join(a for a, bit in (("x", 1), ("y", 2)) if desc.flags & bit)
    pbc = f"|pbc{per}" if per else ""
    return f"{device_name}|{n}{pbc}|fp{desc.precision}|C{3 * desc.n_lines}|B{desc.batch}|{LAYOUT}"


def _read(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _write(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path), prefix=".tuning")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def to_dict(t):
    return {"rows_x": t.rows_x, "tk_y": t.tk_y, "tk_z": t.tk_z, "ex": t.ex, "ey": t.ey, "ez": t.ez,
            "z_groups": t.z_groups, "yx": t.yx, "xy": t.xy, "ms": [round(float(v), 5) for v in t.ms]}


def from_dict(d):
    t = B.Tuning()
    t.rows_x, t.tk_y, t.tk_z = int(d["rows_x"]), int(d["tk_y"]), int(d["tk_z"])
    t.ex, t.ey, t.ez = int(d.get("ex", 0)), int(d.get("ey", 0)), int(d.get("ez", 0))
    t.z_groups = int(d.get("z_groups", 0))
    t.yx = int(d.get("yx", 0))
    t.xy = int(d.get("xy", 0))
    for i, v in enumerate(d.get("ms", [0, 0, 0])[:3]):
        t.ms[i] = float(v)
    return t


def get_tuning(desc, stream=None, path=None, refresh=False):
    """The cached tuning for this shape, running the autotuner on a miss."""
    import torch
    path = path or cache_path()
    key = shape_key(desc, device_tag())
    data = _read(path)
    if not refresh and key in data:
        return from_dict(data[key])
    t = B.autotune(desc, stream)
    data = _read(path)
    data[key] = to_dict(t)
    _write(path, data)
    return t


def tuned_plan(desc, stream=None, path=None):
    """A plan built with the cached (or freshly measured) launch shapes."""
    return B.Plan(desc, stream=stream, tuning=get_tuning(desc, stream, path))
