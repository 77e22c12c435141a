#!/usr/bin/env python3
"""Write the stored expected values used by the full-size GPU parity tests.

Every value here is computed by the FP64 oracle (``oracle.stress_direct``,
the direct sum of Eq. (10) over all cells) on inputs from the seeded
generators in ``paper_1804_01830_amd.workloads``; nothing comes from the HIP
path. Run from the repository root:

    python tests/golden/make_golden.py [name ...]

Each fixture is a JSON file with the generator call, the target cells
(i, j, k) and the six Voigt stress components at each target.
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import stress_direct  # noqa: E402
from paper_1804_01830_amd import workloads as W  # noqa: E402


def _targets(n, count, seed):
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    fixed = [[0, 0, 0], [nx - 1, ny - 1, nz - 1], [nx // 2, ny // 2, 0], [nx - 1, 0, nz // 2]]
    rand = [[int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))] for _ in range(count - len(fixed))]
    return np.array(fixed + rand)


FIXTURES = {
    # 256 x 256 x 64 columnar polycrystal, edge and 15.6-degree mixed lines, nu = 0.2
    "poly_layer_256x256x64": dict(gen="poly_layer", kwargs={}, batch_index=0, targets=10, seed=31),
    # the largest served shape: 256 x 256 x 128 (z transforms of length 256)
    "poly_layer_256x256x128": dict(gen="poly_layer", kwargs={"nz": 128}, batch_index=0, targets=10, seed=51),
    # two realisations of the 64-realisation sweep (grain sizes 4 and 32 cells)
    "poly_sweep_128x128x32_b0": dict(gen="poly_sweep", kwargs={}, batch_index=0, targets=6, seed=41),
    "poly_sweep_128x128x32_b63": dict(gen="poly_sweep", kwargs={}, batch_index=63, targets=6, seed=42),
}


def _one(args):
    rho, d, lines, mu, nu, tg = args
    return stress_direct(rho, d, lines, mu, nu, targets=tg[None, :])[:, 0]


def make(name):
    spec = FIXTURES[name]
    w = getattr(W, spec["gen"])(**spec["kwargs"])
    tg = _targets(w["n"], spec["targets"], spec["seed"])
    rho = w["rho"][spec["batch_index"]]
    t = time.time()
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        vals = pool.map(_one, [(rho, w["d"], w["lines"], w["mu"], w["nu"], x) for x in tg])
    out = {
        "name": name,
        "generator": f"paper_1804_01830_amd.workloads.{spec['gen']}(**{spec['kwargs']})",
        "batch_index": spec["batch_index"],
        "n": list(w["n"]), "d": list(w["d"]), "mu": w["mu"], "nu": w["nu"],
        "lines": np.asarray(w["lines"]).tolist(),
        "oracle": "oracle.stress_direct (FP64 direct sum of Eq. 10 over all cells)",
        "targets": tg.tolist(),
        "sigma_voigt": [[float(repr_v) for repr_v in v] for v in vals],
    }
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {len(tg)} targets in {time.time() - t:.1f} s", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(FIXTURES)):
        make(n)
