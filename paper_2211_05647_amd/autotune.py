"""Launch-shape autotuner for the step kernels.

For a workload it times every candidate tile (E nodes per work-group in 1D, cells per
work-group in 2D) with HIP events around ``fdtd_plasma_run`` and keeps the fastest in a
JSON cache keyed by (dims, nv, precision, size class).  Timing runs are short and start
from the zero state; the chosen tile only changes the launch shape, never the result
(every tile gives bitwise-identical fields).
"""
from __future__ import annotations

import json
import os

from . import binding as B

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

CANDIDATES_1D = (32, 64, 128, 256)
CANDIDATES_2D = (64, 128, 256, 512)


def key(run, precision):
    dims = 2 if hasattr(run, "ny") else 1
    size = run.plasma_cells
    cls = "s" if size < 4096 else ("m" if size < 262144 else "l")
    return f"d{dims}-nv{run.nv}-p{precision}-{cls}"


def load():
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(run, precision):
    return load().get(key(run, precision), {}).get("tile", 0)


def tune(run, precision=B.FP32, steps=200, candidates=None, save=True, log=print):
    dims = 2 if hasattr(run, "ny") else 1
    cands = candidates or (CANDIDATES_2D if dims == 2 else CANDIDATES_1D)
    res = {}
    for t in cands:
        sim = B.Sim(run, precision=precision, tile=t)
        sim.run(20)
        sim.run(steps)
        ms = sim.last_run_ms()
        res[t] = ms
        sim.close()
        log(f"[autotune] {key(run, precision)} tile={t}: {ms * 1e3:.2f} us/step")
    best = min(res, key=res.get)
    if save:
        d = load()
        d[key(run, precision)] = {"tile": best, "us_per_step": {str(k): v * 1e3 for k, v in res.items()}}
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
    return best, res
