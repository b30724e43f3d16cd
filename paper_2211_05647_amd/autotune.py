"""Launch-shape autotuner for the step kernels.

For a workload it times every candidate tile (E nodes per work-group in 1D, cells per
work-group in 2D) and, for single 1D runs and for batches of 1D runs, every
steps-per-launch value of the temporally blocked kernel, and keeps the fastest in a JSON
cache keyed by (dims, nv, precision, size class) -- for a batch, by its set of Nv and
size class.  Timing runs are short and start
from the zero state; the choices only change the launch shape, never the result (every
tile and every steps-per-launch value gives bitwise-identical fields).
``python -m paper_2211_05647_amd.autotune`` tunes the benchmark workloads.
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
        # 1D tiles shape the one-step kernel: time it without temporal blocking
        sim = B.Sim(run, precision=precision, tile=t, time_block=1 if dims == 1 else None)
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


CANDIDATES_TB = (1, 3, 5, 7, 9)


def lookup_time_block(run, precision):
    """Steps per launch chosen for this workload class (0 = not tuned: library default)."""
    return load().get(key(run, precision), {}).get("time_block", 0)


def tune_time_block(run, precision=B.FP32, steps=630, save=True, log=print):
    """Time every steps-per-launch candidate of the temporally blocked 1D kernel (the
    result is bitwise the same for all of them) and keep the fastest."""
    tile = lookup(run, precision)
    res = {}
    for k in CANDIDATES_TB:
        sim = B.Sim(run, precision=precision, tile=tile, time_block=k)
        if sim.time_block() != k:
            sim.close()
            continue
        sim.run(63)
        sim.run(steps)
        res[k] = sim.last_run_ms()
        sim.close()
        log(f"[autotune] {key(run, precision)} time_block={k}: {res[k] * 1e3:.2f} us/step")
    if not res:
        return 0, res
    best = min(res, key=res.get)
    if save:
        d = load()
        e = d.setdefault(key(run, precision), {})
        e["time_block"] = best
        e["us_per_step_by_time_block"] = {str(k): v * 1e3 for k, v in res.items()}
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
    return best, res


def batch_key(runs, precision):
    """Cache key of a 1D batch: its set of Nv and its size class (total plasma cells)."""
    nvs = ",".join(str(v) for v in sorted({r.nv for r in runs}))
    size = sum(r.plasma_cells for r in runs)
    cls = "s" if size < 65536 else ("m" if size < 1048576 else "l")
    return f"batch-d1-nv{nvs}-p{precision}-{cls}"


def lookup_batch_time_block(runs, precision=B.FP32):
    """Steps per launch chosen for this kind of batch (0 = not tuned: library default)."""
    return load().get(batch_key(runs, precision), {}).get("time_block", 0)


def tune_batch_time_block(runs, precision=B.FP32, steps=1800, save=True, log=print):
    """Time every steps-per-launch candidate of the batch's blocked launch form over the
    first `steps` steps (every run is still going; the result is bitwise the same for
    all candidates) and keep the fastest.  The tile width per Nv group is the widest a
    work-group holds (narrower tiles measured slower: more halo per owned node)."""
    import time
    import torch
    res = {}
    for k in CANDIDATES_TB:
        sim = B.Sim(runs, precision=precision, time_block=k)
        sim.run(2 * max(k, 1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(steps)
        torch.cuda.synchronize()
        res[k] = (time.perf_counter() - t0) / steps
        sim.close()
        log(f"[autotune] {batch_key(runs, precision)} time_block={k}: {res[k] * 1e6:.2f} us/step")
    best = min(res, key=res.get)
    if save:
        d = load()
        e = d.setdefault(batch_key(runs, precision), {})
        e["time_block"] = best
        e["us_per_step_by_time_block"] = {str(k): v * 1e6 for k, v in res.items()}
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
    return best, res


if __name__ == "__main__":
    # tune the launch shapes of the benchmark workloads on the current device
    from . import workloads as W
    for run in (W.c1(), W.c1_large()):
        tune(run)
        tune_time_block(run)
    tune(W.c2(), candidates=(8, 16, 32, 64))
    tune_batch_time_block(W.c3())
