#!/usr/bin/env python3
"""Throughput of the kinetic-FDTD step on one MI355X.

One benchmark step is one leap-frog time step of the whole coupled path (H update,
F1 update driven by E, FP64 current moment, E update with -J, Mur ends, soft source) on
the large 1D workload: Nx = 65536 cells, Nv = 512 velocity bins, plasma over nodes
[400, Nx-100) with a smoothed random density (omega_p/omega in [0.2, 2]) and
log-uniform collision rates, FP32 storage with FP64 moments.  Inputs are synthetic and
seeded.  The metric counts phase-space updates (plasma cell x signed velocity bin x
step) per second.

Prints one JSON line.  The timed region (exactly --steps steps after --warmup untimed
ones) is repeated --reps times; ``value`` is the median.  Inside it the K-step
temporally blocked launches run back to back in one call bracketed by HIP events on the
launch stream, which gives the dominant kernel's average launch time for the roofline;
the remainder steps follow in a second call.  The other workloads (Nx =
2^20 line, the 2D column, the batch of 256 runs, the learned closure, the full and
two-term models, the 3D slab) are timed under "extra" unless --quick is given.  All use
of the FP64 oracle sits in one leg that runs after the GPU timing (``cpu_baseline_leg``):
the oracle's own rate on the host cores (all threads and one), and the error of every
result against it on a bounded sample.

``--calibrate-copy`` only runs a plain device copy of known size (the reference kernel
for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE).  ``--gpus N`` with N > 1 exits: this
path runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
# MI355X published peaks: FP32 vector 157.3 TFLOP/s (dual-issue / packed FP32), dense
# BF16 MFMA 2.5 PFLOP/s.  The single-issue FP32 rate, 256 CUs x 4 SIMDs x 16 lanes x 2
# flops (FMA) x 2.4 GHz, is what code without packed FP32 instructions can reach.
FP32_PEAK_TFLOPS = 157.3
FP32_SINGLE_ISSUE_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
BF16_PEAK_TFLOPS = 2500.0
# arithmetic of one stored-bin update in the blocked kernel: per step two FP32 FMAs
# (F1 + c n E, then + d F1: 4) and the FP64 moment FMA (2); once per launch the
# Crank-Nicolson coefficients d = -2x / (2 + x) and c = b / (2 + x) (an FMA and a
# reciprocal for 1 / (2 + x), two products for d, one for c: 6)
FLOPS_PER_BIN_STEP = 6
FLOPS_PER_BIN_LAUNCH = 6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash(files):
    """Hash of the kernel sources a counter summary was taken on."""
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2211_05647_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


PMC_FILES = {
    "k_step1d_tb_c1_pmc.json": ("common.h", "kernels1d_tb.hip"),
    "k_step1d_c1_pmc.json": ("common.h", "kernels1d.hip"),
    "k_step1d_tb_c1l_pmc.json": ("common.h", "kernels1d_tb.hip"),
    "k_step1d_c3_batch_pmc.json": ("common.h", "kernels1d.hip", "kernels1d_tb.hip"),
}


def pmc_file(name):
    """A counter summary from profiles/ if it was taken on the kernel sources as they are."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash(PMC_FILES[name]):
        return None
    return d


def pmc_bytes(name):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was taken on
    the kernel sources as they are now (else None)."""
    d = pmc_file(name)
    return d.get("hbm_bytes_per_launch") if d else None


def bytes_1d(run, fb=4):
    """Algorithmic bytes of one launch of the 1D step kernel: F1 read + write (half grid,
    fb-byte values: 4 in FP32 storage, 8 in FP64), per-cell scalars (node index, dt*nu,
    density), fields (E and H read and written, J written) over the whole line."""
    ncell, half, nx = run.plasma_cells, run.nv // 2, run.nx
    return ncell * half * fb * 2 + ncell * (4 + 2 * fb) + (nx + 1) * fb * 5


def bytes_1d_blocked(run, rows, row_values=None):
    """Algorithmic bytes of one launch of a temporally blocked kernel (K steps): the rows
    it reads (owned + halo) with their per-cell scalars, the owned rows written back,
    the fields read and written once per launch.  row_values: stored values per row
    (Nv/2 for the linear model)."""
    rv = run.nv // 2 if row_values is None else row_values
    return rows * (rv * 4 + 12) + run.plasma_cells * rv * 4 + (run.nx + 1) * 4 * 5


def bytes_2d(run):
    """Algorithmic bytes of one 2D step (both launches): F1 read + write, per-cell
    scalars and E gather, Ex/Ey/Hz read + written, cell currents written and read."""
    ncell, half, nx, ny = run.plasma_cells, run.nv * run.nv // 2, run.nx, run.ny
    npt = nx * ny
    return ncell * half * 4 * 2 + ncell * (12 + 16 + 8) + npt * 4 * (6 + 4)


def bytes_1d_full(run):
    """Algorithmic bytes of one launch of the full-model one-step kernel: the node's whole
    row (odd and even halves of f - n fhat, Nv values, FP32) read + written, per-cell
    scalars, fields over the line."""
    ncell, nv, nx = run.plasma_cells, run.nv, run.nx
    return ncell * nv * 4 * 2 + ncell * 12 + (nx + 1) * 4 * 5


def bytes_3d(run, npoints, row):
    """Algorithmic bytes of one 3D step (three launches): H read + written and E read once
    by the H update; E read + written and H read by the E update; CPML memory read +
    written inside the strips; F1 rows read + written with their scalars, E read and
    written (J taken off in place) and J written by the kinetic update (FP32)."""
    X, Y, Z, m = run.nx, run.ny, run.nz, run.ncpml
    cells = X * Y * Z
    strips = 4 * 2 * m * (X * Y + Y * Z + Z * X) if m > 0 else 0.0
    return (cells * 3 * 4 * 3 + cells * 3 * 4 * 3 + strips * 8
            + npoints * (row * 8 + 12 + 12))


def bytes_3d_tt(run, npoints, ncells, row):
    """bytes_3d plus the two-term traffic (FP32): per plasma cell its F0 row read by the
    kinetic update and read + written by the l = 0 update, and its 12 (point, E index)
    pairs; per plasma point its four cell rows' indices and its E^n (written by the
    kinetic update), and its F1 row, E^n and E^{n+1} read by the l = 0 update."""
    return (bytes_3d(run, npoints, row) + ncells * (row * 4 * 3 + 96)
            + npoints * (16 + 4 + row * 4 + 8))


def hbm(by, ms):
    """GB/s and fraction of the HBM peak of `by` bytes moved in `ms` milliseconds."""
    gbs = by / (ms * 1e-3) / 1e9
    return gbs, gbs / HBM_PEAK_GBS


# ---------------------------------------------------------------------------------------
# GPU timing
# ---------------------------------------------------------------------------------------
def blocked_kernel(k, half):
    """Name of the kernel a single run's K-step launches use."""
    return f"k_step1d_tb<{k}, {half // 4}>"


def time_1d(run, B, torch, steps, warmup, tile=0, time_block=0, reps=1):
    """Time `reps` regions of exactly `steps` steps of a single 1D run.  A region is two
    library calls: the q K-step blocked launches (K = steps per launch in effect,
    q = steps // K), then the remainder steps; HIP events on the launch stream around the
    first call give the blocked kernel's mean time per launch (back-to-back launches of
    one call, so per-launch events do not perturb the timeline).  Returns wall seconds
    per region, the mean blocked-launch time (ms), K and the rows one blocked launch
    reads."""
    sim = B.Sim(run, precision=B.FP32, tile=tile, time_block=time_block or None)
    k, rows = sim.time_block(rows=True)
    if k > 1 and warmup < 2 * k:
        # a short warm-up (fewer steps than two blocked launches) would leave the blocked
        # kernel's first launch -- code-object load included -- inside the timed region:
        # take it on a throwaway copy of the run instead, so that the run itself still
        # takes exactly `warmup` untimed steps
        pre = B.Sim(run, precision=B.FP32, tile=tile, time_block=k)
        pre.run(2 * k + 1)
        torch.cuda.synchronize()
        pre.close()
    sim.run(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    walls, launch, nlaunch = [], [], 0
    for _ in range(reps):
        q, r = divmod(steps, k) if k > 1 else (0, steps)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if q:
            e0.record(stream)
            sim.run(q * k)
            e1.record(stream)
        if r:
            sim.run(r)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        if q:
            launch.append(e0.elapsed_time(e1) / q)
            nlaunch += q
    if hasattr(run, "ny"):
        sim.read(B.F_EY)
    else:
        sim.read(B.F_E)
    sim.close()
    return dict(walls=walls, k=k, rows=rows,
                launch_ms=(statistics.median(launch) if launch else None),
                launch_ms_reps=launch, launches_timed=nlaunch)


def time_steps(run, B, torch, steps, warmup, reps=3, **kw):
    """Median device time per step (HIP events around fdtd_plasma_run) and wall time of
    `reps` calls of `steps` steps each (2D and 3D runs, one-step-per-launch 1D runs)."""
    kw.setdefault("precision", B.FP32)
    sim = B.Sim(run, **kw)
    sim.run(warmup)
    torch.cuda.synchronize()
    ms, walls = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        sim.run(steps)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        ms.append(sim.last_run_ms())
    extra = sim.closure_counts() if kw.get("closure") else None
    sim.close()
    return statistics.median(ms), statistics.median(walls), extra


def blocked_entry(run, t, steps, row_values=None, kernel=None):
    """Throughput and roofline figures of a 1D run timed with time_1d."""
    wall = statistics.median(t["walls"])
    out = dict(updates_per_s=run.plasma_cells * run.nv * steps / wall,
               ms_per_step=wall / steps * 1e3, steps_per_launch=t["k"],
               wall_s_reps=t["walls"])
    if t["k"] > 1 and t["launch_ms"]:
        by = bytes_1d_blocked(run, t["rows"], row_values)
        gbs, frac = hbm(by, t["launch_ms"])
        out.update(kernel=kernel, launch_ms=t["launch_ms"], launches_timed=t["launches_timed"],
                   bytes_per_launch=by, hbm_gbs=gbs, hbm_frac=frac,
                   one_step_stream_equivalent_gbs=(
                       (run.plasma_cells * (row_values or run.nv // 2) * 8 + run.plasma_cells * 12
                        + (run.nx + 1) * 20) * t["k"] / (t["launch_ms"] * 1e-3) / 1e9))
    return out


def extra_c1l(B, W, torch, autotune):
    """1D line with Nx = 2^20: F1 (1.07 GB) far above every cache."""
    run = W.c1_large()
    log(f"c1l: Nx={run.nx} plasma cells={run.plasma_cells}")
    tile = autotune.lookup(run, B.FP32)
    t = time_1d(run, B, torch, run.steps, 49, tile, autotune.lookup_time_block(run, B.FP32), reps=3)
    out = blocked_entry(run, t, run.steps, kernel=blocked_kernel(t["k"], run.nv // 2))
    out["workload"] = "1D Yee + 1V kinetic, Nx=1048576, Nv=512, FP32, 2000 steps"
    out["hbm_bytes_per_launch_counters"] = pmc_bytes("k_step1d_tb_c1l_pmc.json")
    # one step per launch on the same line: the streaming kernel beyond the Infinity Cache
    ms1, _, _ = time_steps(run, B, torch, 300, 20, reps=3, tile=tile, time_block=1)
    gbs, frac = hbm(bytes_1d(run), ms1)
    out["one_step_per_launch"] = dict(kernel="k_step1d<float, 1, true>", ms_per_step=ms1,
                                      bytes_per_launch=bytes_1d(run), hbm_gbs=gbs, hbm_frac=frac)
    return {"c1_nx2e20": out}


def extra_full(B, W, torch, steps=None):
    """The full-distribution model (F0 evolves, electrons heat) on the C1 line and on the
    Nx = 2^20 line, FP32: K steps per launch (9 and 7, the measured best), and one step
    per launch beside it."""
    out = {}
    for key, run, steps, kb in (("full_c1", W.c1(steps=2000), steps or 2000, 9),
                                ("full_c1_nx2e20", W.c1_large(), steps or 300, 7)):
        run.kinetic = "full"
        log(f"{key}: Nx={run.nx} Nv={run.nv} plasma cells={run.plasma_cells}")
        t = time_1d(run, B, torch, steps - steps % kb, 6 * kb, 0, kb, reps=3)
        e = blocked_entry(run, t, steps - steps % kb, row_values=run.nv,
                          kernel=f"k_step1d_tb_full<{t['k']}, 64>")
        ms1, _, _ = time_steps(run, B, torch, steps, 50, reps=3, time_block=1)
        gbs, frac = hbm(bytes_1d_full(run), ms1)
        streamed = run.plasma_cells * run.nv * 4 > (192 << 20)   # the library's threshold
        e["one_step_per_launch"] = dict(
            kernel=f"k_step1d_full<float, 1, {'true' if streamed else 'false'}>",
            ms_per_step=ms1, hbm_gbs=gbs, hbm_frac=frac)
        e["workload"] = (f"1D Yee + full-distribution 1V kinetic, Nx={run.nx}, Nv={run.nv}, "
                         f"FP32, {steps} steps")
        out[key] = e
    return out


def extra_twoterm(B, W, torch, steps=2000):
    """The two-term model on the speed grid (F1 and an evolving F0, v_dim = 31, Druyvesteyn
    F0 at 1 eV) on the large line's density and collision profile, FP32: 9 steps per
    launch, and one step per launch beside it."""
    run = twoterm_line(W, steps)
    log(f"two-term: Nx={run.nx} v_dim={run.nv} plasma cells={run.plasma_cells}")
    n = steps - steps % 9
    t = time_1d(run, B, torch, n, 54, 0, 9, reps=3)
    e = blocked_entry(run, t, n, row_values=64, kernel=f"k_step1d_tb_tt<{t['k']}, 8>")
    e["updates_per_s"] = run.plasma_cells * run.nv * n / statistics.median(t["walls"])
    ms1, _, _ = time_steps(run, B, torch, steps, 50, reps=3, time_block=1)
    by1 = run.plasma_cells * (2 * 32 * 4 * 2 + 12 + 4) + (run.nx + 1) * 4 * 5
    gbs, frac = hbm(by1, ms1)
    e["one_step_per_launch"] = dict(kernel="k_step1d_tt<float>", ms_per_step=ms1, hbm_gbs=gbs,
                                    hbm_frac=frac)
    e["workload"] = (f"1D Yee + two-term speed-grid kinetic (F0 evolving), Nx={run.nx}, "
                     f"v_dim={run.nv}, FP32, {steps} steps")
    return {"two_term_c1": e}


def twoterm_line(W, steps):
    run = W.c1(steps=steps)
    run.kinetic, run.nv, run.f0_model = "two_term", 31, "druyvesteyn"
    run.te_ev, run.vmax_over_vth = 1.0, 5.0
    return run


def extra_3d(B, W, torch, steps=300, kinetic="linear"):
    """The paper's production model in 3D: the argon-style slab (Druyvesteyn F0, v_dim = 31
    speeds, a 4 mm slab along z, sheet source, CPML on all faces) at 128 x 128 x 512, with
    F0 held (linear) or evolving in every plasma cell (two_term; its slab ends where the x
    and y absorbing layers begin, which that model needs to stay stable)."""
    tt = kinetic == "two_term"
    run = W.argon_slab_3d(nx=128, ny=128, nz=512, steps=steps, kinetic=kinetic)
    sim = B.Sim(run, precision=B.FP32)
    npoints = sim.closure_counts()[1]
    sim.close()
    ncells = run.plasma_cells if tt else 0
    key = "argon3d_two_term" if tt else "argon3d"
    log(f"{key}: {run.nx}x{run.ny}x{run.nz}, plasma points {npoints}, cells {ncells}")
    ms, wall, _ = time_steps(run, B, torch, steps, 20, reps=3)
    by = bytes_3d_tt(run, npoints, ncells, 32) if tt else bytes_3d(run, npoints, 32)
    gbs, frac = hbm(by, ms)
    cells = run.nx * run.ny * run.nz
    model = "two-term F1 + evolving F0" if tt else "speed-grid F1"
    return {key: dict(workload=f"3D Yee + CPML + {model} (v_dim {run.nv}, Druyvesteyn), "
                               f"{run.nx}x{run.ny}x{run.nz}, FP32, {steps} steps",
                      plasma_points=npoints, plasma_cells=ncells, cells=cells,
                      updates_per_s=npoints * run.nv / (ms * 1e-3),
                      nmcps=cells / (ms * 1e-3) * 1e-6, ms_per_step=ms,
                      wall_ms_per_step=wall / steps * 1e3, bytes_per_step=by,
                      hbm_gbs=gbs, hbm_frac=frac)}


def extra_fp64(B, W, torch, steps=None):
    """The headline line in FP64 storage and arithmetic (the precision of the paper's
    MATLAB code): one step per launch (temporal blocking is an FP32 path)."""
    run = W.c1()
    steps = steps or 2000
    log(f"fp64: Nx={run.nx} Nv={run.nv} plasma cells={run.plasma_cells}")
    ms, wall, _ = time_steps(run, B, torch, steps, 20, reps=3, precision=B.FP64)
    by = bytes_1d(run, 8)
    gbs, frac = hbm(by, ms)
    return {"c1_fp64": dict(workload=f"1D Yee + 1V kinetic, Nx=65536, Nv=512, FP64, {steps} steps",
                            kernel="k_step1d<double, 2, false>",
                            updates_per_s=run.plasma_cells * run.nv / (ms * 1e-3),
                            ms_per_step=ms, wall_ms_per_step=wall / steps * 1e3,
                            bytes_per_launch=by, hbm_gbs=gbs, hbm_frac=frac)}


def extra_c2(B, W, torch, autotune, steps=None):
    """2D column, 512^2, 32x32 velocity bins."""
    run = W.c2()
    steps = steps or run.steps
    log(f"c2: {run.nx}x{run.ny} plasma cells={run.plasma_cells}")
    ms, wall, _ = time_steps(run, B, torch, steps, 100, reps=3, tile=autotune.lookup(run, B.FP32))
    gbs, frac = hbm(bytes_2d(run), ms)
    return {"c2": dict(workload=f"2D TEz 512x512 + 2V kinetic 32x32, FP32, {steps} steps",
                       updates_per_s=run.plasma_cells * run.nv ** 2 / (ms * 1e-3),
                       ms_per_step=ms, wall_ms_per_step=wall / steps * 1e3,
                       bytes_per_step=bytes_2d(run), hbm_gbs=gbs, hbm_frac=frac)}


def extra_c3(B, W, torch, reps=3, autotune=None, limit=None):
    """Batch of 256 uneven 1D runs, advanced to the last run's end in its default launch
    form (blocked launches per Nv group), with the steps per launch the autotuner stored
    for this batch (the library default if none), and then in one persistent launch
    (batch mode 0) for comparison.  `limit` stops after that many steps
    instead, with a progress line every 1000 steps (for counter collection, which
    serialises every dispatch)."""
    runs = W.c3()
    kb = autotune.lookup_batch_time_block(runs) if autotune else 0
    if limit:
        sim = B.Sim(runs, time_block=kb or None)
        done = 0
        while done < limit:
            n = min(1000, limit - done)
            sim.run(n)
            torch.cuda.synchronize()
            done += n
            log(f"c3: {done} of {limit} steps")
        sim.close()
        return {"c3_prefix": dict(steps=limit, steps_per_launch=kb or None)}
    work = sum(r.plasma_cells * r.nv * r.steps for r in runs)
    stream_by = sum(bytes_1d(r) * r.steps for r in runs)
    tot = max(r.steps for r in runs)
    log(f"c3: {len(runs)} runs, {tot} steps max")
    walls = []
    for _ in range(reps):
        sim = B.Sim(runs, time_block=kb or None)
        k_used = sim.time_block()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(tot)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        sim.close()
    wall = statistics.median(walls)
    # the same batch in one persistent launch (batch mode 0), for comparison
    pwalls = []
    for _ in range(2):
        sim = B.Sim(runs, time_block=kb or None, batch_mode=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(tot)
        torch.cuda.synchronize()
        pwalls.append(time.perf_counter() - t0)
        sim.close()
    out = dict(workload="256 independent 1D runs, Nx in [500, 20000], Nv in {64,128,256}, "
                        "2 Nx steps each",
               updates_per_s=work / wall, seconds=wall, seconds_reps=walls,
               launch_form="K-step blocked launches per Nv group (batch mode 1)",
               persistent_launch_seconds=min(pwalls),
               steps_per_launch=k_used,
               one_step_stream_equivalent_gbs=stream_by / wall / 1e9,
               one_step_stream_equivalent_frac=stream_by / wall / 1e9 / HBM_PEAK_GBS)
    pf = pmc_file("k_step1d_c3_batch_pmc.json")
    if pf:
        # counter traffic of the blocked launches over the batch's first 4500 steps (every
        # run still going), against the same dispatches' trace time
        out["blocked_hbm_gbs_counters_prefix"] = pf["blocked_prefix_hbm_gbs"]
        out["blocked_hbm_frac_counters_prefix"] = pf["blocked_prefix_hbm_gbs"] / HBM_PEAK_GBS
    return {"c3": out}


def c4_steps(B, W, torch, steps):
    """The 4096^2 blob workload for a few steps, kinetic and with a closure network of
    freshly initialised weights (the same instruction stream as a trained one; for
    profiling without the training kernels)."""
    from paper_2211_05647_amd import closure as CL
    run = W.c4()
    dt = run.courant * run.dx / 299792458.0
    blob = CL.make_blob(CL.init_params(3), (0.0, 1.0, -6.0, 1.0), dt)
    res = {}
    for name, kw in (("kinetic", dict()), ("closure", dict(closure=B.CLOSURE_MLP, mlp_blob=blob))):
        ms, _, _ = time_steps(run, B, torch, steps, 3, reps=1, **kw)
        res[name + "_ms_per_step"] = ms
        if name == "kinetic":
            res["kinetic_hbm_frac"] = hbm(bytes_2d(run), ms)[1]
        torch.cuda.empty_cache()
    return {"c4_steps": res}


def slab_transmission(B, W, blob, closure, nu_ratio, ratio=0.8, nsteps=3000):
    """|T(f)| of a plasma slab (2D, 1400 x 18 cells, 32x32 bins) over the pulse's band,
    from the field behind it against a plasma-free run, with the kinetic step or the
    learned closure."""
    import math
    nx, ny, lo, hi = 1400, 18, 650, 850
    ne = np.zeros((ny, nx))
    nu = np.zeros((ny, nx))
    ne[:, lo:hi] = W.density_from_ratio(ratio, W.F_REF)
    nu[:, lo:hi] = nu_ratio * 2 * math.pi * W.F_REF
    mk = lambda a, b, name: W.Run2D(name=name, nx=nx, ny=ny, nv=32, ne=a, nubar=b, src_kind=1,
                                    src_i=350, src_j=0, steps=nsteps, ncpml=8, te_ev=5.0,
                                    **W.pulse(W.F_REF))
    out = []
    for r, cl in ((mk(np.zeros_like(ne), np.zeros_like(nu), "vac"), B.CLOSURE_KINETIC),
                  (mk(ne, nu, "slab"), closure)):
        sim = B.Sim(r, closure=cl, mlp_blob=blob if cl == B.CLOSURE_MLP else None,
                    max_probes=1, probe_capacity=nsteps)
        pid = sim.add_probe(B.F_EY, 950, 9)
        sim.run(nsteps)
        out.append(sim.read_probe(pid, nsteps))
        sim.close()
    dt = 0.5 * W.DX_REF / 299792458.0
    fs = np.linspace(0.6, 1.6, 41) * W.F_REF
    n = np.arange(nsteps)
    dft = lambda x, f: np.sum(x * np.exp(2j * math.pi * f * n * dt))
    pin, ptot = out
    spec = np.array([abs(dft(pin, f)) for f in fs])
    fs = fs[spec >= 0.1 * spec.max()]
    return np.array([abs(dft(ptot, f) / dft(pin, f)) for f in fs])


def closure_speedup(B, W, torch, steps=50):
    """4096^2 blob workload: time per step with every plasma cell on the kinetic F1 step,
    and with the trained closure (cells outside the training box stay kinetic).  The
    closure is trained first on the batch workload's taps (timed separately).  Beside
    it, the accuracy bar of the surrogate: slab |T| against the kinetic model."""
    from paper_2211_05647_amd import closure as CL
    t0 = time.perf_counter()
    data, c = CL.gather_data(log=log)
    t1 = time.perf_counter()
    params, hist = CL.fit(data, c, log=lambda m: None)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    net, zero = CL.evaluate(data, c, data.held)
    blob = CL.make_blob(params, data.box, data.dt)
    c.close()
    run = W.c4()
    log(f"c4: {run.nx}x{run.ny}, plasma cells {run.plasma_cells}")
    res = {}
    for name, kw in (("kinetic", dict()), ("closure", dict(closure=B.CLOSURE_MLP, mlp_blob=blob))):
        ms, wall, cnt = time_steps(run, B, torch, steps, 5, reps=3, **kw)
        res[name] = ms
        res[name + "_wall"] = wall / steps * 1e3
        if cnt:
            res["closure_cells"], res["fallback_cells"] = cnt
        torch.cuda.empty_cache()
    rows = 2 * res["closure_cells"]
    flops = rows * 2 * (18 * 128 + 128 * 128 + 128)
    slab = {}
    zero_blob = CL.make_blob(np.zeros(B.NPARAM, dtype=np.float32), data.box, data.dt)
    for nr in (0.05, 0.4):
        tk = slab_transmission(B, W, None, B.CLOSURE_KINETIC, nr)
        tm = slab_transmission(B, W, blob, B.CLOSURE_MLP, nr)
        tz = slab_transmission(B, W, zero_blob, B.CLOSURE_MLP, nr)
        slab[f"nu_over_w_{nr}"] = dict(max_abs_T_error_network=float(np.max(np.abs(tm - tk))),
                                       max_abs_T_error_without_network=float(np.max(np.abs(tz - tk))))
    return {"c4_closure": dict(
        workload="2D TEz 4096x4096, 48 plasma blobs, 32x32 bins; learned closure vs kinetic",
        kinetic_ms_per_step=res["kinetic"], closure_ms_per_step=res["closure"],
        speedup=res["kinetic"] / res["closure"], closure_cells=res["closure_cells"],
        fallback_cells=res["fallback_cells"],
        kinetic_hbm_frac=hbm(bytes_2d(run), res["kinetic"])[1],
        network_tflops_lower_bound=flops / (res["closure"] * 1e-3) / 1e12,
        network_frac_of_bf16_peak_lower_bound=flops / (res["closure"] * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
        surrogate_slab_T_vs_kinetic=slab,
        training=dict(gather_s=t1 - t0, fit_s=t2 - t1, held_out_mse=net,
                      held_out_mse_without_net=zero))}


def nmcps_sweep(B, W, torch, cpu_budget_s=2.0):
    """Execution speed against mesh size, in the paper's measure (eq. (5): NMCPS = steps x
    cells / seconds x 1e-6): a 2D TEz vacuum grid with 8-cell CPML and a soft line source,
    n x n cells from 32^2 to 4096^2, on the GPU (FP32) and on the host with the FP64 oracle
    (sizes up to 512^2, time-bounded).  Beside it, the coupled 1D kinetic line (Nv = 512,
    plasma over all but the ends) against its length, in phase-space updates/s."""
    sys.path.insert(0, ROOT)
    from oracle.core import Oracle2D, threads
    out = {"vacuum_2d": [], "kinetic_1d": []}
    for n in (32, 64, 128, 256, 512, 1024, 2048, 4096):
        run = W.Run2D(name=f"vac{n}", nx=n, ny=n, nv=8, ne=np.zeros((n, n)),
                      nubar=np.zeros((n, n)), src_kind=1, src_i=n // 8, src_j=0,
                      steps=0, **W.pulse(W.F_REF))
        steps = max(200, min(4000, int(4e9 / (n * n))))
        ms, _, _ = time_steps(run, B, torch, steps, 20, reps=1)
        row = {"n": n, "cells": n * n, "gpu_nmcps": n * n / (ms * 1e-3) * 1e-6, "gpu_us_per_step": ms * 1e3}
        if n <= 512:
            o = Oracle2D(n, n, run.dx, run.courant, run.ne, run.nubar, nv=8, ncpml=run.ncpml,
                         src_kind=1, src_i=run.src_i, src_amp=run.src_amp, src_f=run.src_f,
                         src_tau=run.src_tau, src_t0=run.src_t0)
            t0 = time.perf_counter()
            o.run(5)
            per = (time.perf_counter() - t0) / 5
            k = max(5, int(cpu_budget_s / max(per, 1e-7)))
            t0 = time.perf_counter()
            o.run(k)
            row["cpu_oracle_nmcps"] = n * n * k / (time.perf_counter() - t0) * 1e-6
            row["cpu_threads"] = threads()
        out["vacuum_2d"].append(row)
        log(f"sweep 2D vacuum {n}^2: {row}")
    for nx in (1024, 4096, 16384, 65536, 262144, 1048576):
        run = W.c1(nx=nx, steps=1)
        steps = max(180, min(4500, int(2e10 / (run.plasma_cells * run.nv)))) // 9 * 9
        sim = B.Sim(run, precision=B.FP32)
        sim.run(18)
        sim.run(steps)
        ms = sim.last_run_ms()
        row = {"nx": nx, "plasma_cells": run.plasma_cells, "time_block": sim.time_block(),
               "updates_per_s": run.plasma_cells * run.nv / (ms * 1e-3), "us_per_step": ms * 1e3}
        sim.close()
        out["kinetic_1d"].append(row)
        log(f"sweep 1D kinetic Nx={nx}: {row}")
    return {"nmcps_sweep": out}


def sweep_3d(B, W, torch, cpu_budget_s=2.0):
    """NMCPS (eq. (5)) of the 3D vacuum cube (CPML on all faces, sheet source) from 16^3
    to 384^3 on the GPU (FP32), and on the host with the FP64 oracle up to 96^3."""
    sys.path.insert(0, ROOT)
    from oracle.core import Oracle3D, threads
    out = []
    for n in (16, 32, 64, 96, 128, 192, 256, 384):
        z = np.zeros((n, n, n))
        run = W.Run3D(name=f"vac3d{n}", nx=n, ny=n, nz=n, nv=1, ne=z, nubar=z, src_kind=1,
                      src_i=0, src_j=0, src_k=n // 4, steps=0, ncpml=min(8, n // 4),
                      **W.pulse(W.F_REF))
        steps = max(60, min(2000, int(2e9 / n ** 3)))
        ms, _, _ = time_steps(run, B, torch, steps, 10, reps=1)
        row = {"n": n, "cells": n ** 3, "gpu_nmcps": n ** 3 / (ms * 1e-3) * 1e-6,
               "gpu_us_per_step": ms * 1e3}
        if n <= 96:
            o = Oracle3D(n, n, n, run.dx, run.courant, z, z, vdim=1, ncpml=run.ncpml,
                         src_kind=1, src_k=run.src_k, src_amp=run.src_amp, src_f=run.src_f,
                         src_tau=run.src_tau, src_t0=run.src_t0)
            t0 = time.perf_counter()
            o.run(3)
            per = (time.perf_counter() - t0) / 3
            k = max(3, int(cpu_budget_s / max(per, 1e-7)))
            t0 = time.perf_counter()
            o.run(k)
            row["cpu_oracle_nmcps"] = n ** 3 * k / (time.perf_counter() - t0) * 1e-6
            row["cpu_threads"] = threads()
        out.append(row)
        log(f"sweep 3D vacuum {n}^3: {row}")
    return {"vacuum_3d": out}


# ---------------------------------------------------------------------------------------
# The oracle leg: the FP64 oracle's rate on the host, and the error of each result
# against it on a bounded sample.  Nothing here is timed as GPU throughput.
# ---------------------------------------------------------------------------------------
def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class _Err:
    """Relative L2 and largest single-element error over arrays compared one at a time
    (space and time), both normalised by the reference over the whole set."""

    def __init__(self):
        self.d2 = self.r2 = self.dmax = self.rmax = 0.0

    def add(self, g, o):
        g = np.asarray(g, dtype=np.float64).ravel()
        o = np.asarray(o, dtype=np.float64).ravel()
        d = g - o
        self.d2 += float(np.dot(d, d))
        self.r2 += float(np.dot(o, o))
        if d.size:
            self.dmax = max(self.dmax, float(np.max(np.abs(d))))
            self.rmax = max(self.rmax, float(np.max(np.abs(o))))
        return self

    def out(self):
        return dict(rel_l2=float(np.sqrt(self.d2 / self.r2)) if self.r2 > 0 else 0.0,
                    max_abs_over_max_ref=self.dmax / self.rmax if self.rmax > 0 else 0.0)


def _err(g, o):
    return _Err().add(g, o).out()


def _oracle_1d(run, nx=None):
    from oracle.core import Oracle1D
    n = run.nx if nx is None else nx
    ne = run.ne[: n + 1].copy()
    if nx is not None:
        ne[n - 1:] = 0.0     # the prefix ends in vacuum; the field never gets there
    return Oracle1D(n, run.dx, run.courant, ne, run.nubar[: n + 1].copy(), nv=run.nv,
                    vmax_over_vth=run.vmax_over_vth, te_ev=run.te_ev, nu_model=run.nu_model,
                    bc=run.bc, src_node=run.src_node, src_amp=run.src_amp, src_f=run.src_f,
                    src_tau=run.src_tau, src_t0=run.src_t0,
                    kinetic=getattr(run, "kinetic", "linear"),
                    f0_model=getattr(run, "f0_model", "maxwell"))


def error_1d_prefix(B, run, steps, every, tile=0, time_block=0, precision=None):
    """A fresh run in the benchmark's launch shape for `steps` steps (the pulse crosses
    the source-to-plasma gap and then runs into the plasma) against the oracle on the
    light cone's prefix of the line, which is exact there: E and the stored distribution
    every `every` steps over the prefix, over space and time."""
    cut = run.src_node + steps + 10
    sim = B.Sim(run, precision=precision or B.FP32, tile=tile, time_block=time_block or None)
    orc = _oracle_1d(run, nx=cut)
    e, d = _Err(), _Err()
    done = 0
    while done < steps:
        n = min(every, steps - done)
        sim.run(n)
        orc.run(n)
        done += n
        e.add(sim.read(B.F_E)[: cut + 1], orc.E)
        d.add(sim.read(B.F_DF)[: orc.df.size], orc.df)
    k = sim.time_block()
    sim.close()
    return dict(E_space_time=e.out(), distribution_space_time=d.out(),
                sample=f"first {steps} steps at {k} steps per launch, oracle on the light "
                       f"cone's prefix [0, {cut}], E and the distribution every {every} steps")


def error_2d(B, run, steps, every, tile=0):
    from oracle.core import Oracle2D
    sim = B.Sim(run, precision=B.FP32, tile=tile)
    orc = Oracle2D(run.nx, run.ny, run.dx, run.courant, run.ne, run.nubar, nv=run.nv,
                   te_ev=run.te_ev, ncpml=run.ncpml, src_kind=run.src_kind, src_i=run.src_i,
                   src_j=run.src_j, src_amp=run.src_amp, src_f=run.src_f, src_tau=run.src_tau,
                   src_t0=run.src_t0)
    e, d = _Err(), _Err()
    done = 0
    while done < steps:
        n = min(every, steps - done)
        sim.run(n)
        orc.run(n)
        done += n
        e.add(np.concatenate([sim.read(B.F_EX), sim.read(B.F_EY)]),
              np.concatenate([orc.Ex.ravel(), orc.Ey.ravel()]))
        d.add(sim.read(B.F_DF), orc.df)
    sim.close()
    return dict(E_space_time=e.out(), distribution_space_time=d.out(),
                sample=f"first {steps} steps, whole grid, Ex, Ey and the distribution every "
                       f"{every} steps")


def error_c3(B, W, nruns=4, seed=221105647):
    """The batch as benchmarked (all 256 runs, default launch form) against the oracle on
    `nruns` seeded runs (the longest among them)."""
    runs = W.c3()
    longest = max(range(len(runs)), key=lambda r: runs[r].steps)
    rest = [r for r in range(len(runs)) if r != longest]
    pick = [longest] + sorted(int(r) for r in np.random.default_rng(seed).choice(rest, nruns - 1, replace=False))
    when = {}
    for r in pick:
        run = runs[r]
        # around the pulse peak's arrival at the slab (where the current is largest:
        # an overdense slab reflects it, a lossy one absorbs it), then half and the end
        dt = run.courant * run.dx / 299792458.0
        lo = int(np.nonzero(run.ne > 0)[0][0])
        hit = 2 * (lo - run.src_node) + run.src_t0 / dt
        for q in sorted({int(hit + d) for d in (-50, 0, 100, 300)} | {run.steps // 2, run.steps}):
            if 1 <= q <= run.steps:
                when.setdefault(q, []).append(r)
    sim = B.Sim(runs)
    orcs = {r: _oracle_1d(runs[r]) for r in pick}
    e, j = _Err(), _Err()
    done = 0
    for t in sorted(when):
        sim.run(t - done)
        done = t
        for r in when[t]:
            orcs[r].run(t - orcs[r].step)
            e.add(sim.read(B.F_E, run=r), orcs[r].E)
            j.add(sim.read(B.F_J, run=r), orcs[r].J)
    sim.close()
    return dict(E_space_time=e.out(), J_space_time=j.out(),
                sample=f"runs {pick} of the batch (as benchmarked), E and J around each "
                       f"run's pulse arrival at its slab, at half and at the end")


def error_3d(B, W, kinetic, steps=800):
    from oracle.core import Oracle3D
    run = W.argon_slab_3d(nx=128, ny=128, nz=512, steps=steps, kinetic=kinetic)
    sim = B.Sim(run, precision=B.FP32)
    sim.run(steps)
    orc = Oracle3D(run.nx, run.ny, run.nz, run.dx, run.courant, run.ne, run.nubar,
                   vdim=run.nv, vmax_over_vth=run.vmax_over_vth, te_ev=run.te_ev,
                   nu_model=run.nu_model, f0_model=run.f0_model, ncpml=run.ncpml,
                   src_kind=run.src_kind, src_k=run.src_k, src_amp=run.src_amp,
                   src_f=run.src_f, src_tau=run.src_tau, src_t0=run.src_t0, kinetic=kinetic)
    orc.run(steps)
    ge = np.concatenate([sim.read(f) for f in (B.F_EX, B.F_EY, B.F_EZ)])
    gj = np.concatenate([sim.read(f) for f in (B.F_JX, B.F_JY, B.F_JZ)])
    out = dict(E=_err(ge, orc.E), J=_err(gj, orc.J), distribution=_err(sim.read(B.F_DF), orc.df),
               sample=f"first {steps} steps (the pulse enters the slab), whole box")
    sim.close()
    return out


def oracle_rate_1d(run, budget_s):
    """The oracle on the full line, as many steps as fit the budget: signed-bin updates/s."""
    o = _oracle_1d(run)
    t0 = time.perf_counter()
    o.run(2)
    per = (time.perf_counter() - t0) / 2
    n = max(2, int(budget_s / max(per, 1e-6)))
    t0 = time.perf_counter()
    o.run(n)
    t = time.perf_counter() - t0
    return run.plasma_cells * run.nv * n / t, n, t


def cpu_baseline_leg(out, B, W, autotune, quick):
    """The FP64 oracle on the host (all threads, then one), and the error of each result
    in `out` against it."""
    sys.path.insert(0, ROOT)
    from oracle.core import Oracle3D, set_threads, threads
    run = W.c1()
    nthreads = threads()
    ups, n, t = oracle_rate_1d(run, 15.0)
    set_threads(1)
    ups1, n1, t1 = oracle_rate_1d(run, 8.0)
    set_threads(nthreads)
    out["cpu_baseline"] = dict(
        value=ups, unit="phase-space updates/s", cores=nthreads, kind="oracle",
        sample=f"large 1D workload, full line (Nx={run.nx}, Nv={run.nv}), {n} steps from the "
               f"zero state, FP64 on the full signed grid, {t:.1f} s",
        one_core=dict(value=ups1, cores=1, sample=f"same line, {n1} steps, {t1:.1f} s"),
        cpu_model=cpu_model(), host_cpus=os.cpu_count())
    c1 = W.c1()
    log("oracle leg: headline error")
    out["error_vs_oracle"] = error_1d_prefix(B, c1, 1800, 300, autotune.lookup(c1, B.FP32),
                                             autotune.lookup_time_block(c1, B.FP32))
    if quick:
        return
    ex = out["extra"]
    log("oracle leg: extras")
    r = W.c1_large()
    ex["c1_nx2e20"]["error_vs_oracle"] = error_1d_prefix(
        B, r, 1400, 350, autotune.lookup(r, B.FP32), autotune.lookup_time_block(r, B.FP32))
    ex["c1_fp64"]["error_vs_oracle"] = error_1d_prefix(B, W.c1(), 1800, 300, precision=B.FP64)
    ex["c2"]["error_vs_oracle"] = error_2d(B, W.c2(), 1000, 250, autotune.lookup(W.c2(), B.FP32))
    ex["c3"]["error_vs_oracle"] = error_c3(B, W)
    r = W.c1(steps=2000)
    r.kinetic = "full"
    ex["full_c1"]["error_vs_oracle"] = error_1d_prefix(B, r, 1800, 300, 0, 9)
    ex["two_term_c1"]["error_vs_oracle"] = error_1d_prefix(B, twoterm_line(W, 2000), 1800, 300, 0, 9)
    ex["argon3d"]["error_vs_oracle"] = error_3d(B, W, "linear")
    ex["argon3d_two_term"]["error_vs_oracle"] = error_3d(B, W, "two_term")
    # the oracle's own rate on the other models' workloads (all threads)
    for key, kin in (("full_c1", "full"), ("two_term_c1", "two_term")):
        r = W.c1(steps=1) if kin == "full" else twoterm_line(W, 1)
        r.kinetic = kin
        ups_k, nk, tk = oracle_rate_1d(r, 5.0)
        ex[key]["cpu_oracle"] = dict(kind="oracle", cores=nthreads, updates_per_s=ups_k,
                                     sample=f"Nx=65536 line, {nk} steps, FP64, {tk:.1f} s")
    for key, kin in (("argon3d", "linear"), ("argon3d_two_term", "two_term")):
        r = W.argon_slab_3d(nx=128, ny=128, nz=512, steps=1, kinetic=kin)
        o = Oracle3D(r.nx, r.ny, r.nz, r.dx, r.courant, r.ne, r.nubar, vdim=r.nv,
                     vmax_over_vth=r.vmax_over_vth, te_ev=r.te_ev, nu_model=r.nu_model,
                     f0_model=r.f0_model, ncpml=r.ncpml, src_kind=r.src_kind, src_k=r.src_k,
                     src_amp=r.src_amp, src_f=r.src_f, src_tau=r.src_tau, src_t0=r.src_t0,
                     kinetic=kin)
        o.run(1)
        t0 = time.perf_counter()
        o.run(4)
        cdt = (time.perf_counter() - t0) / 4
        ex[key]["cpu_oracle"] = dict(kind="oracle", cores=nthreads,
                                     nmcps=r.nx * r.ny * r.nz / cdt * 1e-6,
                                     updates_per_s=ex[key]["plasma_points"] * r.nv / cdt,
                                     sample="4 steps after 1, FP64")


def calibrate_copy(torch):
    """Plain device copies of known size: 10 x (1 GiB read + 1 GiB written); the last five
    are timed (the read + write rate a streaming kernel can reach on this device)."""
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(5):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / 5
    print(json.dumps({"copy_bytes_read_per_launch": n * 4, "copy_bytes_written_per_launch": n * 4,
                      "launches": 10, "copy_ms": ms,
                      "copy_read_plus_write_gbs": 2 * n * 4 / (ms * 1e-3) / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--reps", type=int, default=5, help="timed regions; value is their median")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (host rate and errors against the oracle)")
    ap.add_argument("--quick", action="store_true", help="only the headline workload")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--time-block", type=int, default=0,
                    help="steps per launch of the large 1D workload (default: tuned; 1 = one "
                         "step per launch)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--only", choices=["c1l", "fp64", "c2", "c3", "closure", "c4", "sweep", "full", "3d", "sweep3d",
                             "twoterm", "3dtt"], default=None,
                    help="run only one of the extra measurements (for profiling); c2 and c4 "
                         "take --steps steps; c3 with an explicit --steps runs only that many "
                         "steps of the batch")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the kinetic-FDTD path here runs on a single "
              "MI355X (multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    sys.path.insert(0, ROOT)
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    from paper_2211_05647_amd import autotune
    from paper_2211_05647_amd import binding as B
    from paper_2211_05647_amd import workloads as W
    if args.only:
        only = {"c1l": lambda: extra_c1l(B, W, torch, autotune),
                "c2": lambda: extra_c2(B, W, torch, autotune, args.steps),
                "c3": lambda: extra_c3(B, W, torch, reps=1, autotune=autotune,
                                       limit=args.steps if args.steps != ap.get_default("steps") else None),
                "fp64": lambda: extra_fp64(B, W, torch, min(args.steps, 2000)),
                "closure": lambda: closure_speedup(B, W, torch),
                "c4": lambda: c4_steps(B, W, torch, args.steps),
                "sweep": lambda: nmcps_sweep(B, W, torch),
                "full": lambda: extra_full(B, W, torch, min(args.steps, 2000)),
                "3d": lambda: extra_3d(B, W, torch, args.steps),
                "3dtt": lambda: extra_3d(B, W, torch, args.steps, kinetic="two_term"),
                "sweep3d": lambda: sweep_3d(B, W, torch),
                "twoterm": lambda: extra_twoterm(B, W, torch, min(args.steps, 2000))}[args.only]
        print(json.dumps(only()), flush=True)
        return

    run = W.c1()
    log(f"workload c1: Nx={run.nx} Nv={run.nv} plasma cells={run.plasma_cells}")
    tile = args.tile or autotune.lookup(run, B.FP32)
    t = time_1d(run, B, torch, args.steps, args.warmup, tile,
                args.time_block or autotune.lookup_time_block(run, B.FP32), reps=args.reps)
    ncell, nv, half, nx = run.plasma_cells, run.nv, run.nv // 2, run.nx
    wall = statistics.median(t["walls"])
    value = ncell * nv * args.steps / wall
    kb = t["k"]
    if kb > 1 and t["launch_ms"]:
        # one launch = kb steps of the temporally blocked kernel, priced against HBM with
        # its own algorithmic bytes (rows read with their halo, owned rows written, fields
        # once): its arithmetic intensity lies below the FP32 ridge
        kernel = blocked_kernel(kb, half)
        by = bytes_1d_blocked(run, t["rows"])
        launch_ms = t["launch_ms"]
        achieved, frac = hbm(by, launch_ms)
        flops = (FLOPS_PER_BIN_STEP * kb + FLOPS_PER_BIN_LAUNCH) * ncell * half
        tflops = flops / (launch_ms * 1e-3) / 1e12
        roof = {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": frac,
                "traffic": pmc_bytes("k_step1d_tb_c1_pmc.json"),
                "bytes_per_launch": by, "launch_ms": launch_ms,
                "launch_ms_reps": t["launch_ms_reps"], "launches_timed": t["launches_timed"],
                "flops_per_launch": flops, "intensity_flop_per_byte": flops / by,
                "achieved_tflops": tflops, "frac_of_fp32_peak": tflops / FP32_PEAK_TFLOPS,
                "frac_of_fp32_single_issue": tflops / FP32_SINGLE_ISSUE_TFLOPS,
                "one_step_stream_equivalent_gbs": bytes_1d(run) * kb / (launch_ms * 1e-3) / 1e9}
    else:
        kernel = "k_step1d<float, 1, false>"
        by = bytes_1d(run)
        launch_ms = wall / args.steps * 1e3
        achieved, frac = hbm(by, launch_ms)
        roof = {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": frac, "traffic": pmc_bytes("k_step1d_c1_pmc.json"),
                "bytes_per_launch": by, "launch_ms": launch_ms}
    out = {
        "metric": "kinetic-FDTD phase-space updates/s",
        "value": value,
        "unit": "phase-space updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "moment_dtype": "f64",
        "data": "synthetic, seeded",
        "config": {"workload": "1D Yee + 1V kinetic, Nx=65536, Nv=512, FP32",
                   "nx": nx, "nv": nv, "plasma_cells": ncell, "steps": args.steps,
                   "tile": tile, "steps_per_launch": kb},
        "reps": args.reps,
        "wall_s_reps": t["walls"],
        "stored_bin_updates_per_s": ncell * half * args.steps / wall,
        "roofline": roof,
        "context": "paper: MATLAB plasma code ~20x GPU (GTX 1050) over serial CPU (i7-7700HQ)",
    }
    if not args.quick:
        out["extra"] = {}
        for f in (lambda: extra_c1l(B, W, torch, autotune),
                  lambda: extra_fp64(B, W, torch),
                  lambda: extra_c2(B, W, torch, autotune),
                  lambda: extra_c3(B, W, torch, autotune=autotune),
                  lambda: closure_speedup(B, W, torch),
                  lambda: extra_full(B, W, torch),
                  lambda: extra_3d(B, W, torch),
                  lambda: extra_3d(B, W, torch, kinetic="two_term"),
                  lambda: extra_twoterm(B, W, torch)):
            out["extra"].update(f())
    if not args.no_cpu_baseline:
        log("oracle leg")
        cpu_baseline_leg(out, B, W, autotune, args.quick)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
