#!/usr/bin/env python3
"""Throughput of the kinetic-FDTD step on one MI355X.

One benchmark step is one leap-frog time step of the whole coupled path (H update,
F1 update driven by E, FP64 current moment, E update with -J, Mur ends, soft source) on
the large 1D workload: Nx = 65536 cells, Nv = 512 velocity bins, plasma over nodes
[400, Nx-100) with a smoothed random density (omega_p/omega in [0.2, 2]) and
log-uniform collision rates, FP32 storage with FP64 moments.  Inputs are synthetic and
seeded.  The metric counts phase-space updates (plasma cell x signed velocity bin x
step) per second.

Prints one JSON line.  The other workloads (Nx = 2^20 line, the 2D column, the batch of
256 runs) are timed too and reported under "extra" unless --quick is given.
``--calibrate-copy`` only runs a plain device copy of known size (the reference kernel
for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE).  ``--gpus N`` with N > 1 exits: this
path runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
# Vector ALU roofline of the temporally blocked kernel: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops (FMA) x 2.4 GHz, single-issue FP32 (this build does not emit packed FP32,
# which the 157.3 TFLOP/s published figure assumes).
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Arithmetic of one stored-bin update of F1 and its moment: FP32 dt*nu (mul), 2 + x (add),
# reciprocal, 2x (add), drive (mul), two FMAs (4 flops); FP64 moment FMA (2 flops).
# arithmetic of one stored-bin update in the blocked kernel: per step two FP32 FMAs
# (F1 + c n E, then + d F1: 4) and the FP64 moment FMA (2); once per launch the
# Crank-Nicolson coefficients d = -2x / (2 + x) and c = b / (2 + x) (an FMA and a
# reciprocal for 1 / (2 + x), two products for d, one for c: 6)
FLOPS_PER_BIN_STEP = 6
FLOPS_PER_BIN_LAUNCH = 6


def kernel_hash(blocked=True):
    """Hash of the sources the kernel is built from (the blocked kernel: its own file and
    the shared header; the one-step kernel likewise)."""
    h = hashlib.sha256()
    for f in ("common.h", "kernels1d_tb.hip" if blocked else "kernels1d.hip"):
        h.update(open(os.path.join(ROOT, "paper_2211_05647_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def pmc_traffic(kb=1):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the kernel as it is now (else None)."""
    name = "k_step1d_tb_c1_pmc.json" if kb > 1 else "k_step1d_c1_pmc.json"
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_hash") != kernel_hash(blocked=kb > 1):
        return None
    return d.get("hbm_bytes_per_launch")


def bytes_1d(run):
    """Algorithmic bytes of one launch of the 1D step kernel: F1 read + write (half grid,
    FP32), per-cell scalars (node index, dt*nu, density), fields (E and H read and
    written, J written) over the whole line."""
    ncell, half, nx = run.plasma_cells, run.nv // 2, run.nx
    return ncell * half * 4 * 2 + ncell * 12 + (nx + 1) * 4 * 5


def bytes_2d(run):
    """Algorithmic bytes of one 2D step (both launches): F1 read + write, per-cell
    scalars and E gather, Ex/Ey/Hz read + written, cell currents written and read."""
    ncell, half, nx, ny = run.plasma_cells, run.nv * run.nv // 2, run.nx, run.ny
    npt = nx * ny
    return ncell * half * 4 * 2 + ncell * (12 + 16 + 8) + npt * 4 * (6 + 4)


def cpu_baseline(run, budget_s=15.0):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload:
    the full line (all plasma cells, full signed grid) for as many steps as fit the
    time budget.  Returns phase-space updates/s."""
    sys.path.insert(0, ROOT)
    from oracle.core import Oracle1D, threads
    o = Oracle1D(run.nx, run.dx, run.courant, run.ne, run.nubar, nv=run.nv,
                 vmax_over_vth=run.vmax_over_vth, te_ev=run.te_ev, nu_model=run.nu_model,
                 bc=run.bc, src_node=run.src_node, src_amp=run.src_amp, src_f=run.src_f,
                 src_tau=run.src_tau, src_t0=run.src_t0)
    t0 = time.perf_counter()
    o.run(2)
    per = (time.perf_counter() - t0) / 2
    n = max(2, int(budget_s / max(per, 1e-6)))
    t0 = time.perf_counter()
    o.run(n)
    t = time.perf_counter() - t0
    ups = run.plasma_cells * run.nv * n / t
    return dict(value=ups, unit="phase-space updates/s", cores=threads(), kind="oracle",
                sample=f"large 1D workload, full line (Nx={run.nx}, Nv={run.nv}), {n} steps "
                       f"from the zero state, FP64 on the full signed grid, {t:.1f} s")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_single(run, B, torch, steps, warmup, tile=0, info=None, time_block=0):
    sim = B.Sim(run, precision=B.FP32, tile=tile, time_block=time_block or None)
    sim.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sim.last_run_ms()
    if hasattr(run, "ny"):
        sim.read(B.F_EY)
    else:
        sim.read(B.F_E)
        if info is not None:
            info["time_block"], info["rows_per_launch"] = sim.time_block(rows=True)
    sim.close()
    return wall, ms


def bytes_1d_blocked(run, rows):
    """Algorithmic bytes of one launch of the temporally blocked kernel (K steps): the F1
    rows it reads (owned + halo) with their per-cell scalars, the owned rows written
    back, the fields read and written once per launch."""
    half, nx = run.nv // 2, run.nx
    return rows * (half * 4 + 12) + run.plasma_cells * half * 4 + (nx + 1) * 4 * 5


def extra_c1l(B, W, torch, autotune):
    """1D line with Nx = 2^20: F1 (1.07 GB) far above every cache."""
    run = W.c1_large()
    log(f"c1l: Nx={run.nx} plasma cells={run.plasma_cells}")
    tile = autotune.lookup(run, B.FP32) or autotune.lookup(W.c1(nx=4096, steps=1), B.FP32)
    info = {}
    wall, ms = time_single(run, B, torch, run.steps, 50, tile, info,
                           autotune.lookup_time_block(run, B.FP32))
    kb = info.get("time_block", 1)
    by = bytes_1d_blocked(run, info["rows_per_launch"]) / kb if kb > 1 else bytes_1d(run)
    return {"c1_nx2e20": dict(workload="1D Yee + 1V kinetic, Nx=1048576, Nv=512, FP32, 2000 steps",
                              updates_per_s=run.plasma_cells * run.nv * run.steps / wall,
                              ms_per_step=wall / run.steps * 1e3, kernel_ms_per_step=ms,
                              steps_per_launch=kb,
                              hbm_gbs=by / (ms * 1e-3) / 1e9,
                              hbm_frac=by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              one_step_stream_equivalent_gbs=bytes_1d(run) / (ms * 1e-3) / 1e9)}


def bytes_1d_full(run):
    """Algorithmic bytes of one launch of the full-model step kernel: the node's whole
    row (odd and even halves of f - n fhat, Nv values, FP32) read + written, per-cell
    scalars, fields over the line."""
    ncell, nv, nx = run.plasma_cells, run.nv, run.nx
    return ncell * nv * 4 * 2 + ncell * 12 + (nx + 1) * 4 * 5


def extra_full(B, W, torch, steps=None):
    """The full-distribution model (F0 evolves, electrons heat) on the C1 line and on the
    Nx = 2^20 line, FP32: K steps per launch (9 and 7, the measured best: 23.7 us against
    24.3 at 7 and 38.5 at 1 on the C1 line, 311 us against 327 at 9 and 777 at 1 on 2^20),
    and one step per launch beside it (2000 and 300 steps, or ``steps``)."""
    out = {}
    for key, run, steps, kb in (("full_c1", W.c1(steps=2000), steps or 2000, 9),
                                ("full_c1_nx2e20", W.c1_large(), steps or 300, 7)):
        run.kinetic = "full"
        log(f"{key}: Nx={run.nx} Nv={run.nv} plasma cells={run.plasma_cells}")
        info = {}
        wall, ms = time_single(run, B, torch, steps, 6 * kb, 0, info, kb)
        kb, rows = info["time_block"], info["rows_per_launch"]
        wall1, ms1 = time_single(run, B, torch, steps, 50, 0, None, 1)
        by1 = bytes_1d_full(run)
        # K steps per launch: rows read (owned + halo) with their scalars, owned rows
        # written, fields once
        byk = rows * (run.nv * 4 + 12) + run.plasma_cells * run.nv * 4 + (run.nx + 1) * 4 * 5
        by = byk / kb if kb > 1 else by1
        out[key] = dict(workload=f"1D Yee + full-distribution 1V kinetic, Nx={run.nx}, "
                                 f"Nv={run.nv}, FP32, {steps} steps",
                        kernel=f"k_step1d_tb_full<{kb}, 64>" if kb > 1 else "k_step1d_full<float>",
                        steps_per_launch=kb,
                        updates_per_s=run.plasma_cells * run.nv * steps / wall,
                        ms_per_step=wall / steps * 1e3, kernel_ms_per_step=ms,
                        hbm_gbs=by / (ms * 1e-3) / 1e9,
                        hbm_frac=by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        one_step_stream_equivalent_gbs=by1 / (ms * 1e-3) / 1e9,
                        one_step_per_launch=dict(kernel="k_step1d_full<float>",
                                                 ms_per_step=wall1 / steps * 1e3,
                                                 kernel_ms_per_step=ms1,
                                                 hbm_gbs=by1 / (ms1 * 1e-3) / 1e9,
                                                 hbm_frac=by1 / (ms1 * 1e-3) / 1e9 / HBM_PEAK_GBS))
    # the FP64 oracle's full-distribution model on the host, same Nx = 65536 line
    sys.path.insert(0, ROOT)
    from oracle.core import Oracle1D, threads
    run = W.c1(steps=1)
    o = Oracle1D(run.nx, run.dx, run.courant, run.ne, run.nubar, nv=run.nv, te_ev=run.te_ev,
                 src_node=run.src_node, src_amp=run.src_amp, src_f=run.src_f,
                 src_tau=run.src_tau, src_t0=run.src_t0, kinetic="full")
    t0 = time.perf_counter()
    o.run(20)
    per = (time.perf_counter() - t0) / 20
    k = max(20, int(5.0 / per))
    t0 = time.perf_counter()
    o.run(k)
    dt = time.perf_counter() - t0
    out["full_c1"]["cpu_oracle"] = dict(kind="oracle", cores=threads(),
                                        updates_per_s=run.plasma_cells * run.nv * k / dt,
                                        sample=f"Nx=65536 line, {k} steps after 20, FP64 full grid")
    return out


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


def extra_3d(B, W, torch, steps=300, kinetic="linear"):
    """The paper's production model in 3D: the argon-style slab (Druyvesteyn F0, v_dim = 31
    speeds, a 4 mm slab along z, sheet source, CPML on all faces) at 128 x 128 x 512, with
    F0 held (linear) or evolving in every plasma cell (two_term; its slab ends where the x
    and y absorbing layers begin, which that model needs to stay stable)."""
    tt = kinetic == "two_term"
    run = W.argon_slab_3d(nx=128, ny=128, nz=512, steps=steps, kinetic=kinetic)
    sim = B.Sim(run, precision=B.FP32)
    npoints = sim.closure_counts()[1]
    ncells = run.plasma_cells if tt else 0
    key = "argon3d_two_term" if tt else "argon3d"
    log(f"{key}: {run.nx}x{run.ny}x{run.nz}, plasma points {npoints}, cells {ncells}")
    sim.run(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sim.last_run_ms()
    sim.read(B.F_EX)
    sim.close()
    row = 32
    by = bytes_3d_tt(run, npoints, ncells, row) if tt else bytes_3d(run, npoints, row)
    cells = run.nx * run.ny * run.nz
    # the FP64 oracle on the host, same workload, a few steps
    sys.path.insert(0, ROOT)
    from oracle.core import Oracle3D, threads
    o = Oracle3D(run.nx, run.ny, run.nz, run.dx, run.courant, run.ne, run.nubar, vdim=run.nv,
                 vmax_over_vth=run.vmax_over_vth, te_ev=run.te_ev, nu_model=run.nu_model,
                 f0_model=run.f0_model, ncpml=run.ncpml, src_kind=run.src_kind,
                 src_k=run.src_k, src_amp=run.src_amp, src_f=run.src_f, src_tau=run.src_tau,
                 src_t0=run.src_t0, kinetic=kinetic)
    o.run(1)
    t0 = time.perf_counter()
    o.run(4)
    cdt = (time.perf_counter() - t0) / 4
    cpu = dict(kind="oracle", cores=threads(), nmcps=cells / cdt * 1e-6,
               updates_per_s=npoints * run.nv / cdt, sample="4 steps after 1, FP64")
    model = "two-term F1 + evolving F0" if tt else "speed-grid F1"
    return {key: dict(cpu_oracle=cpu, workload=f"3D Yee + CPML + {model} (v_dim {run.nv}, Druyvesteyn), "
                                     f"{run.nx}x{run.ny}x{run.nz}, FP32, {steps} steps",
                            plasma_points=npoints, plasma_cells=ncells, cells=cells,
                            updates_per_s=npoints * run.nv * steps / wall,
                            nmcps=cells * steps / wall * 1e-6,
                            ms_per_step=wall / steps * 1e3, kernel_ms_per_step=ms,
                            hbm_gbs=by / (ms * 1e-3) / 1e9,
                            hbm_frac=by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)}


def sweep_3d(B, W, torch, cpu_budget_s=2.0):
    """NMCPS (eq. (5)) of the 3D vacuum cube (CPML on all faces, sheet source) from 16^3
    to 384^3 on the GPU (FP32), and on the host with the FP64 oracle up to 96^3."""
    sys.path.insert(0, ROOT)
    from oracle.core import Oracle3D, threads
    out = []
    for n in (16, 32, 64, 128, 192, 256, 384):
        z = np.zeros((n, n, n))
        run = W.Run3D(name=f"vac3d{n}", nx=n, ny=n, nz=n, nv=1, ne=z, nubar=z, src_kind=1,
                      src_i=0, src_j=0, src_k=n // 4, steps=0, ncpml=min(8, n // 4),
                      **W.pulse(W.F_REF))
        steps = max(60, min(2000, int(2e9 / n ** 3)))
        sim = B.Sim(run, precision=B.FP32)
        sim.run(10)
        sim.run(steps)
        ms = sim.last_run_ms()
        sim.close()
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


def extra_twoterm(B, W, torch, steps=2000):
    """The two-term model on the speed grid (F1 and an evolving F0, v_dim = 31, Druyvesteyn
    F0 at 1 eV) on the large line's density and collision profile, FP32: K steps per launch
    (the default), and one step per launch beside it; the FP64 oracle timed beside them on
    the same line."""
    run = W.c1(steps=steps)
    run.kinetic, run.nv, run.f0_model = "two_term", 31, "druyvesteyn"
    run.te_ev, run.vmax_over_vth = 1.0, 5.0
    log(f"two-term: Nx={run.nx} v_dim={run.nv} plasma cells={run.plasma_cells}")
    info = {}
    # 9 steps per launch (measured: 3.25 us per step at 9, 3.49 at 7, 3.82 at 5, 7.62 at 1)
    wall, ms = time_single(run, B, torch, steps, 54, 0, info, 9)
    kb, rows = info["time_block"], info["rows_per_launch"]
    wall1, ms1 = time_single(run, B, torch, steps, 50, 0, None, 1)
    row = 32
    # one step per launch: rows [F1 | F0] read and written, per-cell scalars, fields
    by1 = run.plasma_cells * (2 * row * 4 * 2 + 12 + 4) + (run.nx + 1) * 4 * 5
    # K steps per launch: rows read (owned + halo) with their scalars, owned rows written,
    # fields once
    byk = rows * (2 * row * 4 + 12) + run.plasma_cells * 2 * row * 4 + (run.nx + 1) * 4 * 5
    by = byk / kb if kb > 1 else by1
    out = dict(workload=f"1D Yee + two-term speed-grid kinetic (F0 evolving), Nx={run.nx}, "
                        f"v_dim={run.nv}, FP32, {steps} steps",
               kernel=f"k_step1d_tb_tt<{kb}, 8>" if kb > 1 else "k_step1d_tt<float>",
               steps_per_launch=kb,
               updates_per_s=run.plasma_cells * run.nv * steps / wall,
               ms_per_step=wall / steps * 1e3, kernel_ms_per_step=ms,
               hbm_gbs=by / (ms * 1e-3) / 1e9, hbm_frac=by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               one_step_stream_equivalent_gbs=by1 / (ms * 1e-3) / 1e9,
               one_step_per_launch=dict(kernel="k_step1d_tt<float>",
                                        ms_per_step=wall1 / steps * 1e3, kernel_ms_per_step=ms1,
                                        hbm_gbs=by1 / (ms1 * 1e-3) / 1e9,
                                        hbm_frac=by1 / (ms1 * 1e-3) / 1e9 / HBM_PEAK_GBS))
    sys.path.insert(0, ROOT)
    from oracle.core import Oracle1D, threads
    o = Oracle1D(run.nx, run.dx, run.courant, run.ne, run.nubar, nv=run.nv,
                 vmax_over_vth=run.vmax_over_vth, te_ev=run.te_ev, src_node=run.src_node,
                 src_amp=run.src_amp, src_f=run.src_f, src_tau=run.src_tau,
                 src_t0=run.src_t0, kinetic="two_term", f0_model=run.f0_model)
    t0 = time.perf_counter()
    o.run(20)
    per = (time.perf_counter() - t0) / 20
    k = max(20, int(5.0 / per))
    t0 = time.perf_counter()
    o.run(k)
    dt = time.perf_counter() - t0
    out["cpu_oracle"] = dict(kind="oracle", cores=threads(),
                             updates_per_s=run.plasma_cells * run.nv * k / dt,
                             sample=f"same line, {k} steps after 20, FP64")
    return {"two_term_c1": out}


def extra_c2(B, W, torch, autotune, steps=None):
    """2D column, 512^2, 32x32 velocity bins."""
    run = W.c2()
    steps = steps or run.steps
    log(f"c2: {run.nx}x{run.ny} plasma cells={run.plasma_cells}")
    tile = autotune.lookup(run, B.FP32)
    wall, ms = time_single(run, B, torch, steps, 100, tile)
    by = bytes_2d(run)
    return {"c2": dict(workload=f"2D TEz 512x512 + 2V kinetic 32x32, FP32, {steps} steps",
                       updates_per_s=run.plasma_cells * run.nv ** 2 * steps / wall,
                       ms_per_step=wall / steps * 1e3, step_ms=ms,
                       hbm_gbs=by / (ms * 1e-3) / 1e9,
                       hbm_frac=by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)}


def extra_c3(B, W, torch):
    """Batch of 256 uneven 1D runs."""
    runs = W.c3()
    work = sum(r.plasma_cells * r.nv * r.steps for r in runs)
    by = sum(bytes_1d(r) * r.steps for r in runs)
    tot = max(r.steps for r in runs)
    log(f"c3: {len(runs)} runs, {tot} steps max")
    sim = B.Sim(runs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(tot)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    return {"c3": dict(workload="256 independent 1D runs, Nx in [500, 20000], Nv in {64,128,256}, "
                                "2 Nx steps each",
                       updates_per_s=work / wall, seconds=wall, hbm_gbs=by / wall / 1e9,
                       hbm_frac=by / wall / 1e9 / HBM_PEAK_GBS)}


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
        sim = B.Sim(run, precision=B.FP32, **kw)
        sim.run(steps)
        torch.cuda.synchronize()
        res[name + "_ms_per_step"] = sim.last_run_ms()
        by = bytes_2d(run)
        if name == "kinetic":
            res["kinetic_hbm_frac"] = by / (res["kinetic_ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS
        sim.close()
        torch.cuda.empty_cache()
    return {"c4_steps": res}


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
        sim = B.Sim(run, precision=B.FP32)
        sim.run(20)
        sim.run(steps)
        ms = sim.last_run_ms()
        sim.close()
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


def extra_workloads(B, W, torch, autotune):
    out = {}
    out.update(extra_c1l(B, W, torch, autotune))
    out.update(extra_c2(B, W, torch, autotune))
    out.update(extra_c3(B, W, torch))
    out.update(closure_speedup(B, W, torch))
    out.update(extra_full(B, W, torch))
    out.update(extra_3d(B, W, torch))
    out.update(extra_3d(B, W, torch, kinetic="two_term"))
    out.update(extra_twoterm(B, W, torch))
    return out


def closure_speedup(B, W, torch, steps=50):
    """4096^2 blob workload: time per step with every plasma cell on the kinetic F1 step,
    and with the trained closure (cells outside the training box stay kinetic).  The
    closure is trained first on the batch workload's taps (timed separately)."""
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
        sim = B.Sim(run, precision=B.FP32, **kw)
        sim.run(5)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.run(steps)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t) / steps
        res[name + "_event"] = sim.last_run_ms() * 1e-3
        if name == "closure":
            res["closure_cells"], res["fallback_cells"] = sim.closure_counts()
        sim.close()
        torch.cuda.empty_cache()
    rows = 2 * res["closure_cells"]
    flops = rows * 2 * (18 * 128 + 128 * 128 + 128)
    return {"c4_closure": dict(
        workload="2D TEz 4096x4096, 48 plasma blobs, 32x32 bins; learned closure vs kinetic",
        kinetic_ms_per_step=res["kinetic"] * 1e3, closure_ms_per_step=res["closure"] * 1e3,
        speedup=res["kinetic"] / res["closure"], closure_cells=res["closure_cells"],
        fallback_cells=res["fallback_cells"],
        network_tflops_lower_bound=flops / res["closure"] / 1e12,
        network_frac_of_bf16_peak_lower_bound=flops / res["closure"] / 2.5e15,
        training=dict(gather_s=t1 - t0, fit_s=t2 - t1, held_out_mse=net, held_out_mse_without_net=zero))}


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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="only the headline workload")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--time-block", type=int, default=0,
                    help="steps per launch of the large 1D workload (default: tuned; 1 = one "
                         "step per launch)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--only", choices=["c1l", "c2", "c3", "closure", "c4", "sweep", "full", "3d", "sweep3d",
                             "twoterm", "3dtt"], default=None,
                    help="run only one of the extra measurements (for profiling); c2 and c4 "
                         "take --steps steps")
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
                "c3": lambda: extra_c3(B, W, torch),
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
    log(f"tile={tile or 'default'}")
    info = {}
    wall, ms_dev = time_single(run, B, torch, args.steps, args.warmup, tile, info,
                               args.time_block or autotune.lookup_time_block(run, B.FP32))

    ncell, nv, half, nx = run.plasma_cells, run.nv, run.nv // 2, run.nx
    value = ncell * nv * args.steps / wall
    kb = info.get("time_block", 1)
    if kb > 1:
        # one launch = kb steps of the temporally blocked kernel, which is bound by vector
        # ALU issue: priced by the arithmetic of the F1 update and its FP64 moment
        kernel = f"k_step1d_tb<{kb}, {half // 4}>"
        bytes_alg = bytes_1d_blocked(run, info["rows_per_launch"])
        launch_ms = ms_dev * kb
        flops = (FLOPS_PER_BIN_STEP * kb + FLOPS_PER_BIN_LAUNCH) * ncell * half
        roof = {"bound": "alu", "kernel": kernel,
                "achieved": flops / (launch_ms * 1e-3) / 1e12, "peak": VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": flops / (launch_ms * 1e-3) / 1e12 / VALU_PEAK_TFLOPS,
                "traffic": pmc_traffic(kb), "flops_per_launch": flops,
                "hbm_bytes_per_launch": bytes_alg,
                "hbm_gbs": bytes_alg / (launch_ms * 1e-3) / 1e9, "launch_ms": launch_ms,
                "one_step_stream_equivalent_gbs": bytes_1d(run) / (ms_dev * 1e-3) / 1e9}
    else:
        kernel = "k_step1d<float>"
        bytes_alg = bytes_1d(run)
        launch_ms = ms_dev
        achieved = bytes_alg / (launch_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": pmc_traffic(kb),
                "bytes_per_launch": bytes_alg, "launch_ms": launch_ms}
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
        "stored_bin_updates_per_s": ncell * half * args.steps / wall,
        "roofline": roof,
        "context": "paper: MATLAB plasma code ~20x GPU (GTX 1050) over serial CPU (i7-7700HQ)",
    }
    if not args.quick:
        out["extra"] = extra_workloads(B, W, torch, autotune)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(run)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
