"""The 4096 x 4096 blob workload with the trained closure, at full size in the launch shape
the benchmark times, checked on sampled cells one by one: the field history each sampled
closure cell saw (probes on its four edges) and its current before the step go through the
oracle's closure (network in FP64 with bf16 operand emulation); the result must match the
current the GPU produced."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle.core import mlp as cmlp
from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import closure as CL
from paper_2211_05647_amd import workloads as W
import analytic as A

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-c4] {msg}", flush=True)


def test_c4_full_size_sampled_closure_cells(gpu_lib):
    import torch
    data, c = CL.gather_data(log=_banner)
    params, _ = CL.fit(data, c, log=lambda m: None)
    blob = CL.make_blob(params, data.box, data.dt)
    run = W.c4(extra_hot=4)
    dt = run.courant * run.dx / A.C0
    # sampled closure cells: inside the box, nearest the source (reached first)
    jj, ii = np.nonzero(run.ne > 0)
    wp_dt = np.sqrt(A.plasma_omega2(run.ne[jj, ii])) * dt
    q1, q2 = M.scale_params(wp_dt, run.nubar[jj, ii] * dt, data.box)
    inside = (q1 >= -1) & (q1 <= 1) & (q2 >= -1) & (q2 <= 1)
    order = np.argsort(ii + 1e-6 * jj)
    picks = [k for k in order if inside[k]][:4]
    # the plane pulse peaks at the source near t0 (4.5 tau = 348 steps) and moves half a
    # cell per step: check while it crosses the sampled column
    i0 = int(ii[picks[0]])
    nsteps = int(4.5 * run.src_tau / dt) + 2 * (i0 - run.src_i) + 20
    _banner(f"c4 {run.nx}x{run.ny}, plasma cells {run.plasma_cells}, samples at "
            f"{[(int(ii[k]), int(jj[k])) for k in picks]}")
    sim = B.Sim(run, closure=B.CLOSURE_MLP, mlp_blob=blob, max_probes=16, probe_capacity=nsteps + 1)
    pids = []
    for k in picks:
        i, j = int(ii[k]), int(jj[k])
        pids.append((sim.add_probe(B.F_EX, i, j), sim.add_probe(B.F_EX, i, j + 1),
                     sim.add_probe(B.F_EY, i, j), sim.add_probe(B.F_EY, i + 1, j)))
    sim.run(nsteps)
    jx0, jy0 = sim.read(B.F_JCX), sim.read(B.F_JCY)
    sim.step()
    jx1, jy1 = sim.read(B.F_JCX), sim.read(B.F_JCY)
    assert np.all(np.isfinite(jx1))
    w, s = A.velocity_weights(32, 6.0, 5.0, "hard_sphere", dims=2)
    norm = dt / A.EPS0
    checked = 0
    for k, (a, b, cc, d) in zip(picks, pids):
        i, j = int(ii[k]), int(jj[k])
        ex = 0.5 * (sim.read_probe(a, nsteps + 1) + sim.read_probe(b, nsteps + 1))
        ey = 0.5 * (sim.read_probe(cc, nsteps + 1) + sim.read_probe(d, nsteps + 1))
        # E^n for n = nsteps is the probe sample after step nsteps - 1
        hx = ex[nsteps - 1::-1][:16]
        hy = ey[nsteps - 1::-1][:16]
        _banner(f"cell ({i},{j}): max |E| over the window {max(np.max(np.abs(hx)), np.max(np.abs(hy))):.3e}")
        if max(np.max(np.abs(hx)), np.max(np.abs(hy))) < 1e-4:
            continue
        ne, nu = run.ne[j, i], run.nubar[j, i]
        al, be = M.effective_pole(w, s, nu, A.plasma_omega2(ne), dt)
        qa, qb = M.scale_params(math.sqrt(A.plasma_omega2(ne)) * dt, nu * dt, data.box)
        for h, j0, j1 in ((hx, jx0, jx1), (hy, jy0, jy1)):
            sc = max(np.max(np.abs(h)), 1e-30)
            x = np.concatenate([h / sc, [qa, qb]])
            y = cmlp(params.astype(np.float64), x, True)
            want = al * j0[j * run.nx + i] * norm + be * (h[0] + sc * y)
            got = j1[j * run.nx + i] * norm
            _banner(f"cell ({i},{j}): J^(n+1/2) gpu {got:.6e} oracle {want:.6e}")
            assert abs(got - want) <= 1e-3 * max(abs(want), 1e-3 * be * sc)
        checked += 1
    assert checked >= 2
