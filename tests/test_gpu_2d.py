"""GPU parity of the 2D TEz path (CPML + 2V kinetic) against the FP64 oracle through
the C ABI.  FP64 storage <= 1e-12 relative L2; FP32 storage <= 1e-5 relative L2 over
space and time."""
import math

import numpy as np
import pytest

from oracle.core import Oracle2D
from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import workloads as W
from parity import rel_l2

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-2d] {msg}", flush=True)


def oracle_2d(run):
    return Oracle2D(run.nx, run.ny, run.dx, run.courant, run.ne, run.nubar, nv=run.nv,
                    vmax_over_vth=run.vmax_over_vth, te_ev=run.te_ev, nu_model=run.nu_model,
                    ncpml=run.ncpml, src_kind=run.src_kind, src_i=run.src_i, src_j=run.src_j,
                    src_amp=run.src_amp, src_f=run.src_f, src_tau=run.src_tau,
                    src_t0=run.src_t0)


def small_run(nx=70, ny=54, nv=16, ncpml=8, src_kind=2, nu_model="hard_sphere", steps=400):
    jj, ii = np.mgrid[0:ny, 0:nx]
    blob = (ii + 0.5 - 42) ** 2 + (jj + 0.5 - 27) ** 2 < 14 ** 2
    ne = np.where(blob, W.density_from_ratio(1.2, W.F_REF), 0.0)
    nu = np.where(blob, 0.1 * 2 * math.pi * W.F_REF, 0.0)
    return W.Run2D(name="blob", nx=nx, ny=ny, nv=nv, ne=ne, nubar=nu, src_kind=src_kind,
                   src_i=20, src_j=ny // 2, steps=steps, ncpml=ncpml, nu_model=nu_model,
                   **W.pulse(W.F_REF))


def space_time_2d(sim, orc, nsteps, every):
    g, o = [], []
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        sim.run(k)
        orc.run(k)
        done += k
        g.append(np.concatenate([sim.read(B.F_EX), sim.read(B.F_EY)]))
        o.append(np.concatenate([orc.Ex.ravel(), orc.Ey.ravel()]))
    return np.array(g), np.array(o)


@pytest.mark.parametrize("nv", [8, 16, 32])
def test_small_2d_fp64_parity(gpu_lib, nv):
    run = small_run(nv=nv)
    _banner(f"small fp64 nv={nv}")
    sim = B.Sim(run, precision=B.FP64)
    orc = oracle_2d(run)
    g, o = space_time_2d(sim, orc, run.steps, 100)
    assert rel_l2(g, o) <= 1e-12
    assert rel_l2(sim.read(B.F_HZ), orc.Hz.ravel()) <= 1e-12
    assert rel_l2(sim.read(B.F_JX), orc.Jx.ravel()) <= 1e-12
    assert rel_l2(sim.read(B.F_JY), orc.Jy.ravel()) <= 1e-12
    assert rel_l2(sim.read(B.F_DF), orc.df) <= 1e-12


@pytest.mark.parametrize("nv,cpb", [(8, 3), (16, 7), (32, 16), (32, 64)])
def test_small_2d_fp32_parity(gpu_lib, nv, cpb):
    for model, src in (("hard_sphere", 2), ("const", 1)):
        run = small_run(nv=nv, nu_model=model, src_kind=src)
        _banner(f"small fp32 nv={nv} cells/group={cpb} {model}")
        sim = B.Sim(run, precision=B.FP32, cells_per_group=cpb)
        orc = oracle_2d(run)
        g, o = space_time_2d(sim, orc, run.steps, 50)
        assert rel_l2(g, o) <= 1e-5
        assert rel_l2(sim.read(B.F_DF), orc.df) <= 1e-5


def test_pec_box_no_plasma(gpu_lib):
    run = small_run(ncpml=0)
    run.ne[:] = 0.0
    _banner("pec box")
    sim = B.Sim(run, precision=B.FP64)
    orc = oracle_2d(run)
    g, o = space_time_2d(sim, orc, 300, 100)
    assert rel_l2(g, o) <= 1e-12
    assert sim.read(B.F_DF).size == 0


def test_c2_full_size_parity(gpu_lib):
    """The 2D workload at its full size (512x512, 32x32 velocity bins, plasma column of
    31,428 cells, CPML 8, Ey line source) in FP32 for 700 steps, by which time the pulse
    is crossing the column."""
    run = W.c2()
    steps = 700
    _banner("c2 full size")
    sim = B.Sim(run, precision=B.FP32, max_probes=3, probe_capacity=steps)
    pids = [sim.add_probe(B.F_EY, i, 256) for i in (100, 256, 400)]
    orc = oracle_2d(run)
    pr = []
    g, o = [], []
    done = 0
    while done < steps:
        sim.run(100)
        pr.append(orc.run(100, probes=[(100, 256), (256, 256), (400, 256)]))
        done += 100
        g.append(sim.read(B.F_EY))
        o.append(orc.Ey.ravel().copy())
    err = rel_l2(np.array(g), np.array(o))
    gp = np.stack([sim.read_probe(p, steps) for p in pids], axis=1)
    perr = rel_l2(gp, np.concatenate(pr))
    _banner(f"c2 Ey space-time rel L2 = {err:.3e}, probes {perr:.3e}")
    assert err <= 1e-5 and perr <= 1e-5
    assert rel_l2(sim.read(B.F_DF), orc.df) <= 1e-5
    assert rel_l2(sim.read(B.F_JY), orc.Jy.ravel()) <= 1e-5


def test_2d_resume_bitwise(gpu_lib):
    run = small_run()
    _banner("2d resume")
    a = B.Sim(run)
    a.run(150)
    blob = a.save_state()
    a.run(150)
    c = B.Sim(run)
    c.load_state(blob)
    c.run(150)
    for f in (B.F_EX, B.F_EY, B.F_HZ, B.F_JX, B.F_DF):
        assert np.array_equal(a.read(f), c.read(f))


def test_large_grid_fp32_parity(gpu_lib):
    """A grid large enough for the field updates' four-rows-per-thread form (the FP32 path
    of the large workloads): 2048 x 2050 cells with the CPML on every side, a plasma blob
    and a point source, for 300 steps.  Ex and Ey over space and time, Hz at the end, and
    probes next to the source, next to the PEC edges and inside the absorbing strips,
    against the FP64 oracle."""
    nx, ny = 2048, 2050
    jj, ii = np.mgrid[0:ny, 0:nx]
    blob = (ii + 0.5 - 150) ** 2 + (jj + 0.5 - 1030) ** 2 < 20 ** 2
    ne = np.where(blob, W.density_from_ratio(1.2, W.F_REF), 0.0)
    nu = np.where(blob, 0.1 * 2 * math.pi * W.F_REF, 0.0)
    run = W.Run2D(name="large", nx=nx, ny=ny, nv=8, ne=ne, nubar=nu, src_kind=2,
                  src_i=61, src_j=1025, steps=300, ncpml=8, **W.pulse(W.F_REF))
    steps = 300
    where = [(B.F_EY, 60, 1025), (B.F_EY, 61, 1020), (B.F_EY, 62, 1030), (B.F_EY, 63, 1025),
             (B.F_EY, 1, 1025), (B.F_EY, nx - 1, 1025), (B.F_EY, 4, 900), (B.F_EX, 0, 1025),
             (B.F_EX, nx - 1, 1025), (B.F_EX, 150, 1030)]
    _banner(f"large grid fp32 {nx}x{ny}")
    sim = B.Sim(run, precision=B.FP32, max_probes=len(where), probe_capacity=steps)
    pids = [sim.add_probe(f, i, j) for f, i, j in where]
    orc = oracle_2d(run)
    opts = [(i, j) for f, i, j in where]
    g, o, oprobe = [], [], []
    done = 0
    while done < steps:
        sim.run(100)
        done += 100
        # the oracle's probes record Ey; Ex probes are compared through the snapshots
        oprobe.append(orc.run(100, probes=opts))
        g.append(np.concatenate([sim.read(B.F_EX), sim.read(B.F_EY)]))
        o.append(np.concatenate([orc.Ex.ravel(), orc.Ey.ravel()]))
    err = rel_l2(np.array(g), np.array(o))
    gp = np.stack([sim.read_probe(p, steps) for p, (f, _, _) in zip(pids, where) if f == B.F_EY], axis=1)
    op = np.concatenate(oprobe)[:, [k for k, (f, _, _) in enumerate(where) if f == B.F_EY]]
    perr = rel_l2(gp, op)
    _banner(f"large grid: Ex, Ey space-time rel L2 {err:.3e}, Ey probes {perr:.3e}")
    assert err <= 1e-5 and perr <= 1e-5
    assert rel_l2(sim.read(B.F_HZ), orc.Hz.ravel()) <= 1e-5
    assert np.max(np.abs(sim.read(B.F_DF))) > 0.0
