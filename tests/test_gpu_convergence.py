"""Order of accuracy of the GPU path itself (section 4's validation: the Yee scheme is
second order), in FP64 storage, through the C ABI.

1D: the section 4 Gaussian plane pulse (tau = 0.5 ns) in vacuum, started from the exact
travelling pulse (E and H written through fdtd_plasma_write_fields), run for 3 ns; its
RMS error against the exact pulse (the paper's normalized global error) must fall with
order 2.0 +- 0.1 as the cell shrinks.

3D: a cavity mode of the PEC cube sin(kx x) sin(ky y) cos(w t) with the continuous w,
started from the exact fields, run for the same physical time at 8^3, 16^3 and 32^3 cells;
the largest error against the continuous mode must fall by 4 (order 2.0 +- 0.1) per
halving of the cell.  Both runs also match the FP64 oracle to 1e-12."""
import math

import numpy as np
import pytest

from oracle.core import Oracle1D, Oracle3D
from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import workloads as W
import analytic as A

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-convergence] {msg}", flush=True)


def test_gaussian_pulse_order_of_accuracy_1d(gpu_lib):
    tau = 0.5e-9
    L, x0, T = 3.0, 1.0, 3.0e-9
    errs, hs = [], []
    for ppw in (10, 20, 40, 80):
        dx = A.C0 * tau / ppw
        nx = int(round(L / dx))
        z = np.zeros(nx + 1)
        run = W.Run1D(name="pulse", nx=nx, nv=8, ne=z, nubar=z, src_node=0, src_amp=0.0,
                      src_f=0.0, src_tau=1.0, src_t0=0.0, steps=0, dx=dx, courant=0.5,
                      bc="pec")
        sim = B.Sim(run, precision=B.FP64)
        dt = 0.5 * dx / A.C0
        nsteps = int(round(T / dt))
        x = np.arange(nx + 1) * dx
        xh = (np.arange(nx) + 0.5) * dx
        pulse = lambda xx, t: np.exp(-((xx - x0 - A.C0 * t) / (A.C0 * tau)) ** 2)
        E0, H0 = pulse(x, 0.0), -pulse(xh, -0.5 * dt) / A.ETA0   # right-going: Hy = -Ez / eta0
        sim.write(B.F_E, E0)
        sim.write(B.F_H, H0)
        assert np.array_equal(sim.read(B.F_E), E0)
        sim.run(nsteps)
        E = sim.read(B.F_E)
        exact = pulse(x, nsteps * dt)
        errs.append(math.sqrt(np.mean((E - exact) ** 2)))
        hs.append(dx)
        if ppw == 20:
            o = Oracle1D(nx, dx, 0.5, z, z, nv=8, bc="pec")
            o.E[:], o.H[:] = E0, H0
            o.run(nsteps)
            assert np.linalg.norm(E - o.E) <= 1e-12 * np.linalg.norm(o.E)
        _banner(f"1D pulse, {ppw} cells per c tau: RMS error {errs[-1]:.3e}")
        sim.close()
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    _banner(f"1D slopes {slopes}")
    assert np.all(np.abs(slopes - 2.0) < 0.1), slopes


def _cavity_fields(n, dx, dt, L):
    kx = ky = math.pi / L
    w = A.C0 * math.sqrt(kx ** 2 + ky ** 2)
    zz, yy, xx = np.meshgrid(np.arange(n) + 0.5, np.arange(n + 1), np.arange(n + 1), indexing="ij")
    ez = np.sin(kx * xx * dx) * np.sin(ky * yy * dx)
    t0 = -0.5 * dt          # H at t = -dt/2 from the continuous Faraday law
    zz, yy, xx = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, np.arange(n + 1), indexing="ij")
    hx = -(ky / (A.MU0 * w)) * np.sin(kx * xx * dx) * np.cos(ky * yy * dx) * math.sin(w * t0)
    zz, yy, xx = np.meshgrid(np.arange(n) + 0.5, np.arange(n + 1), np.arange(n) + 0.5, indexing="ij")
    hy = (kx / (A.MU0 * w)) * np.cos(kx * xx * dx) * np.sin(ky * yy * dx) * math.sin(w * t0)
    return ez, hx, hy, w, kx, ky


def test_cavity_mode_order_of_accuracy_3d(gpu_lib):
    L = 0.016
    errs, hs = [], []
    for n in (8, 16, 32):
        dx = L / n
        z = np.zeros((n, n, n))
        run = W.Run3D(name="cavity", nx=n, ny=n, nz=n, nv=4, ne=z, nubar=z, src_kind=0,
                      src_i=0, src_j=0, src_k=1, steps=0, ncpml=0, dx=dx, src_amp=0.0,
                      src_f=0.0, src_tau=1.0, src_t0=0.0)
        sim = B.Sim(run, precision=B.FP64)
        dt = run.courant * dx / A.C0
        ez, hx, hy, w, kx, ky = _cavity_fields(n, dx, dt, L)
        sim.write(B.F_EZ, ez)
        sim.write(B.F_HX, hx)
        sim.write(B.F_HY, hy)
        steps = 8 * n
        sim.run(steps)
        got = sim.read(B.F_EZ).reshape(ez.shape)
        zz, yy, xx = np.meshgrid(np.arange(n) + 0.5, np.arange(n + 1), np.arange(n + 1), indexing="ij")
        exact = np.sin(kx * xx * dx) * np.sin(ky * yy * dx) * math.cos(w * steps * dt)
        errs.append(float(np.max(np.abs(got - exact))))
        hs.append(dx)
        if n == 16:
            o = Oracle3D(n, n, n, dx, run.courant, z, z, vdim=4, ncpml=0)
            F = o.fields()
            F["Ez"][...], F["Hx"][...], F["Hy"][...] = ez, hx, hy
            o.run(steps)
            ref = o.fields()["Ez"]
            assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
        _banner(f"3D cavity {n}^3: max error {errs[-1]:.3e}")
        sim.close()
    assert errs[0] < 0.1
    slopes = np.diff(np.log(errs)) / np.diff(np.log(hs))
    _banner(f"3D slopes {slopes}")
    assert np.all(np.abs(slopes - 2.0) < 0.1), slopes


def test_write_fields_rejections(gpu_lib):
    """Only E and H can be written, with exactly the field's length and finite values;
    a rejected write leaves the state untouched."""
    run = W.c0()
    sim = B.Sim(run, precision=B.FP64)
    sim.run(10)
    before = sim.read(B.F_E)
    with pytest.raises(B.FdtdError) as ei:
        sim.write(B.F_J, np.zeros(run.nx + 1))
    assert ei.value.code == B.EINVAL
    with pytest.raises(B.FdtdError) as ei:
        sim.write(B.F_E, np.zeros(run.nx))
    assert ei.value.code == B.ERANGE
    bad = np.zeros(run.nx + 1)
    bad[3] = np.nan
    with pytest.raises(B.FdtdError) as ei:
        sim.write(B.F_E, bad)
    assert ei.value.code == B.EINVAL
    assert np.array_equal(sim.read(B.F_E), before)
    sim.close()
