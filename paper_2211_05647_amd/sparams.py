"""Scattering parameters of a plasma slab (the paper's S11 and S21, section 5.3 results):
E recorded on the device at two ports, before and after the slab, in the slab run and in
the same run with the plasma removed; S11 = spectrum of the reflected part at port 1 over
the incident spectrum there, S21 = transmitted spectrum at port 2 over the vacuum run's.
The time stepping runs in the library; this module only reads the two probe series back
and takes their discrete Fourier transforms."""
import copy

import numpy as np

from . import binding as B


def _series(run, ports, precision):
    sim = B.Sim(run, precision=precision, max_probes=len(ports), probe_capacity=run.steps)
    ids = [sim.add_probe(B.F_E, p) for p in ports]
    sim.run(run.steps)
    out = [sim.read_probe(i, run.steps) for i in ids]
    sim.close()
    return out


def slab_sparams(run, freqs_hz, precision=B.FP32, ports=None):
    """(S11, S21) at ``freqs_hz`` for a 1D Run1D (ports default to run.meta['ports'])."""
    ports = tuple(ports or run.meta["ports"])
    vac = copy.deepcopy(run)
    vac.ne = np.zeros_like(run.ne)
    vac.nubar = np.zeros_like(run.nubar)
    s1, s2 = _series(run, ports, precision)
    v1, v2 = _series(vac, ports, precision)
    dt = run.courant * run.dx / 299792458.0
    t = (np.arange(run.steps) + 1) * dt
    ph = np.exp(-2j * np.pi * np.outer(np.asarray(freqs_hz, dtype=np.float64), t))
    inc = ph @ v1
    return (ph @ (s1 - v1)) / inc, (ph @ s2) / (ph @ v2)


def _series_3d(run, ports, precision):
    sim = B.Sim(run, precision=precision, max_probes=len(ports), probe_capacity=run.steps)
    ids = [sim.add_probe3d(B.F_EX, *p) for p in ports]
    sim.run(run.steps)
    out = [sim.read_probe(i, run.steps) for i in ids]
    sim.close()
    return out


def slab_ports_3d(run):
    """Ex points at the middle of the cross-section on the planes just before and just after
    the slab (the paper's z = 0 and z = 4 mm)."""
    k0, k1 = run.meta["slab"]
    i, j = run.nx // 2, run.ny // 2
    return ((i, j, k0 - 1), (i, j, k1))


def slab_sparams_3d(run, freqs_hz, precision=B.FP32, ports=None):
    """(S11, S21) at ``freqs_hz`` for a 3D Run3D with a sheet source (a plane wave along z),
    from Ex probes at ``ports`` (default: slab_ports_3d), as slab_sparams does in 1D."""
    ports = tuple(ports or slab_ports_3d(run))
    vac = copy.deepcopy(run)
    vac.ne = np.zeros_like(run.ne)
    vac.nubar = np.zeros_like(run.nubar)
    s1, s2 = _series_3d(run, ports, precision)
    v1, v2 = _series_3d(vac, ports, precision)
    dt = run.courant * run.dx / 299792458.0
    t = (np.arange(run.steps) + 1) * dt
    ph = np.exp(-2j * np.pi * np.outer(np.asarray(freqs_hz, dtype=np.float64), t))
    inc = ph @ v1
    return (ph @ (s1 - v1)) / inc, (ph @ s2) / (ph @ v2)
