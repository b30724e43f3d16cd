"""GPU tests of the learned closure inside 2D runs: parity with the oracle's closure cells
(BF16 emulation), the kinetic fallback for cells outside the training box, resume, and the
trained network: its gain over the network-free recurrence on held-out data and the
slab transmission against the kinetic model."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle.core import Oracle2D
from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import closure as CL
from paper_2211_05647_amd import workloads as W
from parity import rel_l2
import analytic as A

pytestmark = pytest.mark.gpu

DT = 0.5 * W.DX_REF / A.C0
BOX = (0.05, 0.2, -3.0, -0.5)   # omega_p dt of the 0.9 blob = 0.071 (inside), 3.0 blob = 0.236 (outside)


def _banner(msg):
    print(f"[gpu-closure2d] {msg}", flush=True)


def _params(seed=21):
    p = M.init_params(seed)
    p[-129:-1] *= 5.0      # a visible correction
    p[-1] = 0.02
    return p.astype(np.float32).astype(np.float64)


def blob_run(nx=72, ny=60, hot_blob=False, steps=400, nu_ratio=0.3):
    jj, ii = np.mgrid[0:ny, 0:nx]
    ratio = np.zeros((ny, nx))
    ratio[(ii + 0.5 - 45) ** 2 + (jj + 0.5 - 30) ** 2 < 11 ** 2] = 0.9
    if hot_blob:
        ratio[(ii + 0.5 - 22) ** 2 + (jj + 0.5 - 14) ** 2 < 6 ** 2] = 3.0   # outside the box
    ne = np.where(ratio > 0, W.density_from_ratio(ratio, W.F_REF), 0.0)
    nu = np.where(ratio > 0, nu_ratio * 2 * math.pi * W.F_REF, 0.0)
    return W.Run2D(name="clo", nx=nx, ny=ny, nv=32, ne=ne, nubar=nu, src_kind=2, src_i=12,
                   src_j=ny // 2, steps=steps, ncpml=8, te_ev=5.0, **W.pulse(W.F_REF))


def oracle_with_closure(run, params, box):
    o = Oracle2D(run.nx, run.ny, run.dx, run.courant, run.ne, run.nubar, nv=run.nv,
                 te_ev=run.te_ev, ncpml=run.ncpml, src_kind=run.src_kind, src_i=run.src_i,
                 src_j=run.src_j, src_amp=run.src_amp, src_f=run.src_f, src_tau=run.src_tau,
                 src_t0=run.src_t0)
    w, s = A.velocity_weights(run.nv, 6.0, run.te_ev, "hard_sphere", dims=2)
    mode, coef = [], []
    for c in o.cells:
        ne, nu = o.ne[c], o.nubar[c]
        q1, q2 = M.scale_params(math.sqrt(A.plasma_omega2(ne)) * o.dt, nu * o.dt, box)
        a, b = M.effective_pole(w, s, nu, A.plasma_omega2(ne), o.dt)
        inside = -1 <= q1 <= 1 and -1 <= q2 <= 1
        mode.append(1 if inside else 0)
        coef.append((a, b, q1, q2))
    o.set_closure(np.array(mode), np.array(coef), params, emulate_bf16=True)
    return o, int(np.sum(mode))


def run_pair(sim, orc, steps, every=50):
    g, o = [], []
    done = 0
    while done < steps:
        sim.run(every)
        orc.run(every)
        done += every
        g.append(np.concatenate([sim.read(B.F_EX), sim.read(B.F_EY)]))
        o.append(np.concatenate([orc.Ex.ravel(), orc.Ey.ravel()]))
    return np.array(g), np.array(o)


def counts(sim):
    return sim.closure_counts()


@pytest.mark.parametrize("hot", [False, True])
def test_closure_cells_match_oracle(gpu_lib, hot):
    run = blob_run(hot_blob=hot)
    p = _params()
    blob = CL.make_blob(p, BOX, DT)
    _banner(f"closure vs oracle, out-of-box blob={hot}")
    sim = B.Sim(run, precision=B.FP32, closure=B.CLOSURE_MLP, mlp_blob=blob)
    orc, nclo = oracle_with_closure(run, p, BOX)
    nm, nk = counts(sim)
    assert nm == nclo and nm + nk == run.plasma_cells
    assert (nk > 0) == hot
    g, o = run_pair(sim, orc, run.steps)
    err = rel_l2(g, o)
    _banner(f"  closure cells {nm}, kinetic {nk}: space-time rel L2 {err:.2e}")
    assert err <= 1e-5


def test_mismatched_closure_falls_back_to_kinetic_bitwise(gpu_lib):
    """A network trained for another time step is not used: every cell runs the kinetic
    step and the run is bitwise the kinetic run."""
    run = blob_run(steps=200)
    blob = CL.make_blob(_params(), BOX, DT * 1.01)
    a = B.Sim(run, closure=B.CLOSURE_MLP, mlp_blob=blob)
    b = B.Sim(run)
    assert counts(a) == (0, run.plasma_cells)
    a.run(run.steps)
    b.run(run.steps)
    for f in (B.F_EX, B.F_EY, B.F_HZ, B.F_DF):
        assert np.array_equal(a.read(f), b.read(f))


def test_closure_resume_bitwise(gpu_lib):
    run = blob_run(hot_blob=True, steps=200)
    blob = CL.make_blob(_params(), BOX, DT)
    a = B.Sim(run, closure=B.CLOSURE_MLP, mlp_blob=blob)
    a.run(100)
    st = a.save_state()
    a.run(100)
    c = B.Sim(run, closure=B.CLOSURE_MLP, mlp_blob=blob)
    c.load_state(st)
    c.run(100)
    for f in (B.F_EX, B.F_EY, B.F_JX, B.F_DF):
        assert np.array_equal(a.read(f), c.read(f))


def _slab_T(blob, closure, nu_ratio, ratio=0.8, nsteps=3000):
    nx, ny, lo, hi = 1400, 18, 650, 850
    ne = np.zeros((ny, nx))
    nu = np.zeros((ny, nx))
    ne[:, lo:hi] = W.density_from_ratio(ratio, W.F_REF)
    nu[:, lo:hi] = nu_ratio * 2 * math.pi * W.F_REF
    run = W.Run2D(name="slab", nx=nx, ny=ny, nv=32, ne=ne, nubar=nu, src_kind=1, src_i=350,
                  src_j=0, steps=nsteps, ncpml=8, te_ev=5.0, **W.pulse(W.F_REF))
    vac = W.Run2D(name="vac", nx=nx, ny=ny, nv=32, ne=np.zeros_like(ne), nubar=np.zeros_like(nu),
                  src_kind=1, src_i=350, src_j=0, steps=nsteps, ncpml=8, te_ev=5.0, **W.pulse(W.F_REF))
    out = []
    for r, cl in ((vac, B.CLOSURE_KINETIC), (run, closure)):
        sim = B.Sim(r, closure=cl, mlp_blob=blob if cl == B.CLOSURE_MLP else None,
                    max_probes=1, probe_capacity=nsteps)
        pid = sim.add_probe(B.F_EY, 950, 9)
        sim.run(nsteps)
        out.append(sim.read_probe(pid, nsteps))
    fs = np.linspace(0.6, 1.6, 41) * W.F_REF
    pin, ptot = out
    spec = np.array([abs(A.dft(pin, 2 * math.pi * f, DT)) for f in fs])
    fs = fs[spec >= 0.1 * spec.max()]
    return np.array([abs(A.dft(ptot, 2 * math.pi * f, DT) / A.dft(pin, 2 * math.pi * f, DT)) for f in fs])


@pytest.fixture(scope="module")
def trained():
    import torch
    _banner("gathering training data from the 256-run batch")
    data, c = CL.gather_data(log=lambda m: _banner(m))
    params, hist = CL.fit(data, c, log=lambda m: _banner(m))
    net, zero = CL.evaluate(data, c, data.held)
    _banner(f"held-out MSE: network {net:.4e}, without network {zero:.4e}")
    return data, c, params, (net, zero)


def test_trained_network_gains_on_held_out_runs(gpu_lib, trained):
    """What the network gains over the method without it (y = 0, the single-pole
    recurrence): one-step error of the current on runs it never saw."""
    data, c, params, (net, zero) = trained
    assert net < 0.5 * zero


def test_surrogate_slab_transmission(gpu_lib, trained):
    """Slab |T| of the surrogate (network + single pole) within 1e-2 of the kinetic model at
    two collision rates inside the training box, and closer to the kinetic |T| than the
    single pole alone (y = 0, the method without the network) at both.  The single pole is
    already close at nu/w = 0.05 (about 1e-3), so that case asks for the smaller margin."""
    data, c, params, _ = trained
    blob = CL.make_blob(params, data.box, data.dt)
    zero_blob = CL.make_blob(np.zeros(B.NPARAM, dtype=np.float32), data.box, data.dt)
    for nu_ratio in (0.05, 0.4):
        Tk = _slab_T(None, B.CLOSURE_KINETIC, nu_ratio)
        Tm = _slab_T(blob, B.CLOSURE_MLP, nu_ratio)
        Tz = _slab_T(zero_blob, B.CLOSURE_MLP, nu_ratio)
        em, ez = np.max(np.abs(Tm - Tk)), np.max(np.abs(Tz - Tk))
        _banner(f"slab nu/w={nu_ratio}: max ||T| - |T_kin||: network {em:.2e}, no network {ez:.2e}")
        assert em <= 1e-2
        assert em < ez, f"the network should beat the single pole at nu/w = {nu_ratio}"
