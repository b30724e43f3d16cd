"""GPU parity of the 3D path (Yee cube with the CPML on all faces, speed-grid F1 at every
plasma E point: the paper's production model) against the FP64 oracle, through the C ABI.
Tolerances: FP64 storage <= 1e-12 relative L2, FP32 storage <= 1e-5 relative L2 over space
and time."""
import numpy as np
import pytest

from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import workloads as W
from parity import oracle_3d, rel_l2, space_time_3d

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-3d] {msg}", flush=True)


def _small(nx=20, ny=18, nz=48, nv=31, f0="druyvesteyn", ncpml=6, steps=420):
    return W.argon_slab_3d(nx=nx, ny=ny, nz=nz, nv=nv, steps=steps, ncpml=ncpml, f0=f0)


def _check(run, prec, tol, every=60):
    """E, the electromagnetic state (E, eta0 H), J and F1 compared over space and time
    (snapshots every ``every`` steps).  H alone is not held to the bar: in a closed PEC
    box a point source leaves a static E whose discrete curl is zero only up to rounding,
    and H (the dynamic part alone) is then small against that rounding."""
    sim = B.Sim(run, precision=prec)
    orc = oracle_3d(run)
    assert sim.closure_counts()[1] == orc.npoints > 0
    snaps = space_time_3d(sim, orc, run.steps, every)
    eta0 = 376.730313668
    ge, oe = snaps["E"]
    gh, oh = snaps["H"]
    snaps["EM"] = (np.concatenate([ge, eta0 * gh], axis=1), np.concatenate([oe, eta0 * oh], axis=1))
    _banner(f"  H alone rel L2 = {rel_l2(gh, oh):.3e}")
    for name in ("E", "EM", "J", "DF"):
        g, o = snaps[name]
        err = rel_l2(g, o)
        _banner(f"  {name} space-time rel L2 = {err:.3e}")
        assert err <= tol, name
    assert np.abs(orc.J).max() > 0
    sim.close()


@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-12), (B.FP32, 1e-5)])
def test_argon_slab_parity(gpu_lib, prec, tol):
    """The paper's slab (Druyvesteyn F0, v_dim = 31, hard-sphere nu) in a small box with
    the layer on every face; E, H, J and F1."""
    run = _small()
    _banner(f"argon slab prec={prec}")
    _check(run, prec, tol)


@pytest.mark.parametrize("nv", [1, 8, 64])
def test_speed_grids_and_models(gpu_lib, nv):
    """Other speed counts (row padding 4 .. 64), the Maxwellian F0, constant nu, ragged
    box sizes."""
    run = _small(nx=17, ny=13, nz=41, nv=nv, f0="maxwell", ncpml=5, steps=400)
    run.nu_model = "const"
    for prec, tol in ((B.FP64, 1e-12), (B.FP32, 1e-5)):
        _banner(f"nv={nv} prec={prec}")
        _check(run, prec, tol)


def test_pec_box_with_point_source(gpu_lib):
    """No layer (PEC faces) and an Ex point source inside a plasma block."""
    run = _small(nx=16, ny=15, nz=22, nv=16, ncpml=0, steps=300)
    run.ne[:] = 0.0
    run.ne[4:18, 3:12, 4:13] = W.ARGON_NE
    run.src_kind, run.src_i, run.src_j, run.src_k = 2, 7, 7, 6
    run.src_t0, run.src_tau = 60e-12, 20e-12
    for prec, tol in ((B.FP64, 1e-12), (B.FP32, 1e-5)):
        _banner(f"pec point prec={prec}")
        _check(run, prec, tol, every=50)


def test_resume_is_bitwise(gpu_lib):
    """Save after k steps, run on; load into a fresh handle and run the same steps: the
    fields agree to the bit."""
    run = _small(steps=300)
    a = B.Sim(run, precision=B.FP32)
    a.run(150)
    blob = a.save_state()
    a.run(150)
    b = B.Sim(run, precision=B.FP32)
    b.load_state(blob)
    b.run(150)
    for f in (B.F_EX, B.F_EY, B.F_EZ, B.F_HX, B.F_DF):
        assert np.array_equal(a.read(f), b.read(f))
    a.close()
    b.close()


def test_3d_rejections(gpu_lib):
    """Probes, a source off the grid and a too-large Courant number are refused."""
    run = _small(steps=10)
    sim = B.Sim(run, precision=B.FP32)
    with pytest.raises(B.FdtdError):
        sim.add_probe(B.F_EX, 3, 3)
    sim.close()
    bad = _small(steps=10)
    bad.src_k = 0
    with pytest.raises(B.FdtdError):
        B.Sim(bad, precision=B.FP32)
    bad = _small(steps=10)
    bad.courant = 0.6
    with pytest.raises(B.FdtdError):
        B.Sim(bad, precision=B.FP32)


def test_benchmark_size_light_cone_parity(gpu_lib):
    """The benchmark's 3D workload at its full size (128 x 128 x 512, FP32, the launch shape
    timed): in 150 steps the sheet source's field reaches at most 151 planes past it, so the
    oracle on the same transverse box cut at 180 planes (its own high-z layer unreached) is
    exact there, and every plane beyond stays zero."""
    run = W.argon_slab_3d(nx=128, ny=128, nz=512, steps=150)
    steps, cutz = 150, 180
    _banner("argon slab, full size, light cone")
    sim = B.Sim(run, precision=B.FP32)
    sim.run(steps)
    small = W.argon_slab_3d(nx=128, ny=128, nz=cutz, steps=steps)
    small.ne[:] = 0.0
    small.src_k = run.src_k
    orc = oracle_3d(small)
    orc.run(steps)
    F = orc.fields()
    ex = sim.read(B.F_EX).reshape(run.nz + 1, run.ny + 1, run.nx)
    ey = sim.read(B.F_EY).reshape(run.nz + 1, run.ny, run.nx + 1)
    ez = sim.read(B.F_EZ).reshape(run.nz, run.ny + 1, run.nx + 1)
    lim = run.src_k + steps + 2
    assert lim < cutz - run.ncpml
    g = np.concatenate([ex[:lim].ravel(), ey[:lim].ravel(), ez[:lim].ravel()])
    o = np.concatenate([F["Ex"][:lim].ravel(), F["Ey"][:lim].ravel(), F["Ez"][:lim].ravel()])
    err = rel_l2(g, o)
    _banner(f"  E rel L2 on the light cone = {err:.3e}")
    assert err <= 1e-5
    assert np.abs(o).max() > 0
    assert np.all(ex[lim:] == 0.0) and np.all(ey[lim:] == 0.0) and np.all(ez[lim:] == 0.0)
    sim.close()


def test_benchmark_size_parity_through_the_slab(gpu_lib):
    """The benchmark's 3D workload at its full size (128 x 128 x 512, FP32, the launch shape
    timed) for 800 steps, until the pulse is well into the slab: E, J and F1 against the
    oracle on the same box."""
    run = W.argon_slab_3d(nx=128, ny=128, nz=512, steps=800)
    _banner("argon slab, full size, 800 steps")
    sim = B.Sim(run, precision=B.FP32)
    sim.run(run.steps)
    orc = oracle_3d(run)
    orc.run(run.steps)
    assert sim.closure_counts()[1] == orc.npoints
    ge = np.concatenate([sim.read(f) for f in (B.F_EX, B.F_EY, B.F_EZ)])
    gj = np.concatenate([sim.read(f) for f in (B.F_JX, B.F_JY, B.F_JZ)])
    for name, g, o in (("E", ge, orc.E), ("J", gj, orc.J), ("F1", sim.read(B.F_DF), orc.df)):
        err = rel_l2(g, o)
        _banner(f"  {name} rel L2 = {err:.3e}")
        assert err <= 1e-5, name
    assert np.abs(orc.J).max() > 0
    sim.close()


def _e_index(run, comp, i, j, k):
    """Flat index into [Ex | Ey | Ez] of the oracle's E of component comp at (i, j, k)."""
    X, Y, Z = run.nx, run.ny, run.nz
    shapes = [(X, Y + 1, Z + 1), (X + 1, Y, Z + 1), (X + 1, Y + 1, Z)]
    base = sum(a * b * c for a, b, c in shapes[:comp])
    nxc, nyc, _ = shapes[comp]
    return base + (k * nyc + j) * nxc + i


@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-12), (B.FP32, 1e-5)])
def test_probes_3d_match_the_oracle(gpu_lib, prec, tol):
    """Probes on the three E components (before, inside and after the slab, off the axis)
    record after every step what the oracle's E holds there."""
    run = _small(steps=400)
    k0, k1 = run.meta["slab"]
    pts = [(0, 10, 9, k0 - 1), (0, 3, 5, k0 + 2), (1, 7, 4, k1 + 1), (2, 8, 8, k0 + 4)]
    fields = [B.F_EX, B.F_EY, B.F_EZ]
    sim = B.Sim(run, precision=prec, max_probes=len(pts), probe_capacity=run.steps)
    ids = [sim.add_probe3d(fields[c], i, j, k) for c, i, j, k in pts]
    sim.run(run.steps)
    g = np.stack([sim.read_probe(q, run.steps) for q in ids], axis=1)
    orc = oracle_3d(run)
    o = orc.run(run.steps, probes=[_e_index(run, c, i, j, k) for c, i, j, k in pts])
    err = rel_l2(g, o)
    _banner(f"probes prec={prec}: rel L2 = {err:.3e}")
    assert err <= tol
    assert np.abs(o).max() > 0
    sim.close()


def test_probe3d_rejections(gpu_lib):
    """add_probe on a 3D handle, another field, an index outside the component's array,
    more probes than slots, a probe after the first step, add_probe3d on a 1D handle."""
    run = _small(steps=10)
    sim = B.Sim(run, precision=B.FP32, max_probes=2, probe_capacity=10)
    with pytest.raises(B.FdtdError):
        sim.add_probe(B.F_EX, 3, 3)
    with pytest.raises(B.FdtdError):
        sim.add_probe3d(B.F_HX, 3, 3, 3)
    with pytest.raises(B.FdtdError):
        sim.add_probe3d(B.F_EX, run.nx, 3, 3)      # Ex has nx points along x
    with pytest.raises(B.FdtdError):
        sim.add_probe3d(B.F_EZ, 3, 3, run.nz)      # Ez has nz points along z
    sim.add_probe3d(B.F_EY, run.nx, 3, 3)          # Ey has nx + 1
    sim.add_probe3d(B.F_EZ, 3, 3, run.nz - 1)
    with pytest.raises(B.FdtdError):
        sim.add_probe3d(B.F_EX, 1, 1, 1)           # no slot left
    sim.close()
    sim = B.Sim(run, precision=B.FP32, max_probes=2, probe_capacity=10)
    sim.run(1)
    with pytest.raises(B.FdtdError):
        sim.add_probe3d(B.F_EX, 1, 1, 1)
    sim.close()
    line = W.slab_1d(100, 8, 40, 60, 0.5, 0.1, W.F_REF, 20, 10)
    s1 = B.Sim(line, precision=B.FP32, max_probes=1, probe_capacity=10)
    with pytest.raises(B.FdtdError):
        s1.add_probe3d(B.F_EX, 1, 1, 1)
    s1.close()
