"""GPU parity of the full-distribution kinetic model (the whole f of each plasma node
evolves: its even part heats, its odd part carries the current) against the FP64 oracle,
through the C ABI.  Tolerances as for the linear model: FP64 storage <= 1e-12 relative
L2, FP32 storage <= 1e-5 relative L2 over space and time."""
import numpy as np
import pytest

from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import workloads as W
from parity import oracle_1d, rel_l2, space_time_1d

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-full] {msg}", flush=True)


def _strong(nv, steps=700, amp64=3e5):
    """Slab over several tiles with a vacuum gap, driven hard enough that the electrons
    heat to a few times their thermal energy (velocity CFL about 0.1-0.2 at every Nv)."""
    run = W.slab_1d(777, nv, 130, 555, 1.1, 0.2, W.F_REF, 40, steps)
    run.ne[300:320] = 0.0
    run.src_amp = amp64 * 64 / nv
    run.kinetic = "full"
    return run


@pytest.mark.parametrize("nv,tile", [(8, 32), (16, 64), (64, 96), (128, 256), (512, 64),
                                     (1024, 32)])
def test_full_model_parity(gpu_lib, nv, tile):
    """Every lane layout of the full-model kernel (lanes per row 1..64, chunks per lane
    1..4), ragged tiles, both storage precisions, both collision models; E over space
    and time, J, and f - n fhat on the signed grid."""
    run = _strong(nv)
    for prec, tol in ((B.FP64, 1e-12), (B.FP32, 1e-5)):
        for model in ("hard_sphere", "const"):
            _banner(f"nv={nv} tile={tile} prec={prec} nu={model}")
            run.nu_model = model
            sim = B.Sim(run, precision=prec, tile=tile, time_block=1)   # one-step kernel
            assert sim.time_block() == 1
            orc = oracle_1d(run)
            snaps = []
            g, o, _, _ = space_time_1d(sim, orc, run.steps, 100, [], df_snaps=snaps)
            err = rel_l2(g, o)
            _banner(f"  E space-time rel L2 = {err:.3e}")
            assert err <= tol, (prec, model)
            assert rel_l2(sim.read(B.F_J), orc.J) <= tol
            gd = np.concatenate([a.ravel() for a, _ in snaps])
            od = np.concatenate([b.ravel() for _, b in snaps])
            assert rel_l2(gd, od) <= tol
            sim.close()


def test_full_model_differs_from_linear_and_keeps_number(gpu_lib):
    """At this drive the full model departs from the linear one by over 10 % (heating
    is exercised), and every node keeps its electron number: the signed-grid rows of
    f - n fhat sum to zero to rounding (FP64)."""
    run = _strong(64)
    sim = B.Sim(run, precision=B.FP64)
    sim.run(run.steps)
    E_full = sim.read(B.F_E)
    rows = sim.read(B.F_DF).reshape(-1, run.nv)
    sim.close()
    assert np.abs(rows).max() > 0
    assert np.max(np.abs(rows.sum(axis=1))) <= 1e-12 * np.abs(rows).max() * run.nv
    run.kinetic = "linear"
    lin = B.Sim(run, precision=B.FP64)
    lin.run(run.steps)
    assert rel_l2(E_full, lin.read(B.F_E)) > 0.1
    lin.close()


def test_full_model_velocity_cfl_flagged(gpu_lib):
    """A field that breaks |(e/m) E dt / dv| <= 1 sets the run status; a run within the
    limit reports none."""
    run = _strong(64, steps=700)
    sim = B.Sim(run, precision=B.FP64)
    sim.run(run.steps)
    assert sim.run_status(0) == 0
    sim.close()
    run.src_amp *= 20.0
    sim = B.Sim(run, precision=B.FP64)
    sim.run(run.steps)
    assert sim.run_status(0) != 0
    sim.close()


def test_full_model_configurations_rejected(gpu_lib):
    """The full model runs 1D single runs and batches of full-model runs: a batch that
    mixes it with the linear model, and 2D runs, refuse it."""
    run = _strong(64)
    lin = _strong(64)
    lin.kinetic = "linear"
    with pytest.raises(B.FdtdError):
        B.Sim([run, lin], precision=B.FP32)
    r2 = W.c2(n=64, radius=10.0, steps=10)
    r2.kinetic = "full"
    with pytest.raises(B.FdtdError):
        B.Sim(r2, precision=B.FP32)


def test_full_model_at_benchmark_size_prefix_parity(gpu_lib):
    """The full-distribution model at the benchmark's size (Nx = 65536, Nv = 512, FP32, 9
    steps per launch as timed): after 1500 steps the field has travelled at most 1500
    nodes, so the oracle on the prefix [0, src + 1510] is exact there; beyond it everything
    stays at its initial value (zero field, f = n fhat)."""
    run = W.c1()
    run.kinetic = "full"
    steps = 1500
    cut = run.src_node + steps + 10
    _banner("full model, Nx=65536 prefix")
    sim = B.Sim(run, precision=B.FP32, time_block=9)
    assert sim.time_block() == 9
    orc = oracle_1d(run, nx=cut)
    snaps = []
    g, o, _, _ = space_time_1d(sim, orc, steps, 250, [], df_snaps=snaps)
    err = rel_l2(g, o)
    _banner(f"  E space-time rel L2 = {err:.3e}")
    assert err <= 1e-5
    err_df = rel_l2(np.concatenate([a for a, _ in snaps]), np.concatenate([b for _, b in snaps]))
    _banner(f"  f - n fhat space-time rel L2 = {err_df:.3e}")
    assert err_df <= 1e-5
    assert np.all(sim.read(B.F_E)[cut + 1:] == 0.0)
    df = sim.read(B.F_DF).reshape(run.plasma_cells, run.nv)
    assert np.all(df[len(orc.cells):] == 0.0)
    sim.close()


def _long(nv, steps=600):
    """A line long enough for K steps per launch (5001 nodes, plasma over many tiles with a
    vacuum gap), the source 90 nodes before the slab, driven until the electrons heat."""
    run = W.slab_1d(5000, nv, 130, 4200, 1.1, 0.2, W.F_REF, 40, steps)
    run.ne[300:320] = 0.0
    run.src_amp = 3e5 * 64 / nv
    run.kinetic = "full"
    return run


@pytest.mark.parametrize("mode", [1, 0])
def test_full_model_batch_equals_solo_bitwise(gpu_lib, mode):
    """A batch of full-model runs of uneven size (Nv 64, 256 and 512; runs that end inside
    and at the end of K-step blocks) ends bitwise where each run ends alone, in either
    batch mode (the persistent launch takes linear runs only, so a full-model batch falls
    back to K-step launches there)."""
    g = np.random.default_rng(5)
    runs = []
    for r, nv in enumerate((64, 256, 512, 64, 256)):
        nx = int(g.integers(400, 1400))
        run = W.slab_1d(nx, nv, int(0.3 * nx), int(0.7 * nx), 1.0, 0.2, W.F_REF, 40,
                        int(g.integers(300, 900)), name=f"fb{r}")
        run.src_amp = 3e5 * 64 / nv
        run.kinetic = "full"
        runs.append(run)
    _banner(f"full-model batch, mode {mode}")
    bat = B.Sim(runs, batch_mode=mode)
    assert bat.time_block() > 1
    bat.run(max(r.steps for r in runs) + 3)
    for r, run in enumerate(runs):
        assert bat.run_status(r) == B.OK
        solo = B.Sim(run)
        solo.run(run.steps)
        for f in (B.F_E, B.F_H, B.F_J, B.F_DF):
            assert np.array_equal(bat.read(f, run=r), solo.read(f)), (r, f)
        solo.close()
    bat.close()


@pytest.mark.parametrize("nv", [64, 512])
def test_blocked_full_model_is_bitwise_the_one_step_run(gpu_lib, nv):
    """K steps per launch (rows of 32 or 256 stored bins per half) against one step per
    launch: E, H, J and the rows agree to the bit, also over calls that end inside a
    block."""
    run = _long(nv)
    a = B.Sim(run, precision=B.FP32)
    kb = a.time_block()
    _banner(f"nv={nv}: {kb} steps per launch")
    assert kb > 1
    b = B.Sim(run, precision=B.FP32, time_block=1)
    for n in (kb * 20, 1, 2 * kb + 3, 250):
        a.run(n)
        b.run(n)
        for f in (B.F_E, B.F_H, B.F_J, B.F_DF):
            assert np.array_equal(a.read(f), b.read(f)), (n, f)
    assert a.run_status(0) == 0
    a.close(); b.close()


@pytest.mark.parametrize("nv", [64, 512])
def test_blocked_full_model_parity(gpu_lib, nv):
    """The blocked run against the FP64 oracle: E over space and time, f - n fhat."""
    run = _long(nv, steps=540)
    sim = B.Sim(run, precision=B.FP32)
    assert sim.time_block() > 1
    orc = oracle_1d(run)
    snaps = []
    g, o, _, _ = space_time_1d(sim, orc, run.steps, 90, [], df_snaps=snaps)
    err = rel_l2(g, o)
    _banner(f"nv={nv} blocked: E space-time rel L2 = {err:.3e}")
    assert err <= 1e-5
    gd = np.concatenate([a.ravel() for a, _ in snaps])
    od = np.concatenate([b.ravel() for _, b in snaps])
    err_f = rel_l2(gd, od)
    _banner(f"  f - n fhat space-time rel L2 = {err_f:.3e}")
    assert err_f <= 1e-5
    sim.close()
