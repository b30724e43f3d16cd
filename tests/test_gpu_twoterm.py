"""GPU parity of the 1D two-term model (speed-grid F1 and an evolving F0: the paper's
l = 0 and l = 1 equations) against the FP64 oracle, through the C ABI.  Tolerances as for
the other models: FP64 storage <= 1e-12 relative L2, FP32 storage <= 1e-5 relative L2 over
space and time."""
import numpy as np
import pytest

from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import workloads as W
from parity import oracle_1d, rel_l2, space_time_1d

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-twoterm] {msg}", flush=True)


def _run(nv, f0="druyvesteyn", amp=3e4, steps=700):
    """777-node line, slab over several tiles with a vacuum gap, Te = 1 eV, speeds to 5 v_th;
    driven hard enough that F0 visibly widens (heating)."""
    run = W.slab_1d(777, 8, 130, 555, 1.1, 0.2, W.F_REF, 40, steps, te_ev=1.0)
    run.ne[300:320] = 0.0
    run.nv = nv
    run.vmax_over_vth = 5.0
    run.src_amp = amp
    run.kinetic = "two_term"
    run.f0_model = f0
    return run


@pytest.mark.parametrize("nv,tile", [(2, 32), (8, 64), (31, 96), (64, 256), (256, 64)])
def test_two_term_parity(gpu_lib, nv, tile):
    """Speed counts 2..256 (rows padded to 4..256 bins: lanes per row 1..64, one or two
    chunks per lane), ragged tiles, both precisions, both F0 shapes and collision models;
    E over space and time (snapshots every 100 steps: each run() call ends with the
    deferred l = 0 update), J, and [F1 | F0 - n F0hat]."""
    for prec, tol in ((B.FP64, 1e-12), (B.FP32, 1e-5)):
        for f0, model in (("druyvesteyn", "hard_sphere"), ("maxwell", "const")):
            run = _run(nv, f0=f0)
            run.nu_model = model
            _banner(f"nv={nv} tile={tile} prec={prec} f0={f0} nu={model}")
            sim = B.Sim(run, precision=prec, tile=tile, time_block=1)   # one-step kernel
            assert sim.time_block() == 1
            orc = oracle_1d(run)
            snaps = []
            g, o, _, _ = space_time_1d(sim, orc, run.steps, 100, [], df_snaps=snaps)
            err = rel_l2(g, o)
            _banner(f"  E space-time rel L2 = {err:.3e}")
            assert err <= tol
            if prec == B.FP64:
                # (in FP32 the last step's J alone can be small against its rounding; F1,
                # whose moment J is, is compared over space and time below)
                assert rel_l2(sim.read(B.F_J), orc.J) <= tol
            gd = np.concatenate([a.ravel() for a, _ in snaps])
            od = np.concatenate([b.ravel() for _, b in snaps])
            assert rel_l2(gd, od) <= tol
            rows = sim.read(B.F_DF).reshape(-1, 2 * nv)
            orows = orc.df_rows()
            assert np.abs(orows[:, nv:]).max() > 0          # F0 has moved
            err0 = rel_l2(rows[:, nv:], orows[:, nv:])
            _banner(f"  F0 - n F0hat rel L2 = {err0:.3e}")
            assert err0 <= tol
            sim.close()


def test_call_boundaries_do_not_change_the_result(gpu_lib):
    """One run of 300 steps and the same 300 steps in calls of 1, 2, 97 and 200 steps give
    the same fields and rows to the bit (the deferred l = 0 update is flushed at every
    call's end with the same arithmetic)."""
    run = _run(31, steps=300)
    a = B.Sim(run, precision=B.FP32)
    a.run(300)
    b = B.Sim(run, precision=B.FP32)
    for n in (1, 2, 97, 200):
        b.run(n)
    for f in (B.F_E, B.F_H, B.F_J, B.F_DF):
        assert np.array_equal(a.read(f), b.read(f))
    blob = b.save_state()
    a.run(50)
    c = B.Sim(run, precision=B.FP32)
    c.load_state(blob)
    c.run(50)
    assert np.array_equal(a.read(B.F_DF), c.read(B.F_DF))
    a.close(); b.close(); c.close()


def test_two_term_batch_rules(gpu_lib):
    """Two-term runs batch with each other, in FP32 only, and not with runs of another
    model."""
    run = _run(31)
    lin = _run(31)
    lin.kinetic = "linear"
    lin.nv = 64
    with pytest.raises(B.FdtdError):
        B.Sim([run, lin], precision=B.FP32)
    with pytest.raises(B.FdtdError):
        B.Sim([run, run], precision=B.FP64)
    B.Sim([run, run], precision=B.FP32).close()


def test_two_term_cfl_flagged(gpu_lib):
    """A field with (e/m) |E| dt / gam > 1 sets the run status; the tested drive does not."""
    run = _run(31, steps=700)
    sim = B.Sim(run, precision=B.FP64)
    sim.run(run.steps)
    assert sim.run_status(0) == 0
    sim.close()
    run.src_amp *= 100.0
    sim = B.Sim(run, precision=B.FP64)
    sim.run(run.steps)
    assert sim.run_status(0) != 0
    sim.close()


def _long(nv, amp=3e4, steps=600):
    """A line long enough for K steps per launch (5001 nodes; plasma over many tiles with
    a vacuum gap), the source 90 nodes before the slab, so that the pulse is well inside
    it within the run and F0 widens."""
    run = W.slab_1d(5000, 8, 130, 4200, 1.1, 0.2, W.F_REF, 40, steps, te_ev=1.0)
    run.ne[300:320] = 0.0
    run.nv = nv
    run.vmax_over_vth = 5.0
    run.src_amp = amp
    run.kinetic = "two_term"
    run.f0_model = "druyvesteyn"
    return run


@pytest.mark.parametrize("nv", [31, 64])
def test_blocked_two_term_is_bitwise_the_one_step_run(gpu_lib, nv):
    """K steps per launch (rows of 32 or 64 speeds) against one step per launch: E, H, J,
    F1 and F0 agree to the bit, also over calls that end inside a block (their last steps
    run one per launch and end with the deferred l = 0 update)."""
    run = _long(nv)
    a = B.Sim(run, precision=B.FP32)
    kb = a.time_block()
    _banner(f"nv={nv}: {kb} steps per launch")
    assert kb > 1
    b = B.Sim(run, precision=B.FP32)
    b.set_time_block(1)
    assert b.time_block() == 1
    for n in (kb * 20, 1, 2 * kb + 3, 250):
        a.run(n)
        b.run(n)
        for f in (B.F_E, B.F_H, B.F_J, B.F_DF):
            assert np.array_equal(a.read(f), b.read(f)), (n, f)
    assert a.run_status(0) == 0
    a.close(); b.close()


@pytest.mark.parametrize("nv", [31, 64])
def test_blocked_two_term_parity(gpu_lib, nv):
    """The blocked run against the FP64 oracle: E over space and time, F1 and F0."""
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
    assert rel_l2(gd, od) <= 1e-5
    rows = sim.read(B.F_DF).reshape(-1, 2 * nv)
    assert np.abs(orc.df_rows()[:, nv:]).max() > 0
    err0 = rel_l2(rows[:, nv:], orc.df_rows()[:, nv:])
    _banner(f"  F0 - n F0hat rel L2 = {err0:.3e}")
    assert err0 <= 1e-5
    sim.close()


@pytest.mark.parametrize("mode", [1, 0])
def test_two_term_batch_equals_solo_bitwise(gpu_lib, mode):
    """A batch of two-term runs of uneven length (31 and 64 speeds; runs that stop inside a
    K-step pass, at its end, and after the call boundaries), advanced over calls of uneven
    length, ends bitwise where each run ends alone: every run takes its own last deferred
    l = 0 update when it stops (the persistent form takes linear runs only, so the batch
    uses K-step launches in either mode)."""
    g = np.random.default_rng(7)
    runs = []
    for r, nv in enumerate((31, 64, 31, 64, 31)):
        run = _run(nv, steps=int(g.integers(200, 700)))
        run.name = f"tb{r}"
        runs.append(run)
    runs[2].steps = 9 * 40          # stops at the end of a pass
    runs[4].steps = 9 * 40 + 4      # stops inside one
    _banner(f"two-term batch, mode {mode}")
    bat = B.Sim(runs, batch_mode=mode)
    assert bat.time_block() > 1
    total = max(r.steps for r in runs) + 5
    done = 0
    for k in (1, 100, 7, 251, 1000):
        k = min(k, total - done)
        if k <= 0:
            break
        bat.run(k)
        done += k
    assert done == total
    for r, run in enumerate(runs):
        assert bat.run_status(r) == B.OK
        solo = B.Sim(run)
        solo.run(run.steps)
        for f in (B.F_E, B.F_H, B.F_J, B.F_DF):
            assert np.array_equal(bat.read(f, run=r), solo.read(f)), (r, f)
        solo.close()
    bat.close()
