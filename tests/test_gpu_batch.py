"""GPU tests of the batched 1D path: many independent runs of uneven size, in K-step
blocked launches (the default) or in one persistent launch (work-groups take (tile, block)
items from a counter, each waiting for its neighbours' previous block), the training-pair
taps, per-run status, and parity with solo runs and with the FP64 oracle."""
import math

import numpy as np
import pytest

from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import workloads as W
from parity import oracle_1d, rel_l2

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-batch] {msg}", flush=True)


def small_batch(n=10, seed=3, nx_hi=1500):
    g = np.random.default_rng(seed)
    runs = []
    for r in range(n):
        nx = int(g.integers(300, nx_hi))
        nv = int(g.choice([64, 128, 256]))
        f_src = W.F_REF * (1 + g.uniform(-0.3, 0.3))
        run = W.slab_1d(nx, nv, int(0.4 * nx), int(0.6 * nx), g.uniform(0.2, 2.0),
                        10 ** g.uniform(-2, 0), f_src, int(0.1 * nx), 2 * nx,
                        name=f"b{r}")
        runs.append(run)
    return runs


def tap_nodes(runs, ntap, seed=9):
    g = np.random.default_rng(seed)
    out = np.zeros((len(runs), ntap), dtype=np.int32)
    for r, run in enumerate(runs):
        cells = np.nonzero(run.ne > 0)[0]
        out[r] = g.choice(cells, size=ntap, replace=False)
    return out


FIELDS = (B.F_E, B.F_H, B.F_J, B.F_DF)


@pytest.mark.parametrize("mode,groups", [(0, 0), (0, 3), (1, 0)])
def test_batch_equals_solo_bitwise(gpu_lib, mode, groups):
    """Run r of a batch ends bitwise equal to run r simulated alone, whatever the launch
    form (the persistent launch with every work-group that fits or with only three, or
    K-step blocked launches)."""
    runs = small_batch()
    _banner(f"batch == solo, mode={mode} groups={groups}")
    bat = B.Sim(runs, batch_mode=mode, groups=groups)
    bat.run(max(r.steps for r in runs) + 5)
    for r, run in enumerate(runs):
        solo = B.Sim(run)
        solo.run(run.steps)
        for f in FIELDS:
            assert np.array_equal(bat.read(f, run=r), solo.read(f)), (r, f)
        solo.close()


def test_batch_in_chunks_equals_one_call(gpu_lib):
    runs = small_batch(6, seed=11)
    _banner("batch in chunks")
    a = B.Sim(runs)
    a.run(max(r.steps for r in runs))
    b = B.Sim(runs)
    for k in (1, 7, 250, 999, 4000):
        b.run(k)
    for r in range(len(runs)):
        for f in FIELDS:
            assert np.array_equal(a.read(f, run=r), b.read(f, run=r))


def test_persistent_batch_in_chunks_equals_default(gpu_lib):
    """The persistent launch over calls of uneven length (1, 7, 250, ... steps: calls that
    end inside runs' K-step blocks, odd and even rests, runs that finish early) ends
    bitwise where the default launch form ends in one call, also with K = 5."""
    runs = small_batch(7, seed=17)
    total = max(r.steps for r in runs)
    for kb in (9, 5):
        _banner(f"persistent batch in chunks, K={kb}")
        a = B.Sim(runs, time_block=kb)
        a.run(total)
        b = B.Sim(runs, batch_mode=0, time_block=kb)
        done = 0
        for k in (1, 7, 250, 2, 999, 4000):
            b.run(k)
            done += k
        assert done >= total
        for r in range(len(runs)):
            assert b.run_status(r) == B.OK
            for f in FIELDS:
                assert np.array_equal(a.read(f, run=r), b.read(f, run=r)), (kb, r, f)
        a.close()
        b.close()


def test_persistent_batch_with_many_segments(gpu_lib):
    """300 short runs with 300 different step counts: more distinct block counts than the
    persistent launch keeps in LDS, so its segment table is read from global memory; the
    runs end bitwise where the default launch form takes them."""
    g = np.random.default_rng(13)
    runs = []
    for r in range(300):
        nx = int(g.integers(300, 400))
        # 2r + 1 blocks of 9 steps, plus one odd step for odd r: 300 distinct block counts
        run = W.slab_1d(nx, 64, int(0.4 * nx), int(0.6 * nx), 1.0, 0.1, W.F_REF, 30,
                        18 * r + 9 + (r % 2), name=f"m{r}")
        runs.append(run)
    _banner("persistent batch, 300 segments")
    total = max(r.steps for r in runs)
    a = B.Sim(runs)
    a.run(total)
    b = B.Sim(runs, batch_mode=0)
    b.run(total)
    for r in range(0, len(runs), 7):
        assert b.run_status(r) == B.OK
        for f in FIELDS:
            assert np.array_equal(a.read(f, run=r), b.read(f, run=r)), (r, f)
    a.close()
    b.close()


def test_batch_parity_with_oracle(gpu_lib):
    runs = small_batch(5, seed=21, nx_hi=900)
    _banner("batch vs oracle")
    bat = B.Sim(runs)
    snaps_g, snaps_o = [[] for _ in runs], [[] for _ in runs]
    orcs = [oracle_1d(run) for run in runs]
    done = 0
    total = max(r.steps for r in runs)
    while done < total:
        bat.run(200)
        done += 200
        for r, run in enumerate(runs):
            k = min(done, run.steps) - orcs[r].step
            if k > 0:
                orcs[r].run(k)
            snaps_g[r].append(bat.read(B.F_E, run=r))
            snaps_o[r].append(orcs[r].E.copy())
    for r in range(len(runs)):
        err = rel_l2(np.array(snaps_g[r]), np.array(snaps_o[r]))
        _banner(f"run {r}: space-time rel L2 {err:.2e}")
        assert err <= 1e-5


@pytest.mark.parametrize("mode", [1, 0])
def test_taps_record_drive_and_current(gpu_lib, mode):
    """Taps hold (E^n, J^{n+1/2}) at their nodes for every step: checked against the
    oracle stepped one step at a time, in both launch forms."""
    runs = small_batch(3, seed=31, nx_hi=500)
    taps = tap_nodes(runs, 4)
    _banner(f"taps, batch mode {mode}")
    bat = B.Sim(runs, taps=taps, batch_mode=mode)
    bat.run(max(r.steps for r in runs))
    for r, run in enumerate(runs):
        got = bat.read_taps(r)
        assert got.shape == (4, run.steps, 2)
        o = oracle_1d(run)
        E = np.zeros((run.steps, 4))
        J = np.zeros((run.steps, 4))
        for s in range(run.steps):
            E[s] = o.E[taps[r]]
            o.run(1)
            J[s] = o.J[taps[r]]
        assert rel_l2(got[:, :, 0].T, E) <= 1e-5
        assert rel_l2(got[:, :, 1].T, J) <= 1e-5


@pytest.mark.parametrize("mode", [1, 0])
def test_nonfinite_run_is_flagged_alone(gpu_lib, mode):
    """A run whose density overflows FP32 storage turns non-finite; only that run is
    flagged and the others stay bitwise equal to their solo runs, in both launch forms."""
    runs = small_batch(4, seed=41)
    runs[2].ne[runs[2].ne > 0] = 1e39
    _banner(f"non-finite run, batch mode {mode}")
    bat = B.Sim(runs, batch_mode=mode)
    bat.run(max(r.steps for r in runs))
    assert bat.run_status(2) == B.ENUMERIC
    with pytest.raises(B.FdtdError) as ei:
        bat.read(B.F_E, run=2)
    assert ei.value.code == B.ENUMERIC
    for r in (0, 1, 3):
        assert bat.run_status(r) == B.OK
        solo = B.Sim(runs[r])
        solo.run(runs[r].steps)
        assert np.array_equal(bat.read(B.F_E, run=r), solo.read(B.F_E))


def test_time_blocked_batch_is_bitwise_the_stepped_batch(gpu_lib):
    """The batch with K steps per launch (runs ending inside a pass finish one step per
    launch) against one step per launch: fields, F1 and taps bit for bit, for several K
    and a step count that is not a multiple of K."""
    runs = small_batch(8, seed=51, nx_hi=3000)
    taps = tap_nodes(runs, 3)
    total = max(r.steps for r in runs)
    _banner(f"time-blocked batch, {total} steps")
    ref = B.Sim(runs, taps=taps, time_block=1)
    assert ref.time_block() == 1
    ref.run(total // 3)
    ref.run(total - total // 3)
    for k in (3, 7):
        bat = B.Sim(runs, taps=taps, time_block=k)
        assert bat.time_block() == k
        bat.run(total // 3)
        bat.run(total - total // 3)
        for r in range(len(runs)):
            for f in FIELDS:
                assert np.array_equal(bat.read(f, run=r), ref.read(f, run=r)), (k, r, f)
            assert np.array_equal(bat.read_taps(r), ref.read_taps(r)), (k, r)
        bat.close()
