"""GPU parity of the 1D path (fused Yee + kinetic step kernel) against the FP64 oracle,
through the C ABI.  Tolerances: FP64 storage <= 1e-12 relative L2; FP32 storage
<= 1e-5 relative L2 over space and time (E snapshots plus probe series)."""
import math

import numpy as np
import pytest

from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import workloads as W
from parity import oracle_1d, rel_l2, space_time_1d

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-1d] {msg}", flush=True)


def test_c0_fp64_parity(gpu_lib):
    """Small workload in FP64: every field after 1000 steps, and E at two probes."""
    run = W.c0()
    _banner("c0 fp64")
    sim = B.Sim(run, precision=B.FP64, max_probes=4, probe_capacity=run.steps)
    orc = oracle_1d(run)
    g, o, gp, op = space_time_1d(sim, orc, run.steps, 100, [300, 500, 700])
    assert rel_l2(g, o) <= 1e-12
    assert rel_l2(gp, op) <= 1e-12
    assert rel_l2(sim.read(B.F_H), orc.H) <= 1e-12
    assert rel_l2(sim.read(B.F_J), orc.J) <= 1e-12
    assert rel_l2(sim.read(B.F_DF), orc.df) <= 1e-12


def test_c0_fp32_parity(gpu_lib):
    run = W.c0()
    _banner("c0 fp32")
    sim = B.Sim(run, precision=B.FP32, max_probes=4, probe_capacity=run.steps)
    orc = oracle_1d(run)
    g, o, gp, op = space_time_1d(sim, orc, run.steps, 100, [300, 500, 700])
    err = rel_l2(np.concatenate([g.ravel(), gp.ravel()]), np.concatenate([o.ravel(), op.ravel()]))
    _banner(f"c0 fp32 space-time rel L2 = {err:.3e}")
    assert err <= 1e-5
    assert rel_l2(sim.read(B.F_J), orc.J) <= 1e-5
    assert rel_l2(sim.read(B.F_DF), orc.df) <= 1e-5


@pytest.mark.parametrize("nv,tile", [(8, 32), (16, 64), (64, 96), (128, 256), (256, 32), (1024, 64)])
def test_ragged_tiles_parity(gpu_lib, nv, tile):
    """Plasma spread over several tiles with a ragged last tile, every lane layout of the
    kinetic kernel (lanes per cell 1..64, chunks per lane 1..2), both collision models."""
    run = W.slab_1d(777, nv, 130, 555, 1.1, 0.2, W.F_REF, 40, 700)
    run.ne[300:320] = 0.0          # a vacuum gap inside the plasma
    _banner(f"ragged nv={nv} tile={tile}")
    for prec, tol in ((B.FP64, 1e-12), (B.FP32, 1e-5)):
        for model in ("hard_sphere", "const"):
            run.nu_model = model
            sim = B.Sim(run, precision=prec, tile=tile)
            orc = oracle_1d(run)
            g, o, _, _ = space_time_1d(sim, orc, run.steps, 70, [])
            assert rel_l2(g, o) <= tol, (prec, model)
            assert rel_l2(sim.read(B.F_DF), orc.df) <= tol


def test_pec_and_vacuum_only(gpu_lib):
    """Degenerate cases: no plasma node at all, and PEC ends."""
    run = W.slab_1d(300, 16, 0, 0, 1.0, 0.1, W.F_REF, 50, 500, bc="pec")
    _banner("vacuum pec")
    sim = B.Sim(run, precision=B.FP64)
    orc = oracle_1d(run)
    g, o, _, _ = space_time_1d(sim, orc, run.steps, 50, [])
    assert run.plasma_cells == 0
    assert rel_l2(g, o) <= 1e-12
    assert sim.read(B.F_DF).size == 0


def test_c1_full_size_prefix_parity(gpu_lib):
    """Large workload at its full size (Nx=65536, Nv=512, FP32) in the launch shape the
    benchmark times: after 1500 steps the field has travelled at most 1500 nodes, so the
    oracle on the prefix [0, 1610] is exact there, and everything beyond stays zero."""
    run = W.c1()
    steps = 1500
    cut = run.src_node + steps + 10
    _banner("c1 full size prefix")
    sim = B.Sim(run, precision=B.FP32, max_probes=4, probe_capacity=steps)
    orc = oracle_1d(run, nx=cut)
    snaps = []
    g, o, gp, op = space_time_1d(sim, orc, steps, 250, [450, 700, 900], df_snaps=snaps)
    err = rel_l2(np.concatenate([g.ravel(), gp.ravel()]), np.concatenate([o.ravel(), op.ravel()]))
    _banner(f"c1 prefix space-time rel L2 = {err:.3e}")
    assert err <= 1e-5
    E = sim.read(B.F_E)
    assert np.all(E[cut + 1:] == 0.0)
    df = sim.read(B.F_DF).reshape(run.plasma_cells, run.nv)
    ncut = len(orc.cells)
    err_df = rel_l2(np.concatenate([a for a, _ in snaps]), np.concatenate([b for _, b in snaps]))
    _banner(f"c1 prefix F1 space-time rel L2 = {err_df:.3e}")
    assert err_df <= 1e-5
    assert np.all(df[ncut:] == 0.0)


def test_repeat_is_bitwise_and_resume_is_bitwise(gpu_lib):
    run = W.slab_1d(900, 64, 300, 600, 0.9, 0.1, W.F_REF, 60, 600)
    _banner("bitwise repeat / resume")
    a = B.Sim(run, precision=B.FP32)
    a.run(300)
    blob = a.save_state()
    a.run(300)
    b = B.Sim(run, precision=B.FP32)
    b.run(600)
    c = B.Sim(run, precision=B.FP32)
    c.load_state(blob)
    c.run(300)
    for f in (B.F_E, B.F_H, B.F_J, B.F_DF):
        assert np.array_equal(a.read(f), b.read(f))
        assert np.array_equal(a.read(f), c.read(f))
    assert c.steps == 600


def test_short_buffer_and_bad_field(gpu_lib):
    run = W.slab_1d(100, 8, 40, 60, 0.5, 0.1, W.F_REF, 20, 10)
    sim = B.Sim(run)
    import ctypes as C
    buf = np.zeros(5)
    rc = gpu_lib.fdtd_plasma_read_fields(sim.h, 0, B.F_E, buf.ctypes.data_as(C.POINTER(C.c_double)), 5, None)
    assert rc == B.ERANGE and np.all(buf == 0)
    rc = gpu_lib.fdtd_plasma_read_fields(sim.h, 0, B.F_EX, buf.ctypes.data_as(C.POINTER(C.c_double)), 5, None)
    assert rc == B.EINVAL


@pytest.mark.parametrize("nv,k", [(512, 3), (512, 5), (512, 7), (512, 9), (64, 5), (128, 3), (256, 7)])
def test_time_blocked_run_is_bitwise_the_stepped_run(gpu_lib, nv, k):
    """K steps per launch with halo recomputation against one step per launch: fields,
    current, F1, probe series and a non-multiple step count (remainder steps) must agree
    bit for bit."""
    run = W.c1(nx=6000 if nv == 512 else 12000, steps=1)
    run.nv = nv
    steps = 1201 + k          # the pulse reaches the plasma (node 400) after ~600 steps
    _banner(f"time block nv={nv} k={k}, {steps} steps")
    probes = [run.src_node, 450, 1000, 3000]
    sims = []
    for tb in (1, k):
        sim = B.Sim(run, precision=B.FP32, max_probes=len(probes) + 1, probe_capacity=steps,
                    time_block=tb)
        ids = [sim.add_probe(B.F_E, p) for p in probes] + [sim.add_probe(B.F_H, 2000)]
        sims.append((sim, ids))
    assert sims[0][0].time_block() == 1
    assert sims[1][0].time_block() == k, "the line should be long enough to be blocked"
    for sim, _ in sims:
        sim.run(steps // 2)
        sim.run(steps - steps // 2)
    (a, ia), (b, ib) = sims
    for f in (B.F_E, B.F_H, B.F_J, B.F_DF):
        assert np.array_equal(a.read(f), b.read(f)), f
    for p, q in zip(ia, ib):
        assert np.array_equal(a.read_probe(p, steps), b.read_probe(q, steps))
    assert np.max(np.abs(a.read(B.F_E))) > 1e-3
    assert np.max(np.abs(a.read(B.F_DF))) > 0.0


def test_time_block_rejects_even_and_reports_off_for_fp64(gpu_lib):
    run = W.c1(nx=6000, steps=1)
    sim = B.Sim(run, precision=B.FP64)
    with pytest.raises(B.FdtdError):
        sim.set_time_block(4)
    sim.set_time_block(5)
    assert sim.time_block() == 1


def test_blocked_launch_over_several_rounds_is_bitwise(gpu_lib):
    """The large line (Nx=65536: about three work-groups per resident slot) with the
    source moved next to the tiles where a launch's second and third rounds of
    work-groups begin: 9 steps per launch against one step per launch, bit for bit.  A
    work-group that starts after its neighbour finished must still see that neighbour's
    rows as they were at the launch's start (the rows are read from one copy and written
    to the other)."""
    for src in (21950, 43990):
        run = W.c1(steps=2000)
        run.src_node = src
        a = B.Sim(run, precision=B.FP32, time_block=9)
        b = B.Sim(run, precision=B.FP32, time_block=1)
        assert a.time_block() == 9
        _banner(f"rounds: source at {src}")
        for n in (450, 451):
            a.run(n)
            b.run(n)
            for f in (B.F_E, B.F_H, B.F_J, B.F_DF):
                assert np.array_equal(a.read(f), b.read(f)), (src, n, f)
        assert np.max(np.abs(b.read(B.F_DF))) > 0
        a.close()
        b.close()


@pytest.mark.parametrize("k", [5, 9])
def test_blocked_tiles_with_vacuum_gaps_are_bitwise_the_stepped_run(gpu_lib, k):
    """A single line of Nv = 512 at K steps per launch with the plasma in seeded
    segments of 1-80 nodes and vacuum gaps of 1-40 (rows and nodes no longer line up,
    tiles span several gaps, some halos hold no row), probes on both sides of gaps, and
    calls that end inside a block: against one step per launch, bit for bit."""
    run = W.c1(nx=9000, steps=1)
    g = np.random.default_rng(2211)
    keep = np.zeros(run.nx + 1, bool)
    i = 300
    while i < run.nx - 60:
        n = int(g.integers(1, 81))
        keep[i:i + n] = True
        i += n + int(g.integers(1, 41))
    run.ne = np.where(keep, np.where(run.ne > 0, run.ne, 1e17), 0.0)
    run.nubar = np.where(keep, np.where(run.nubar > 0, run.nubar, 1e9), 0.0)
    steps = 1300 + k
    probes = [run.src_node, 301, 2222, 4500, 8999]
    _banner(f"blocked tiles with gaps, k={k}, {steps} steps")
    sims = []
    for tb in (1, k):
        sim = B.Sim(run, precision=B.FP32, max_probes=len(probes) + 1, probe_capacity=steps,
                    time_block=tb)
        ids = [sim.add_probe(B.F_E, p) for p in probes] + [sim.add_probe(B.F_J, 2222)]
        sims.append((sim, ids))
    assert sims[1][0].time_block() == k
    for sim, _ in sims:
        sim.run(steps // 3)
        sim.run(steps - steps // 3)
    (a, ia), (b, ib) = sims
    for f in (B.F_E, B.F_H, B.F_J, B.F_DF):
        assert np.array_equal(a.read(f), b.read(f)), f
    for p, q in zip(ia, ib):
        assert np.array_equal(a.read_probe(p, steps), b.read_probe(q, steps))
    assert np.max(np.abs(a.read(B.F_DF))) > 0.0
