"""CPU-side checks of the C ABI: the library loads, exports every entry point the
headers declare, and rejects bad problem statements without touching a device."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(fdtd_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared()
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(L, n), n
    # and the binding declares a signature for each of them
    assert names <= set(B._SIGS), names - set(B._SIGS)


def _grid_profile(run, precision=B.FP32):
    g = B.make_grid(1, run.nx, 1, run.dx, run.courant, precision, B.BC_MUR1, 0)
    ne = np.ascontiguousarray(run.ne)
    nu = np.ascontiguousarray(run.nubar)
    p = B.Profile(ne.ctypes.data_as(C.POINTER(C.c_double)), nu.ctypes.data_as(C.POINTER(C.c_double)),
                  run.te_ev, run.nv, run.vmax_over_vth, 0, 0, None)
    return g, p, (ne, nu)


def test_workspace_size_scales_with_problem():
    L = B.lib()
    run = W.c0()
    g, p, keep = _grid_profile(run, B.FP64)
    n64 = C.c_size_t()
    assert L.fdtd_plasma_workspace_size(C.byref(g), C.byref(p), None, C.byref(n64)) == 0
    g.precision = B.FP32
    n32 = C.c_size_t()
    assert L.fdtd_plasma_workspace_size(C.byref(g), C.byref(p), None, C.byref(n32)) == 0
    # F1 dominates: 200 nodes x 32 stored bins x 8 or 4 bytes
    assert n64.value > n32.value > 200 * 32 * 4


@pytest.mark.parametrize("mutate", [
    lambda g, p: setattr(g, "courant", 1.5),
    lambda g, p: setattr(g, "courant", 0.0),
    lambda g, p: setattr(g, "nx", 4),
    lambda g, p: setattr(g, "dx", -1.0),
    lambda g, p: setattr(g, "precision", 7),
    lambda g, p: setattr(g, "boundary", B.BC_CPML),
    lambda g, p: setattr(p, "nv", 48),
    lambda g, p: setattr(p, "nv", 4),
    lambda g, p: setattr(p, "te_ev", 0.0),
    lambda g, p: setattr(p, "nu_model", 9),
    lambda g, p: setattr(p, "closure", B.CLOSURE_MLP),
])
def test_bad_problem_statements_are_rejected(mutate):
    L = B.lib()
    run = W.c0()
    g, p, keep = _grid_profile(run)
    mutate(g, p)
    n = C.c_size_t(12345)
    rc = L.fdtd_plasma_workspace_size(C.byref(g), C.byref(p), None, C.byref(n))
    assert rc == B.EINVAL
    assert n.value == 12345
    assert len(L.fdtd_plasma_last_error()) > 0


@pytest.mark.parametrize("models,ok", [
    ((B.KINETIC_LINEAR, B.KINETIC_LINEAR), True),
    ((B.KINETIC_FULL, B.KINETIC_FULL), True),
    ((B.KINETIC_LINEAR, B.KINETIC_FULL), False),
    ((B.KINETIC_TWO_TERM, B.KINETIC_TWO_TERM), True),
    ((B.KINETIC_FULL, B.KINETIC_TWO_TERM), False),
])
def test_batch_kinetic_models(models, ok):
    """A batch takes runs of one kinetic model (checked before any device is touched, by
    the workspace-size call)."""
    L = B.lib()
    run = W.c0()
    gs, ps, keep = [], [], []
    for m in models:
        g, p, k = _grid_profile(run)
        p.kinetic = m
        gs.append(g)
        ps.append(p)
        keep.append(k)
    ga = (B.Grid * len(gs))(*gs)
    pa = (B.Profile * len(ps))(*ps)
    steps = (C.c_int64 * len(gs))(*([100] * len(gs)))
    n = C.c_size_t(0)
    rc = L.fdtd_plasma_workspace_size_batch(len(gs), ga, pa, steps, 0, None, C.byref(n))
    assert (rc == 0) == ok, (models, rc, L.fdtd_plasma_last_error())
    if ok:
        assert n.value > 0


def test_plasma_at_the_ends_is_rejected():
    L = B.lib()
    run = W.c0()
    run.ne[1] = 1e18
    g, p, keep = _grid_profile(run)
    n = C.c_size_t()
    assert L.fdtd_plasma_workspace_size(C.byref(g), C.byref(p), None, C.byref(n)) == B.EINVAL


def test_negative_density_is_rejected():
    L = B.lib()
    run = W.c0()
    run.ne[500] = -1.0
    g, p, keep = _grid_profile(run)
    n = C.c_size_t()
    assert L.fdtd_plasma_workspace_size(C.byref(g), C.byref(p), None, C.byref(n)) == B.EINVAL


def test_strerror_names_every_code():
    L = B.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.fdtd_plasma_strerror(code).decode() != "unknown error"
    assert L.fdtd_plasma_strerror(-99).decode() == "unknown error"


def test_seeded_workloads_are_reproducible():
    a, b = W.c1(nx=4096, steps=10), W.c1(nx=4096, steps=10)
    assert np.array_equal(a.ne, b.ne) and np.array_equal(a.nubar, b.nubar)
    r = a.ne[400:a.nx - 100]
    ratio = np.sqrt(r * W._QE ** 2 / (W._EPS0 * W._ME)) / (2 * np.pi * W.F_REF)
    assert 0.2 <= ratio.min() and ratio.max() <= 2.0
    runs = W.c3()
    assert len(runs) == 256 and {x.nv for x in runs} == {64, 128, 256}
    assert all(500 <= x.nx <= 20000 and x.steps == 2 * x.nx for x in runs)


def test_two_term_slab_stays_out_of_the_side_layers():
    """The 3D slab runs through the x and y absorbing layers for the linear model and stops
    where they begin for the two-term model (whose point set grows a mode with plasma in
    them); the slab's cells inside the box are the same in both."""
    m = 6
    lin = W.argon_slab_3d(nx=20, ny=18, nz=48, ncpml=m, steps=0)
    tt = W.argon_slab_3d(nx=20, ny=18, nz=48, ncpml=m, steps=0, kinetic="two_term")
    k0, k1 = lin.meta["slab"]
    assert np.all(lin.ne[k0:k1] > 0)
    side = np.ones(lin.ne.shape[1:], bool)
    side[m:-m, m:-m] = False
    assert np.all(tt.ne[:, side] == 0) and np.all(tt.nubar[:, side] == 0)
    assert np.array_equal(tt.ne[:, ~side], lin.ne[:, ~side])
    forced = W.argon_slab_3d(nx=20, ny=18, nz=48, ncpml=m, steps=0, kinetic="two_term",
                             plasma_in_cpml=True)
    assert np.array_equal(forced.ne, lin.ne)


def _grid_profile_3d(run, precision=B.FP32):
    g = B.make_grid(3, run.nx, run.ny, run.dx, run.courant, precision, B.BC_CPML, run.ncpml,
                    nz=run.nz)
    ne = np.ascontiguousarray(run.ne, dtype=np.float64)
    nu = np.ascontiguousarray(run.nubar, dtype=np.float64)
    p = B.Profile(ne.ctypes.data_as(C.POINTER(C.c_double)), nu.ctypes.data_as(C.POINTER(C.c_double)),
                  run.te_ev, run.nv, run.vmax_over_vth, B.NU_HARD_SPHERE, B.CLOSURE_KINETIC, None,
                  B.KINETIC_TWO_TERM, B.F0_DRUYVESTEYN)
    return g, p, (ne, nu)


@pytest.mark.parametrize("where", ["x_low", "x_high", "y_low", "y_high"])
def test_two_term_3d_plasma_in_the_side_layers_is_refused(where):
    """The 3D two-term model refuses plasma inside the x or y absorbing layers (its point
    set grows a mode there until the fields overflow) before touching a device, both when
    sizing the workspace and at create; a single plasma cell in a layer is enough, and the
    same box with that cell emptied is accepted."""
    L = B.lib()
    m = 6
    run = W.argon_slab_3d(nx=20, ny=18, nz=48, ncpml=m, steps=0, kinetic="two_term")
    k0, _ = run.meta["slab"]
    g, p, keep = _grid_profile_3d(run)
    n = C.c_size_t()
    assert L.fdtd_plasma_workspace_size(C.byref(g), C.byref(p), None, C.byref(n)) == B.OK
    j, i = {"x_low": (9, m - 1), "x_high": (9, run.nx - m), "y_low": (m - 1, 10),
            "y_high": (run.ny - m, 10)}[where]
    assert run.ne[k0, j, i] == 0.0
    run.ne[k0, j, i] = W.ARGON_NE
    g, p, keep = _grid_profile_3d(run)
    n = C.c_size_t(777)
    assert L.fdtd_plasma_workspace_size(C.byref(g), C.byref(p), None, C.byref(n)) == B.EINVAL
    assert n.value == 777
    assert b"absorbing" in L.fdtd_plasma_last_error()
    h = C.c_void_p()
    src = B.Source(B.SRC_NONE, 0, 0, 0.0, 0.0, 0.0, 0.0, 0)
    assert L.fdtd_plasma_create(C.byref(g), C.byref(p), C.byref(src), None, C.byref(h)) == B.EINVAL
    assert not h.value
    # the linear model takes the same profile (its point set does not grow there)
    p.kinetic = B.KINETIC_LINEAR
    assert L.fdtd_plasma_workspace_size(C.byref(g), C.byref(p), None, C.byref(n)) == B.OK


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the size and field offsets the C
    compiler gives the header's structs (a field added on one side only would shift every
    later field silently)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"fdtd_grid": B.Grid, "fdtd_profile": B.Profile, "fdtd_source": B.Source,
               "fdtd_device": B.Device}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fdtd_plasma.h"',
             'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
