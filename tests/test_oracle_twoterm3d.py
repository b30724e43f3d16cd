"""Pins of the oracle's 3D two-term model: the paper's production representation (section
5.1 expansion F = F0 + (v/|v|).F1, l = 0 and l = 1 equations, section 5.3 speed grid) on
the Yee cube, with F0 of every plasma cell evolving under the l = 0 equation and the F1
vector held component by component at the E points whose four cells are plasma.

Facts checked: the field energy the current removes is exactly the kinetic energy the
cells' electrons gain, each cell keeps its electron number, the heating respects the
box's mirror symmetries (which pins which cells an edge heats), F0 evolution is second
order in the field, and an F0 that starts at another temperature drives F1 as the held
model built at that temperature does (which pins the F0 term of the F1 drive).
"""
import math

import numpy as np
import pytest

from oracle.core import Oracle3D, sgrid
import analytic as A

NX, NY, NZ = 8, 9, 10


def _box(kinetic, ne, nubar=0.0, nu_model="hard_sphere", f0="druyvesteyn", vdim=16,
         vmax=5.0, te=1.0, seed=4, amp=1e3, n=(NX, NY, NZ)):
    nx, ny, nz = n
    nu = np.where(ne > 0, nubar, 0.0)
    o = Oracle3D(nx, ny, nz, 1e-3, 0.5, ne, nu, vdim=vdim, vmax_over_vth=vmax, te_ev=te,
                 nu_model=nu_model, f0_model=f0, ncpml=0, kinetic=kinetic)
    g = np.random.default_rng(seed)
    F = o.fields()
    F["Ex"][1:-1, 1:-1, :] = amp * g.standard_normal(F["Ex"][1:-1, 1:-1, :].shape)
    F["Ey"][1:-1, :, 1:-1] = amp * g.standard_normal(F["Ey"][1:-1, :, 1:-1].shape)
    F["Ez"][:, 1:-1, 1:-1] = amp * g.standard_normal(F["Ez"][:, 1:-1, 1:-1].shape)
    return o


def _block_density(seed=4):
    ne = np.zeros((NZ, NY, NX))
    g = np.random.default_rng(seed)
    ne[1:8, 2:7, 1:7] = 1e18 * (0.5 + g.random((7, 5, 6)))
    return ne


@pytest.mark.parametrize("f0", ["maxwell", "druyvesteyn"])
@pytest.mark.parametrize("nu_model,nubar", [("hard_sphere", 0.0), ("hard_sphere", 3e11),
                                            ("const", 5e11)])
def test_energy_and_cell_number_exact(f0, nu_model, nubar):
    """eps0 |E^n|^2 / 2 + mu0 H^{n-1/2}.H^{n+1/2} / 2 + sum over cells (m/2) 4 pi gam
    sum v^4 (F0^n - n F0hat) is constant to rounding, and each cell's 4 pi gam sum v^2 F0
    does not move -- while with nu > 0 most of the field energy becomes heat."""
    o = _box("two_term", _block_density(), nubar=nubar, nu_model=nu_model, f0=f0)
    assert o.npoints > 100 and o.ncells == 7 * 5 * 6
    v, F0, dF0, gam, vth = sgrid(o.vdim, o.vmax, o.te, o.f0_model)
    tot, Wf0 = [], None
    for _ in range(250):
        En, Hlo = o.E.copy(), o.H.copy()
        d0 = o.f0_rows().copy()
        o.run(1)
        Wf = 0.5 * (A.EPS0 * np.sum(En ** 2) + A.MU0 * np.sum(Hlo * o.H))
        Kin = 0.5 * A.ME * 4 * math.pi * gam * np.sum(v ** 4 * d0)
        Wf0 = Wf if Wf0 is None else Wf0
        tot.append(Wf + Kin)
        dn = 4 * math.pi * gam * np.sum(v ** 2 * d0, axis=1)
        assert np.max(np.abs(dn)) < 1e-13 * o.ne.max()
    tot = np.array(tot)
    assert np.max(np.abs(tot - tot[0])) < 1e-12 * tot[0]
    assert Kin > 1e-3 * Wf0
    if nubar > 0:
        assert Wf < 0.85 * Wf0 and Kin > 0.1 * Wf0


def _mirror_e(o, axis):
    """Mirror image of E through the box's mid-plane normal to ``axis`` (E is a polar
    vector: the normal component flips sign)."""
    F = o.fields()
    out = {}
    for c, name in enumerate(("Ex", "Ey", "Ez")):
        a = F[name]
        ax = {0: 2, 1: 1, 2: 0}[axis]         # array axis of the mirrored coordinate
        out[name] = (-1.0 if c == axis else 1.0) * np.flip(a, axis=ax)
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_heating_keeps_the_mirror_symmetry(axis):
    """A box, density and initial field symmetric under the mirror normal to x, y or z
    heat mirror-image cells alike, and the heating is not uniform."""
    n = (8, 8, 8)
    g = np.random.default_rng(7)
    ne = np.zeros(n[::-1])
    ne[1:7, 1:7, 1:7] = 1e18 * (0.5 + g.random((6, 6, 6)))
    ax = {0: 2, 1: 1, 2: 0}[axis]
    ne = 0.5 * (ne + np.flip(ne, axis=ax))
    o = _box("two_term", ne, nubar=2e11, n=n, amp=3e3)
    m = _mirror_e(o, axis)
    F = o.fields()
    for name in ("Ex", "Ey", "Ez"):
        F[name][...] = 0.5 * (F[name] + m[name])
    o.run(150)
    v, F0, dF0, gam, vth = sgrid(o.vdim, o.vmax, o.te, o.f0_model)
    heat = np.zeros(n[::-1])
    heat.reshape(-1)[o.cells] = np.sum(v ** 4 * o.f0_rows(), axis=1)
    assert np.all(heat[ne > 0] > 0)
    assert heat.max() > 1.5 * heat[ne > 0].min()
    assert np.max(np.abs(heat - np.flip(heat, axis=ax))) < 1e-9 * heat.max()


def test_f0_evolution_is_second_order_in_the_field():
    """Against the run with F0 held the field differs by a relative amount that grows 4x
    when the amplitude doubles."""
    gaps = []
    for amp in (1e3, 2e3):
        a = _box("two_term", _block_density(), nubar=2e11, amp=amp)
        b = _box("two_term_frozen", _block_density(), nubar=2e11, amp=amp)
        a.run(200)
        b.run(200)
        gaps.append(np.linalg.norm(a.E - b.E) / np.linalg.norm(b.E))
    assert 0 < gaps[0] < 1e-3
    assert 3.8 < gaps[1] / gaps[0] < 4.2


@pytest.mark.parametrize("f0", ["maxwell", "druyvesteyn"])
def test_hotter_f0_drives_f1_as_the_model_built_hotter(f0):
    """Start the evolving model with F0 = n F0hat(T2) on the grid of F0hat(T1) (same
    speeds, a weak field so F0 barely moves): its fields follow the held model built at
    T2 (with the same collision frequencies per speed) far closer than they follow the
    one at T1 -- the F0 term of the F1 drive enters with its sign and its 1/(2 gam)."""
    t1, t2, vdim = 1.0, 1.44, 24
    vmo1 = 6.0
    vmo2 = vmo1 * math.sqrt(t1 / t2)          # same vmax, hence the same speed grid
    fm = {"maxwell": 0, "druyvesteyn": 1}[f0]
    v1, F01, _, gam1, vth1 = sgrid(vdim, vmo1, t1, fm)
    v2, F02, _, gam2, vth2 = sgrid(vdim, vmo2, t2, fm)
    assert abs(gam1 / gam2 - 1) < 1e-14
    mean = lambda v, F, g: np.sum(4 * math.pi * g * v ** 3 * F)
    nu1 = 3e11
    nu2 = nu1 * mean(v2, F02, gam2) / mean(v1, F01, gam1)   # equal nu at every speed
    ne = _block_density()

    def mk(kinetic, te, vmo, nub):
        return _box(kinetic, ne, nubar=nub, f0=f0, vdim=vdim, vmax=vmo, te=te, amp=1.0)

    hot = mk("two_term", t1, vmo1, nu1)
    n_cell = hot.ne[hot.cells]
    hot.f0_rows()[:] = n_cell[:, None] * (F02 - F01)[None, :]
    ref2 = mk("two_term_frozen", t2, vmo2, nu2)
    ref1 = mk("two_term_frozen", t1, vmo1, nu1)
    for o in (hot, ref1, ref2):
        o.run(300)
    d2 = np.linalg.norm(hot.J - ref2.J)
    d1 = np.linalg.norm(ref1.J - ref2.J)
    assert d1 > 0.02 * np.linalg.norm(ref2.J)
    assert d2 < 0.1 * d1
    # the slowest speed: F0 is even in v, so its difference below v_0 mirrors the one
    # above (dropping that reflection leaves F1 there off by 10x the T1-T2 gap or more)
    a = np.linalg.norm(hot.df_rows()[:, 0] - ref2.df_rows()[:, 0])
    b = np.linalg.norm(ref1.df_rows()[:, 0] - ref2.df_rows()[:, 0])
    assert a < {"maxwell": 0.5, "druyvesteyn": 10.0}[f0] * b


def _late_over_early(kinetic, in_cpml):
    """max |E| after 1500 steps of the slab's own pulse over max |E| at step 500, in a
    16 x 14 x 40 box with a 6-cell layer on every face."""
    from paper_2211_05647_amd import workloads as W
    run = W.argon_slab_3d(nx=16, ny=14, nz=40, nv=31, steps=0, ncpml=6, kinetic=kinetic,
                          plasma_in_cpml=in_cpml)
    o = Oracle3D(run.nx, run.ny, run.nz, run.dx, run.courant, run.ne, run.nubar,
                 vdim=run.nv, vmax_over_vth=run.vmax_over_vth, te_ev=run.te_ev,
                 nu_model=run.nu_model, f0_model=run.f0_model, ncpml=run.ncpml,
                 src_kind=run.src_kind, src_k=run.src_k, src_amp=run.src_amp,
                 src_f=run.src_f, src_tau=run.src_tau, src_t0=run.src_t0,
                 kinetic=kinetic)
    o.run(500)
    early = np.abs(o.E).max()
    o.run(1000)
    return np.abs(o.E).max() / early


def test_slab_kept_out_of_the_side_layers_decays():
    """Once the slab ends where the x and y absorbing layers begin (the 3D slab workload's
    default for the two-term model, and the only profile the library accepts for it), the
    field decays after the pulse has passed, with F0 evolving and with F0 held; the linear
    model's point set decays with the slab running on through those layers too."""
    assert _late_over_early("two_term", False) < 0.5
    assert _late_over_early("two_term_frozen", False) < 0.5
    assert _late_over_early("linear", True) < 0.5


@pytest.mark.xfail(strict=False, reason="open discretisation issue: the two-term point set "
                   "(E points with four plasma cells) with plasma inside the x and y "
                   "absorbing layers carries a growing mode (about 6x per 500 steps here); "
                   "the library refuses such profiles")
def test_slab_through_the_side_layers_stays_bounded():
    """Characterisation of the open issue, not a requirement: with plasma inside the side
    layers the two-term model should decay like the others.  It grows instead, so this is
    expected to fail until the treatment of the layer-plasma interface is fixed."""
    assert _late_over_early("two_term", True) < 0.5
