"""Pins of the oracle's 1D two-term model: the paper's own representation (section 5.1
expansion F = F0 + (v/|v|).F1 with the l = 0 and l = 1 equations, section 5.3 speed grid)
with the field along the line, F0 evolving under the l = 0 equation.

Facts checked: the field energy the current removes is exactly the kinetic energy the
electrons gain (also with collisions, which only turn F1 around), the electron number of
every node is kept, F0 evolution is a second-order effect of the field, and with F0 held
and a constant collision frequency the current is a Drude current whose plasma frequency
tends to e^2 n / (eps0 m) as the speed grid is refined.
"""
import math

import numpy as np
import pytest

from oracle.core import Oracle1D, sgrid
from paper_2211_05647_amd import workloads as W
import analytic as A


def _cavity(kinetic, f0="druyvesteyn", nu_model="hard_sphere", nu_ratio=0.3, amp=1e3, vdim=31):
    nx = 120
    ne, nu = np.zeros(nx + 1), np.zeros(nx + 1)
    ne[40:80] = W.density_from_ratio(np.linspace(0.8, 1.2, 40), W.F_REF)
    nu[40:80] = nu_ratio * 2 * math.pi * W.F_REF
    o = Oracle1D(nx, W.DX_REF, 0.5, ne, nu, nv=vdim, vmax_over_vth=5.0, te_ev=1.0, bc="pec",
                 kinetic=kinetic, f0_model=f0, nu_model=nu_model)
    o.E[1:-1] = amp * np.sin(3 * math.pi * np.arange(1, nx) / nx)
    return o


@pytest.mark.parametrize("f0", ["maxwell", "druyvesteyn"])
@pytest.mark.parametrize("nu_model,nu_ratio", [("hard_sphere", 0.0), ("hard_sphere", 0.3),
                                               ("const", 0.5)])
def test_energy_and_number_exact(f0, nu_model, nu_ratio):
    """Field energy at level n (eps0 |E^n|^2 + mu0 H^{n-1/2} H^{n+1/2}, halved) plus the
    electrons' (m/2) 4 pi gam sum v^4 F0^n is constant to rounding, and so is each node's
    4 pi gam sum v^2 F0 -- while most of the field energy ends up as heat when nu > 0."""
    o = _cavity("two_term", f0=f0, nu_model=nu_model, nu_ratio=nu_ratio)
    v, F0, dF0, gam, vth = sgrid(o.nv, o.vmax, o.te, o.f0_model)
    nv = o.nv
    tot, Wf0 = [], None
    for _ in range(500):
        En, Hlo = o.E.copy(), o.H.copy()
        d0 = o.df_rows()[:, nv:].copy()
        o.run(1)
        Wf = 0.5 * (A.EPS0 * np.sum(En ** 2) + A.MU0 * np.sum(Hlo * o.H))
        K = 0.5 * A.ME * 4 * math.pi * gam * np.sum(v ** 4 * d0)
        Wf0 = Wf if Wf0 is None else Wf0
        tot.append(Wf + K)
        n_change = 4 * math.pi * gam * np.sum(v ** 2 * d0, axis=1)
        assert np.max(np.abs(n_change)) < 1e-13 * np.max(o.ne)
    tot = np.array(tot)
    assert np.max(np.abs(tot - tot[0])) < 1e-13 * tot[0]
    if nu_ratio > 0:
        assert Wf < 0.3 * Wf0                 # the wave has turned mostly into heat
    assert np.max(np.abs(o.df_rows()[:, nv:])) > 0


def test_f0_evolution_is_second_order_in_the_field():
    """Against the same run with F0 held, the field differs by a relative amount that
    grows 4x when the amplitude doubles (F0 - n F0hat grows as E^2, so its effect on the
    current, relative to the linear response, as E^2)."""
    gaps = []
    for amp in (1e3, 2e3):
        a, b = _cavity("two_term", amp=amp), _cavity("two_term_frozen", amp=amp)
        a.run(400)
        b.run(400)
        gaps.append(np.linalg.norm(a.E - b.E) / np.linalg.norm(b.E))
    assert 0 < gaps[0] < 1e-3
    assert 3.8 < gaps[1] / gaps[0] < 4.2


def test_held_f0_const_nu_is_a_drude_current():
    """F0 held, nu independent of v: the current obeys the Drude recurrence
    J^{n+1/2} = a J^{n-1/2} + b E^n (an independent Drude FDTD written here) with the
    plasma frequency scaled by S = (4 pi / 3) gam sum w_k (-dF0/dv), S -> 1 as the speed
    grid is refined (second order)."""
    run = W.slab_1d(600, 31, 250, 350, 0.9, 0.05, W.F_REF, 60, 900, nu_model="const")
    o = Oracle1D(run.nx, run.dx, run.courant, run.ne, run.nubar, nv=31, vmax_over_vth=5.0,
                 te_ev=1.0, nu_model="const", src_node=run.src_node, src_amp=1.0,
                 src_f=run.src_f, src_tau=run.src_tau, src_t0=run.src_t0,
                 kinetic="two_term_frozen", f0_model="druyvesteyn")
    o.run(run.steps)

    def S_of(vdim, vmax):
        v, F0, dF0, gam, vth = sgrid(vdim, vmax, 1.0, 1)
        faces = np.arange(vdim + 1) * gam
        cube = faces ** 3
        cube[-1] = 0.0                        # no flux through vmax
        w = 0.5 * (cube[:-1] + cube[1:])
        return (4 * math.pi / 3) * gam * np.sum(w * -dF0)

    S = S_of(31, 5.0)
    wp2 = A.plasma_omega2(run.ne) * S
    dt = run.courant * run.dx / A.C0
    E, H, J = np.zeros(run.nx + 1), np.zeros(run.nx), np.zeros(run.nx + 1)
    q = (A.C0 * dt - run.dx) / (A.C0 * dt + run.dx)
    al = (2 - dt * run.nubar) / (2 + dt * run.nubar)
    be = 2 * dt * A.EPS0 * wp2 / (2 + dt * run.nubar)
    for n in range(run.steps):
        H += dt / (A.MU0 * run.dx) * np.diff(E)
        J = al * J + be * E
        e0, e1, en1, en = E[0], E[1], E[-2], E[-1]
        E[1:-1] += dt / (A.EPS0 * run.dx) * np.diff(H) - dt / A.EPS0 * J[1:-1]
        E[0] = e1 + q * (E[1] - e0)
        E[-1] = en1 + q * (E[-2] - en)
        t = (n + 1) * dt - run.src_t0
        E[run.src_node] += math.sin(2 * math.pi * run.src_f * t) * math.exp(-(t / run.src_tau) ** 2)
    assert np.max(np.abs(o.E - E)) < 1e-12 * np.max(np.abs(E))
    assert np.max(np.abs(o.J - J)) < 1e-11 * np.max(np.abs(J))
    # S -> 1: the error falls 4x per doubling of the speed count at a fixed vmax far out
    errs = [abs(S_of(n, 8.0) - 1) for n in (64, 128, 256)]
    assert errs[0] < 1e-2
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.5 < e0 / e1 < 4.5


def test_heating_keeps_f0_positive_and_raises_the_mean_energy():
    """With collisions the driven electrons' F0 widens: the mean energy per electron rises
    and F0 stays positive on the grid."""
    o = _cavity("two_term", nu_ratio=0.3, amp=3e4)
    v, F0, dF0, gam, vth = sgrid(o.nv, o.vmax, o.te, o.f0_model)
    o.run(600)
    n = o.ne[o.cells]
    f0 = n[:, None] * F0[None, :] + o.df_rows()[:, o.nv:]
    assert np.all(f0 > -1e-9 * f0.max())
    e_mean = np.sum(v ** 4 * f0, axis=1) / np.sum(v ** 2 * f0, axis=1)
    e_init = np.sum(v ** 4 * F0) / np.sum(v ** 2 * F0)
    assert np.all(e_mean > e_init)
    assert np.max(e_mean / e_init) > 1.01
