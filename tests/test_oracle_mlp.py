"""Pins of the learned-closure oracle (network, training step, recurrence, replay cells)
against library routines, finite differences, closed forms and the full kinetic oracle."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle.core import Oracle1D, replay1v, replay2v
from paper_2211_05647_amd import workloads as W
import analytic as A


def _batch(n=8, seed=0):
    g = np.random.default_rng(seed)
    return g.standard_normal((n, M.NIN)), g.standard_normal(n)


def test_parameter_count():
    assert M.NPARAM == 19073


def test_finite_difference_gradient():
    """Central differences of the FP64 loss agree with the manual backward pass."""
    p = M.init_params(1) + 0.05 * np.random.default_rng(2).standard_normal(M.NPARAM)
    X, t = _batch()
    loss, g = M.loss_and_grad(p, X, t)
    idx = np.random.default_rng(3).choice(M.NPARAM, 300, replace=False)
    idx = np.concatenate([idx, [M.NPARAM - 1, 0, M.NH * M.NIN + 5]])
    h = 1e-6
    num = np.empty(len(idx))
    for k, i in enumerate(idx):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        num[k] = (M.loss_and_grad(pp, X, t)[0] - M.loss_and_grad(pm, X, t)[0]) / (2 * h)
    scale = np.max(np.abs(g[idx]))
    assert np.max(np.abs(num - g[idx])) <= 1e-7 * scale + 1e-12


def test_bf16_matches_library_rounding():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(4)
    x = np.concatenate([g.standard_normal(10000) * 10.0 ** g.integers(-8, 8, 10000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)


def test_relu_matches_library():
    torch = pytest.importorskip("torch")
    x = np.concatenate([np.linspace(-8, 8, 2001), [0.0, -0.0, 1e-300, -1e-300]])
    ref = torch.nn.functional.relu(torch.tensor(x)).numpy()
    assert np.array_equal(M.relu(x), ref)
    # derivative: 1 above zero, 0 below, by central differences away from the kink, and
    # torch's own gradient everywhere (0 at x = 0)
    h = 1e-6
    xs = x[np.abs(x) > 1e-3]
    fd = (M.relu(xs + h) - M.relu(xs - h)) / (2 * h)
    assert np.max(np.abs(fd - M.relu_grad(xs))) < 1e-9
    t = torch.tensor(x, requires_grad=True)
    torch.nn.functional.relu(t).sum().backward()
    assert np.array_equal(M.relu_grad(x), t.grad.numpy())


def test_adam_matches_library():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(5)
    p0 = g.standard_normal(50)
    tgt = g.standard_normal(50)
    opt = M.Adam(50)
    p = p0.copy()
    tp = torch.tensor(p0.copy(), requires_grad=True)
    topt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(20):
        grad = 2 * (p - tgt) * (1 + p ** 2)
        p = opt.step(p, grad, 1e-2)
        topt.zero_grad()
        tp.grad = 2 * (tp.detach() - torch.tensor(tgt)) * (1 + tp.detach() ** 2)
        topt.step()
    assert np.max(np.abs(p - tp.detach().numpy())) < 1e-12


def test_bf16_emulation_changes_little():
    p = M.init_params(6)
    X, t = _batch(64, 7)
    y64 = M.forward(p, X)[0]
    y16 = M.forward(p, X, emulate_bf16=True)[0]
    assert 0 < np.max(np.abs(y64 - y16)) < 3e-2 * np.max(np.abs(y64))


def _drive(n, dt, f=W.F_REF):
    t = (np.arange(n) + 1) * dt
    p = W.pulse(f)
    return np.sin(2 * math.pi * f * (t - p["src_t0"])) * np.exp(-((t - p["src_t0"]) / p["src_tau"]) ** 2)


def test_closure_without_network_is_kinetic_at_constant_nu():
    """Section 5.2 F1 model with nu independent of v: the closure with y = 0 (one pole
    with the w-weighted weights) reproduces the kinetic cell current exactly."""
    dt = 0.5 * W.DX_REF / A.C0
    ne = W.density_from_ratio(0.9, W.F_REF)
    nubar = 0.07 * 2 * math.pi * W.F_REF
    E = _drive(1500, dt)
    Jk = replay1v(E, ne, nubar, dt, nv=64, nu_model="const") * dt / A.EPS0
    w, s = A.velocity_weights(64, 6.0, 2.0, "const")
    al, be = M.effective_pole(w, s, nubar, A.plasma_omega2(ne), dt)
    Jc = M.closure_run(E, al, be)
    assert np.max(np.abs(Jc - Jk)) < 1e-12 * np.max(np.abs(Jk))


def test_closure_without_network_differs_for_hard_sphere():
    """With nu proportional to |v| the kinetic response is not a single pole: the y = 0
    closure is close but not equal -- the gap the network is trained to close."""
    dt = 0.5 * W.DX_REF / A.C0
    ne = W.density_from_ratio(0.9, W.F_REF)
    nubar = 0.3 * 2 * math.pi * W.F_REF
    E = _drive(1500, dt)
    Jk = replay1v(E, ne, nubar, dt, nv=64) * dt / A.EPS0
    w, s = A.velocity_weights(64, 6.0, 2.0, "hard_sphere")
    al, be = M.effective_pole(w, s, nubar, A.plasma_omega2(ne), dt)
    Jc = M.closure_run(E, al, be)
    rel = np.max(np.abs(Jc - Jk)) / np.max(np.abs(Jk))
    assert 1e-4 < rel < 0.2


def test_targets_make_closure_exact():
    """Feeding the closure the target output at every step reproduces the kinetic current."""
    dt = 0.5 * W.DX_REF / A.C0
    ne = W.density_from_ratio(1.3, W.F_REF)
    nubar = 0.2 * 2 * math.pi * W.F_REF
    E = _drive(600, dt)
    Jk = replay1v(E, ne, nubar, dt, nv=64) * dt / A.EPS0
    w, s = A.velocity_weights(64, 6.0, 2.0, "hard_sphere")
    al, be = M.effective_pole(w, s, nubar, A.plasma_omega2(ne), dt)
    hist = np.zeros(M.HIST)
    jp, out = 0.0, []
    for n in range(len(E)):
        hist = np.concatenate([[E[n]], hist[:-1]])
        sc = max(np.max(np.abs(hist)), 1e-30)
        y = M.targets(jp, Jk[n], E[n], sc, al, be)
        jp = al * jp + be * (E[n] + sc * y)
        out.append(jp)
    assert np.max(np.abs(np.array(out) - Jk)) < 1e-10 * np.max(np.abs(Jk))


def test_replay1v_reproduces_the_coupled_oracle():
    """The isolated 1V cell driven by the E^n a coupled run saw at a plasma node returns
    exactly that node's J^{n+1/2}."""
    run = W.slab_1d(500, 64, 200, 300, 0.8, 0.1, W.F_REF, 50, 700)
    o = Oracle1D(run.nx, run.dx, run.courant, run.ne, run.nubar, nv=run.nv, te_ev=run.te_ev,
                 src_node=run.src_node, src_amp=1.0, src_f=run.src_f, src_tau=run.src_tau,
                 src_t0=run.src_t0)
    node = 230
    E, J = [], []
    for _ in range(run.steps):
        E.append(o.E[node])
        o.run(1)
        J.append(o.J[node])
    Jr = replay1v(np.array(E), run.ne[node], run.nubar[node], o.dt, nv=run.nv)
    assert np.max(np.abs(Jr - np.array(J))) <= 1e-14 * np.max(np.abs(J))


def test_replay2v_const_nu_is_drude():
    """2V cell with constant nu: each current component is a Drude pole with
    wp~^2 = wp^2 sum_ab vx_a^2 fhat_a fhat_b dv^2 / vth^2, and x and y decouple."""
    dt = 0.5 * W.DX_REF / A.C0
    ne = W.density_from_ratio(1.1, W.F_REF)
    nubar = 0.05 * 2 * math.pi * W.F_REF
    Ex = _drive(800, dt)
    Ey = 0.3 * _drive(800, dt, 1.2 * W.F_REF)
    Jx, Jy = replay2v(Ex, Ey, ne, nubar, dt, nv=16, nu_model="const")
    w, s = A.velocity_weights(16, 6.0, 5.0, "const", dims=2)
    al, be = M.effective_pole(w, s, nubar, A.plasma_omega2(ne), dt)
    jx = M.closure_run(Ex, al, be) * A.EPS0 / dt
    jy = M.closure_run(Ey, al, be) * A.EPS0 / dt
    assert np.max(np.abs(Jx - jx)) < 1e-12 * np.max(np.abs(jx))
    assert np.max(np.abs(Jy - jy)) < 1e-12 * np.max(np.abs(jy))


def test_c_and_numpy_networks_agree():
    """The oracle's two independent network codes (plain C loops and numpy matmuls) agree,
    with and without bf16 operand emulation."""
    from oracle.core import mlp as cmlp
    p = M.init_params(11) + 0.02 * np.random.default_rng(12).standard_normal(M.NPARAM)
    X, _ = _batch(20, 13)
    for bf in (False, True):
        ref = M.forward(p, X, emulate_bf16=bf)[0]
        got = np.array([cmlp(p, x, bf) for x in X])
        assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_2d_closure_without_network_is_kinetic_at_constant_nu():
    """2D oracle: cells switched to the closure with a zero network and the const-nu single
    pole evolve exactly as kinetic cells (section 5.2 model with nu independent of v)."""
    from oracle.core import Oracle2D
    nx, ny, nv = 48, 40, 8
    ne = np.zeros((ny, nx))
    nu = np.zeros((ny, nx))
    jj, ii = np.mgrid[0:ny, 0:nx]
    blob = (ii - 27.5) ** 2 + (jj - 19.5) ** 2 < 81
    ne[blob] = W.density_from_ratio(1.2, W.F_REF)
    nu[blob] = 0.1 * 2 * math.pi * W.F_REF
    kw = dict(nv=nv, te_ev=5.0, ncpml=0, nu_model="const", src_kind=2, src_i=10, src_j=20,
              **W.pulse(W.F_REF))
    kin = Oracle2D(nx, ny, W.DX_REF, 0.5, ne, nu, **kw)
    clo = Oracle2D(nx, ny, W.DX_REF, 0.5, ne, nu, **kw)
    w, s = A.velocity_weights(nv, 6.0, 5.0, "const", dims=2)
    coef = []
    for c in clo.cells:
        a, b = M.effective_pole(w, s, clo.nubar[c], A.plasma_omega2(clo.ne[c]), clo.dt)
        coef.append((a, b, 0.0, 0.0))
    clo.set_closure(np.ones(len(clo.cells)), np.array(coef), np.zeros(M.NPARAM), emulate_bf16=False)
    kin.run(400)
    clo.run(400)
    assert np.max(np.abs(clo.Ey - kin.Ey)) < 1e-12 * np.max(np.abs(kin.Ey))
    assert np.max(np.abs(clo.Jx - kin.Jx)) < 1e-11 * np.max(np.abs(kin.Jx))
