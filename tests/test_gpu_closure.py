"""GPU parity of the learned-closure kernels (BF16 MFMA forward/backward, Adam, 2V replay
cells, training-pair assembly) against the FP64 oracle with BF16 operand emulation."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle.core import replay2v
from paper_2211_05647_amd import binding as B
from paper_2211_05647_amd import workloads as W
from parity import rel_l2
import analytic as A

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-closure] {msg}", flush=True)


def _params(seed=1):
    g = np.random.default_rng(seed)
    p = M.init_params(seed)
    p[M.NH * M.NIN:M.NH * M.NIN + M.NH] = 0.1 * g.standard_normal(M.NH)          # b1
    off = M.NH * M.NIN + M.NH + M.NH * M.NH
    p[off:off + M.NH] = 0.1 * g.standard_normal(M.NH)                             # b2
    p[-1] = 0.05
    return p.astype(np.float32).astype(np.float64)


def _rows(n, seed=2):
    g = np.random.default_rng(seed)
    X = g.uniform(-1, 1, (n, M.NIN))
    T = g.standard_normal(n) * 0.3
    return X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("n", [64, 1000, 4096])
def test_forward_matches_oracle(gpu_lib, n):
    import torch
    _banner(f"forward n={n}")
    p = _params()
    X, _ = _rows(n)
    c = B.Closure(max_rows=4096)
    c.set_params(p)
    y = c.forward(torch.tensor(X, dtype=torch.float32, device="cuda")).cpu().numpy()
    ref = M.forward(p, X, emulate_bf16=True)[0]
    assert rel_l2(y, ref) <= 1e-3
    ref64 = M.forward(p, X)[0]
    _banner(f"forward rel err vs bf16 oracle {rel_l2(y, ref):.2e}, vs fp64 {rel_l2(y, ref64):.2e}")


@pytest.mark.parametrize("n", [64, 640, 4096])
def test_gradient_matches_oracle(gpu_lib, n):
    import torch
    _banner(f"gradient n={n}")
    p = _params(3)
    X, T = _rows(n, 4)
    c = B.Closure(max_rows=4096)
    c.set_params(p)
    loss, g = c.grad(torch.tensor(X, dtype=torch.float32, device="cuda"),
                     torch.tensor(T, dtype=torch.float32, device="cuda"))
    lref, gref = M.loss_and_grad(p, X, T, emulate_bf16=True)
    assert abs(loss / lref - 1) <= 1e-3
    W1, b1, W2, b2, w3, b3 = M.unpack(gref)
    G1, c1, G2, c2, g3, c3 = M.unpack(g.astype(np.float64))
    for name, a, b in (("W1", G1, W1), ("b1", c1, b1), ("W2", G2, W2), ("b2", c2, b2),
                       ("w3", g3, w3)):
        err = rel_l2(a, b)
        _banner(f"  {name}: rel L2 {err:.2e}")
        assert err <= 1e-3, name
    assert abs(c3 - b3) <= 1e-3 * abs(b3) + 1e-7


def test_adam_step_matches_oracle(gpu_lib):
    import torch
    p = _params(5)
    X, T = _rows(512, 6)
    c = B.Closure(max_rows=4096)
    c.set_params(p)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Td = torch.tensor(T, dtype=torch.float32, device="cuda")
    opt = M.Adam(M.NPARAM)
    q = p.copy()
    for it in range(3):
        _, g = c.grad(Xd, Td)
        c.adam(1e-3)
        q = opt.step(q, g.astype(np.float64), 1e-3)
    got = c.get_params().astype(np.float64)
    assert np.max(np.abs(got - q)) <= 1e-6 * max(1.0, np.max(np.abs(q)))


def test_training_lowers_the_loss(gpu_lib):
    import torch
    p = _params(7)
    g = np.random.default_rng(8)
    X = g.uniform(-1, 1, (4096, M.NIN))
    T = np.sin(2 * X[:, 0]) * X[:, 16] + 0.5 * X[:, 3] * X[:, 5]
    c = B.Closure(max_rows=4096)
    c.set_params(p)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Td = torch.tensor(T, dtype=torch.float32, device="cuda")
    l0 = c.train_step(Xd, Td, 1e-3, want_loss=True)
    for _ in range(300):
        c.train_step(Xd, Td, 1e-3)
    l1 = c.train_step(Xd, Td, 1e-3, want_loss=True)
    _banner(f"loss {l0:.3e} -> {l1:.3e}")
    assert l1 < 0.2 * l0


def test_replay2v_and_pairs_match_oracle(gpu_lib):
    """Isolated 2V cells driven by a recorded field give the oracle's current; pairs built
    from them give the oracle's features and targets."""
    import torch
    dt = 0.5 * W.DX_REF / A.C0
    nsteps, nser = 900, 3
    t = (np.arange(nsteps) + 1) * dt
    pulse = W.pulse(W.F_REF)
    E = np.stack([np.sin(2 * math.pi * W.F_REF * f * (t - pulse["src_t0"])) *
                  np.exp(-((t - pulse["src_t0"]) / pulse["src_tau"]) ** 2) for f in (0.8, 1.0, 1.25)])
    E = E.astype(np.float32).astype(np.float64)
    ne = W.density_from_ratio(np.array([0.5, 1.1, 1.6]), W.F_REF)
    nu = np.array([0.02, 0.2, 0.8]) * 2 * math.pi * W.F_REF
    c = B.Closure(max_rows=4096, max_series=16)
    Ed = torch.tensor(E, dtype=torch.float32, device="cuda")
    Jd = torch.zeros((nser, nsteps), dtype=torch.float32, device="cuda")
    c.replay2v(Ed.data_ptr(), 1, nsteps, nser, nsteps, ne, nu, 5.0, dt, Jd, nsteps)
    J = Jd.cpu().numpy()
    for s in range(nser):
        Jx, _ = replay2v(E[s], np.zeros(nsteps), ne[s], nu[s], dt, nv=32, te_ev=5.0)
        err = rel_l2(J[s], Jx * dt / A.EPS0)
        _banner(f"replay series {s}: rel L2 {err:.2e}")
        assert err <= 1e-5
    # pairs
    ser = []
    box = (0.0, 0.3, -4.0, 0.0)
    for s in range(nser):
        a, b = B.single_pole(2, 32, 5.0, "hard_sphere", ne[s], nu[s], dt)
        wp_dt = math.sqrt(A.plasma_omega2(ne[s])) * dt
        q1, q2 = M.scale_params(wp_dt, nu[s] * dt, box)
        ser.append((a, b, q1, q2))
    g = np.random.default_rng(9)
    sidx = g.integers(0, nser, 500)
    nidx = g.integers(15, nsteps, 500)
    idx = (sidx.astype(np.int64) << 32) | nidx
    X, T = c.make_pairs(Ed.data_ptr(), 1, nsteps, Jd, nsteps, np.array(ser), idx)
    X, T = X.cpu().numpy(), T.cpu().numpy()
    Jn = J.astype(np.float64)
    for k in range(0, 500, 7):
        s, n = sidx[k], nidx[k]
        hist = E[s, n - np.arange(16)]
        Xr, sc = M.features(hist[None, :], math.sqrt(A.plasma_omega2(ne[s])) * dt, nu[s] * dt, box)
        assert np.max(np.abs(X[k] - Xr[0])) <= 2e-6
        a, b = ser[s][0], ser[s][1]
        tr = M.targets(Jn[s, n - 1], Jn[s, n], E[s, n], sc[0], a, b)
        assert abs(T[k] - tr) <= 1e-4 * max(1.0, abs(tr))


def test_single_pole_matches_oracle():
    """Library single-pole parameters equal the oracle's effective pole."""
    lib = B.lib()
    dt = 0.5 * W.DX_REF / A.C0
    for dims, nv in ((1, 64), (2, 32)):
        w, s = A.velocity_weights(nv, 6.0, 5.0, "hard_sphere", dims=dims)
        ne = W.density_from_ratio(0.9, W.F_REF)
        nu = 0.3 * 2 * math.pi * W.F_REF
        a, b = B.single_pole(dims, nv, 5.0, "hard_sphere", ne, nu, dt)
        ar, br = M.effective_pole(w, s, nu, A.plasma_omega2(ne), dt)
        assert abs(a - ar) < 1e-12 and abs(b / br - 1) < 1e-12
