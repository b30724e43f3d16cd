"""FP64 oracle of the learned closure: a small MLP that corrects the single-pole (Drude)
recurrence of the cell current, trained on currents the kinetic model produces.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The kinetic F1 model of section 5.2 gives, per velocity bin j, a Crank-Nicolson recursion
J_j^{n+1/2} = alpha_j J_j^{n-1/2} + beta_j E^n.  The closure replaces the sum over bins by
one pole with the w-weighted mean collision rate and lets a network correct the drive:

    J^{n+1/2} = alpha_eff J^{n-1/2} + beta_eff (E^n + s * y),
    y = MLP([E^n .. E^{n-15}] / s, p1, p2),    s = max |E window| (floored),

with p1 = omega_p dt and p2 = log10(nu_mean dt) mapped linearly onto [-1, 1] over the
training box.  y = 0 is the method without the network (exactly the Drude recurrence).
Network: 18 -> 128 (ReLU) -> 128 (ReLU) -> 1.  Optional BF16 emulation rounds
weights and the GEMM operands to bfloat16 (round to nearest even) with FP64 arithmetic
otherwise, mirroring the GPU kernels' operand precision.
"""
import math

import numpy as np

NIN, NH, HIST = 18, 128, 16
NPARAM = NH * NIN + NH + NH * NH + NH + NH + 1   # 19073


def bf16(x):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def relu(x):
    """The hidden layers' activation, max(x, 0)."""
    return np.maximum(x, 0.0)


def relu_grad(x):
    """Its derivative, taken as 0 at x = 0."""
    return (np.asarray(x) > 0.0).astype(np.float64)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == NPARAM
    o = 0
    W1 = p[o:o + NH * NIN].reshape(NH, NIN); o += NH * NIN
    b1 = p[o:o + NH]; o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = p[o:o + NH]; o += NH
    w3 = p[o:o + NH]; o += NH
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def init_params(seed):
    """He-style random initialisation (uniform), seeded."""
    g = np.random.default_rng(seed)
    W1 = g.uniform(-1, 1, (NH, NIN)) * math.sqrt(3.0 / NIN)
    W2 = g.uniform(-1, 1, (NH, NH)) * math.sqrt(3.0 / NH)
    w3 = g.uniform(-1, 1, NH) * math.sqrt(3.0 / NH) * 0.1
    return pack(W1, np.zeros(NH), W2, np.zeros(NH), w3, 0.0)


def forward(p, X, emulate_bf16=False):
    """y for rows X [B, 18]; returns (y, cache)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    Xq, W1q, W2q, w3q = r(X), r(W1), r(W2), r(w3)
    Z1 = Xq @ W1q.T + b1
    A1 = relu(Z1)
    A1q = r(A1)
    Z2 = A1q @ W2q.T + b2
    A2 = relu(Z2)
    y = A2 @ w3q + b3
    return y, (Xq, W1q, W2q, w3q, Z1, A1q, Z2, A2)


def loss_and_grad(p, X, t, emulate_bf16=False):
    """Mean squared error over the batch and its gradient w.r.t. every parameter."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    y, (Xq, W1q, W2q, w3q, Z1, A1q, Z2, A2) = forward(p, X, emulate_bf16)
    B = X.shape[0]
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / B
    gw3 = A2.T @ dy
    gb3 = float(np.sum(dy))
    dA2 = np.outer(dy, w3q)
    dZ2 = dA2 * relu_grad(Z2)
    dZ2q = r(dZ2)
    gW2 = dZ2q.T @ A1q
    gb2 = dZ2.sum(axis=0)
    dA1 = dZ2q @ W2q
    dZ1 = dA1 * relu_grad(Z1)
    dZ1q = r(dZ1)
    gW1 = dZ1q.T @ Xq
    gb1 = dZ1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)


class Adam:
    """Adam (Kingma & Ba 2015) on the FP64 parameter vector."""

    def __init__(self, n, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = beta1, beta2, eps

    def step(self, p, g, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return p - lr * mh / (np.sqrt(vh) + self.eps)


# --- the closure recurrence ----------------------------------------------------------
def effective_pole(w, s, nubar, wp2, dt):
    """Single-pole parameters from the per-bin weights w_j and collision shapes s_j:
    nu_eff = sum w_j nu_j / sum w_j, wp~^2 = wp^2 sum w_j,
    alpha = (2 - dt nu_eff)/(2 + dt nu_eff), beta = 2 dt^2 wp~^2 / (2 + dt nu_eff)
    (beta multiplies E in the normalised current dt/eps0 * J)."""
    nu_eff = nubar * np.sum(w * s) / np.sum(w)
    wt2 = wp2 * np.sum(w)
    return (2 - dt * nu_eff) / (2 + dt * nu_eff), 2 * dt * dt * wt2 / (2 + dt * nu_eff)


def scale_params(wp_dt, nu_dt, box):
    """Map (omega_p dt, log10(nu dt)) onto [-1, 1] over box = (p1lo, p1hi, p2lo, p2hi)."""
    p1lo, p1hi, p2lo, p2hi = box
    q1 = 2.0 * (wp_dt - p1lo) / (p1hi - p1lo) - 1.0
    q2 = 2.0 * (np.log10(nu_dt) - p2lo) / (p2hi - p2lo) - 1.0
    return q1, q2


def features(Ehist, wp_dt, nu_dt, box, floor=1e-30):
    """Ehist [B, 16] with column 0 = E^n, column k = E^{n-k}.  Returns (X [B, 18], s [B])."""
    s = np.maximum(np.max(np.abs(Ehist), axis=1), floor)
    q1, q2 = scale_params(np.asarray(wp_dt, dtype=np.float64), np.asarray(nu_dt, dtype=np.float64), box)
    X = np.concatenate([Ehist / s[:, None], np.broadcast_to(np.atleast_1d(q1), (Ehist.shape[0],))[:, None],
                        np.broadcast_to(np.atleast_1d(q2), (Ehist.shape[0],))[:, None]], axis=1)
    return X, s


def targets(J_prev, J_next, E_n, s, alpha, beta):
    """The network output that makes the closure reproduce J_next exactly."""
    return ((J_next - alpha * J_prev) / beta - E_n) / s


def closure_run(E, alpha, beta, p=None, wp_dt=None, nu_dt=None, box=None, emulate_bf16=False):
    """Drive the closure with a prescribed E series (E[n] = E^n); returns J^{n+1/2} for
    every n.  p = None runs the plain Drude recurrence (y = 0)."""
    E = np.asarray(E, dtype=np.float64)
    J = np.zeros_like(E)
    jp = 0.0
    hist = np.zeros(HIST)
    for n in range(len(E)):
        hist = np.concatenate([[E[n]], hist[:-1]])
        y = 0.0
        if p is not None:
            X, s = features(hist[None, :], wp_dt, nu_dt, box)
            y = forward(p, X, emulate_bf16)[0][0] * s[0]
        jp = alpha * jp + beta * (E[n] + y)
        J[n] = jp
    return J
