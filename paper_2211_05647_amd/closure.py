"""Training pipeline of the learned closure and the closure blob for 2D runs.

Marshalling and orchestration only: the kinetic batch run, the 2V replay cells, pair
assembly, forward/backward/Adam all run in the library's HIP kernels.  Data flow:

  1. a batch of independent 1D kinetic runs (the 256-run workload) records (E^n, J^{n+1/2})
     at seeded plasma nodes of every run (training-pair taps);
  2. each recorded E series drives an isolated 2V kinetic cell (32 x 32 bins, the 2D
     workloads' temperature) -- the kinetic step is local, so this gives exactly the
     current a 2D plasma cell of that density and collision rate would carry;
  3. random (series, step) pairs after the pulse has arrived become feature rows and
     targets; a held-out set of runs is kept for evaluation;
  4. Adam on minibatches; the result is written as an fdtd_mlp_blob.
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass

import numpy as np

from . import binding as B
from . import workloads as W

MAGIC = 0x4D4C5043
BLOB_HEADER = struct.Struct("<IIiiii" + "d" * 7)   # magic .. reserved, te, vmax, dt, box[4]
BLOB_BYTES = ((BLOB_HEADER.size + 4 * B.NPARAM) + 7) // 8 * 8

_C = 299792458.0
_EPS0 = 8.8541878128e-12
_QE = 1.602176634e-19
_ME = 9.1093837015e-31


def make_blob(params, box, dt, te_ev=5.0, nv=32, nu_model="hard_sphere", vmax_over_vth=6.0,
              dims=2):
    """Bytes of an fdtd_mlp_blob (see include/fdtd_closure.h) as a numpy uint8 array."""
    head = BLOB_HEADER.pack(MAGIC, 1, dims, nv, 0 if nu_model == "hard_sphere" else 1, 0,
                            te_ev, vmax_over_vth, dt, *[float(b) for b in box])
    out = np.zeros(BLOB_BYTES, dtype=np.uint8)
    out[:BLOB_HEADER.size] = np.frombuffer(head, dtype=np.uint8)
    out[BLOB_HEADER.size:BLOB_HEADER.size + 4 * B.NPARAM] = np.frombuffer(
        np.ascontiguousarray(params, dtype=np.float32).tobytes(), dtype=np.uint8)
    return out


def plasma_dt(ne):
    return np.sqrt(np.asarray(ne) * _QE ** 2 / (_EPS0 * _ME))


def scaled(ne, nu, dt, box):
    p1 = plasma_dt(ne) * dt
    p2 = np.log10(nu * dt)
    return (2 * (p1 - box[0]) / (box[1] - box[0]) - 1, 2 * (p2 - box[2]) / (box[3] - box[2]) - 1)


@dataclass
class TrainingData:
    E: object          # torch [nseries, T] recorded fields
    J: object          # torch [nseries, T] replayed normalised 2V currents
    series4: np.ndarray
    lo: np.ndarray     # first usable step of each series
    hi: np.ndarray     # one past the last usable step
    train: np.ndarray  # series indices for training
    held: np.ndarray   # held-out series indices
    box: tuple
    dt: float
    te_ev: float


def gather_data(runs=None, ntap=8, te_ev=5.0, seed=2211, held_runs=24, closure=None, log=print):
    import torch
    runs = W.c3() if runs is None else runs
    g = np.random.default_rng(seed)
    taps = np.zeros((len(runs), ntap), dtype=np.int32)
    for r, run in enumerate(runs):
        cells = np.nonzero(run.ne > 0)[0]
        taps[r] = np.sort(g.choice(cells, size=ntap, replace=False))
    sim = B.Sim(runs, taps=taps)
    T = max(r.steps for r in runs)
    log(f"[closure] batch of {len(runs)} runs, {T} steps, {ntap} taps per run")
    sim.run(T)
    torch.cuda.synchronize()
    ns = len(runs) * ntap
    E = torch.zeros((ns, T), dtype=torch.float32, device="cuda")
    base = sim.workspace.data_ptr()
    for r, run in enumerate(runs):
        ptr, cap, nt = sim.tap_buffer(r)
        off = ptr - base
        view = sim.workspace[off:off + nt * cap * 2 * 4].view(torch.float32).view(nt, cap, 2)
        E[r * ntap:(r + 1) * ntap, :run.steps].copy_(view[:, :run.steps, 0])
    torch.cuda.synchronize()
    sim.close()
    dt = runs[0].courant * runs[0].dx / _C
    ne = np.repeat([run.ne[run.ne > 0][0] for run in runs], ntap)
    nu = np.repeat([run.nubar[run.ne > 0][0] for run in runs], ntap)
    p1 = plasma_dt(ne) * dt
    p2 = np.log10(nu * dt)
    box = (float(p1.min()), float(p1.max()), float(p2.min()), float(p2.max()))
    c = closure or B.Closure(max_rows=8192, max_series=max(ns, 16))
    J = torch.zeros_like(E)
    c.replay2v(E.data_ptr(), 1, T, ns, T, ne, nu, te_ev, dt, J, T)
    torch.cuda.synchronize()
    series4 = np.zeros((ns, 4), dtype=np.float32)
    for s in range(ns):
        a, b = B.single_pole(2, 32, te_ev, "hard_sphere", ne[s], nu[s], dt)
        q1, q2 = scaled(ne[s], nu[s], dt, box)
        series4[s] = (a, b, q1, q2)
    Eh = E.abs().cpu().numpy()
    lo = np.zeros(ns, dtype=np.int64)
    hi = np.zeros(ns, dtype=np.int64)
    steps = np.repeat([run.steps for run in runs], ntap)
    for s in range(ns):
        m = Eh[s].max()
        first = np.argmax(Eh[s] > 1e-3 * m) if m > 0 else steps[s]
        lo[s] = max(first, 15)
        hi[s] = steps[s]
    order = np.random.default_rng(seed + 1).permutation(len(runs))
    held_r = order[:held_runs]
    held = np.concatenate([np.arange(r * ntap, (r + 1) * ntap) for r in held_r])
    train = np.setdiff1d(np.arange(ns), held)
    return TrainingData(E, J, series4, lo, hi, train, held, box, dt, te_ev), c


def sample(data, series, n, g):
    s = g.choice(series, size=n)
    span = np.maximum(data.hi[s] - data.lo[s], 1)
    t = data.lo[s] + (g.random(n) * span).astype(np.int64)
    return (s.astype(np.int64) << 32) | t


def init_params(seed):
    """He-style uniform initialisation of the 19073 parameters, last layer scaled down."""
    g = np.random.default_rng(seed)
    nh, nin = 128, 18
    W1 = g.uniform(-1, 1, (nh, nin)) * math.sqrt(3.0 / nin)
    W2 = g.uniform(-1, 1, (nh, nh)) * math.sqrt(3.0 / nh)
    w3 = g.uniform(-1, 1, nh) * math.sqrt(3.0 / nh) * 0.1
    return np.concatenate([W1.ravel(), np.zeros(nh), W2.ravel(), np.zeros(nh), w3, [0.0]]).astype(np.float32)


def fit(data, closure, iters=6000, batch=8192, lr=2e-3, lr_end=2e-5, seed=7, log=print):
    """Adam on fresh random minibatches of training pairs (cosine-decayed learning rate).
    Returns the trained parameters and the loss history (every 500 iterations)."""
    g = np.random.default_rng(seed)
    closure.set_params(init_params(seed))
    hist = []
    T = data.J.shape[1]
    for it in range(iters):
        idx = sample(data, data.train, batch, g)
        X, Tt = closure.make_pairs(data.E.data_ptr(), 1, T, data.J, T, data.series4, idx)
        rate = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * it / max(iters - 1, 1)))
        want = (it % 500 == 0) or it == iters - 1
        loss = closure.train_step(X, Tt, rate, want_loss=want)
        if want:
            hist.append((it, loss))
            log(f"[closure] iter {it}: loss {loss:.4e}")
    return closure.get_params(), hist


def evaluate(data, closure, series, n=4096 * 8, seed=11):
    """Mean squared error of the network and of y = 0 on pairs from `series`."""
    import torch
    g = np.random.default_rng(seed)
    T = data.J.shape[1]
    se_net, se_zero, cnt = 0.0, 0.0, 0
    for _ in range(n // 4096):
        idx = sample(data, series, 4096, g)
        X, Tt = closure.make_pairs(data.E.data_ptr(), 1, T, data.J, T, data.series4, idx)
        y = closure.forward(X)
        se_net += float(torch.sum((y - Tt) ** 2).item())
        se_zero += float(torch.sum(Tt ** 2).item())
        cnt += 4096
    return se_net / cnt, se_zero / cnt
