"""Helpers shared by the GPU parity tests: run a workload through the C ABI and through
the oracle on the same seeded inputs, and compare."""
import numpy as np

from oracle.core import Oracle1D


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2)) / (den if den > 0 else 1.0))


def oracle_1d(run, nx=None):
    """Oracle for a Run1D, optionally on the prefix [0, nx] of the line (exact as long as
    the field has not reached the cut: the Yee stencil moves information one node per step)."""
    n = run.nx if nx is None else nx
    ne = run.ne[: n + 1].copy()
    if nx is not None:
        ne[n - 1:] = 0.0     # the oracle's line ends in vacuum; the field never gets there
    return Oracle1D(n, run.dx, run.courant, ne, run.nubar[: n + 1].copy(),
                    nv=run.nv, vmax_over_vth=run.vmax_over_vth, te_ev=run.te_ev,
                    nu_model=run.nu_model, bc=run.bc, src_node=run.src_node,
                    src_amp=run.src_amp, src_f=run.src_f, src_tau=run.src_tau,
                    src_t0=run.src_t0, kinetic=getattr(run, "kinetic", "linear"),
                    f0_model=getattr(run, "f0_model", "maxwell"))


def space_time_1d(sim, orc, nsteps, every, probes, df_snaps=None):
    """Advance both sides ``nsteps`` in chunks of ``every``; collect E snapshots (and the
    probe series) from both.  Returns (gpu, oracle) stacked arrays.  With a list
    ``df_snaps``, (gpu, oracle) F1 pairs of the oracle's cells are appended after each
    chunk (a late single snapshot of F1 can be a small residual of a zero-mean drive,
    so F1 is compared over space and time like the fields)."""
    from paper_2211_05647_amd import binding as B
    g_snap, o_snap = [], []
    g_pr, o_pr = [], []
    pids = [sim.add_probe(B.F_E, p) for p in probes] if probes else []
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        sim.run(k)
        pr, _ = orc.run(k, probes=probes)
        o_pr.append(pr)
        done += k
        g_snap.append(sim.read(B.F_E)[: orc.nx + 1])
        o_snap.append(orc.E.copy())
        if df_snaps is not None:
            gd = sim.read(B.F_DF)[: orc.df.size]
            df_snaps.append((gd, orc.df.copy()))
    if pids:
        g_pr = np.stack([sim.read_probe(p, nsteps) for p in pids], axis=1)
        o_pr = np.concatenate(o_pr, axis=0)
    return np.array(g_snap), np.array(o_snap), g_pr, o_pr


def oracle_3d(run):
    """Oracle for a Run3D (same per-cell inputs, same source and layer)."""
    from oracle.core import Oracle3D
    return Oracle3D(run.nx, run.ny, run.nz, run.dx, run.courant, run.ne, run.nubar,
                    vdim=run.nv, vmax_over_vth=run.vmax_over_vth, te_ev=run.te_ev,
                    nu_model=run.nu_model, f0_model=run.f0_model, ncpml=run.ncpml,
                    src_kind=run.src_kind, src_i=run.src_i, src_j=run.src_j, src_k=run.src_k,
                    src_amp=run.src_amp, src_f=run.src_f, src_tau=run.src_tau,
                    src_t0=run.src_t0, kinetic=run.kinetic)


def space_time_3d(sim, orc, nsteps, every):
    """Snapshots after every ``every`` steps from both sides: E, H and J (all three
    components each) and the F1 rows (then, for the two-term model, the cells' F0 rows).  Returns {name: (gpu, oracle)} of stacked arrays."""
    from paper_2211_05647_amd import binding as B
    out = {k: ([], []) for k in ("E", "H", "J", "DF")}
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        sim.run(k)
        orc.run(k)
        done += k
        for name, fs, ref in (("E", (B.F_EX, B.F_EY, B.F_EZ), orc.E),
                              ("H", (B.F_HX, B.F_HY, B.F_HZ), orc.H),
                              ("J", (B.F_JX, B.F_JY, B.F_JZ), orc.J),
                              ("DF", (B.F_DF,), orc.df)):
            out[name][0].append(np.concatenate([sim.read(f) for f in fs]))
            out[name][1].append(ref.copy())
    return {k: (np.array(a), np.array(b)) for k, (a, b) in out.items()}


def max_rel(a, b):
    """Largest single-element error relative to the largest reference magnitude: bounds an
    error confined to a few cells, which a whole-array relative L2 can average away."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = float(np.max(np.abs(b))) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0)) if b.size else 0.0


class ErrSum:
    """Running relative L2 and max-abs figures over pairs of arrays compared one at a time
    (so that large snapshots need not be kept)."""

    def __init__(self):
        self.d2 = 0.0
        self.r2 = 0.0
        self.dmax = 0.0
        self.rmax = 0.0

    def add(self, a, b):
        a = np.asarray(a, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        d = a - b
        self.d2 += float(np.dot(d, d))
        self.r2 += float(np.dot(b, b))
        if d.size:
            self.dmax = max(self.dmax, float(np.max(np.abs(d))))
            self.rmax = max(self.rmax, float(np.max(np.abs(b))))

    @property
    def rel_l2(self):
        return float(np.sqrt(self.d2 / self.r2)) if self.r2 > 0 else float(np.sqrt(self.d2))

    @property
    def max_rel(self):
        return self.dmax / self.rmax if self.rmax > 0 else self.dmax
