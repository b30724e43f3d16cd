"""Seeded synthetic workloads shaped like the paper's plasma-slab problem (section 5).

This module only draws inputs: grids, density and collision-rate profiles, source
parameters.  It holds none of the method's arithmetic and is shared by the oracle
tests and the HIP path.  Everything is derived from ``numpy.random.default_rng``
seeded with 221105647, one spawned sub-stream per workload, so a workload is a pure
function of its name (and the run index for the batched set).

Common frame (a reading of the paper's pulse table in section 5.2):
  * reference frequency f_ref = 20 GHz (the pulse centre frequency), cell size
    dx = lambda_ref / 40, Courant number S = c dt / dx = 0.5;
  * Gaussian-modulated sine source, tau = 0.966 / f_src and t0 = 4.5 tau (this
    reproduces the table's 48 ps / 217 ps at 20 GHz), amplitude 1 V/m;
  * densities are given through the plasma-to-source frequency ratio
    r = omega_p / omega_src and converted to m^-3 here:
    n = eps0 m_e (r omega_src)^2 / e^2 (CODATA 2018 constants);
  * collision rates are given as nu_mean / omega_src and converted to 1/s.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED = 221105647
F_REF = 20e9

# CODATA 2018 (input conversion only)
_C = 299792458.0
_EPS0 = 8.8541878128e-12
_QE = 1.602176634e-19
_ME = 9.1093837015e-31

DX_REF = _C / F_REF / 40.0
COURANT_1D = 0.5
COURANT_2D = 0.5

_STREAMS = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4": 4, "c1l": 5, "mlp": 6, "misc": 7}


def rng(name: str) -> np.random.Generator:
    """Independent, reproducible sub-stream for workload ``name``."""
    ss = np.random.SeedSequence(SEED).spawn(len(_STREAMS))[_STREAMS[name]]
    return np.random.default_rng(ss)


def density_from_ratio(r, f_src):
    w = 2.0 * math.pi * f_src
    return _EPS0 * _ME * (np.asarray(r, dtype=np.float64) * w) ** 2 / _QE ** 2


def pulse(f_src):
    tau = 0.966 / f_src
    return dict(src_amp=1.0, src_f=f_src, src_tau=tau, src_t0=4.5 * tau)


@dataclass
class Run1D:
    """One 1D (Ez, Hy) run with a 1V kinetic plasma: per-node inputs of length nx+1."""
    name: str
    nx: int
    nv: int
    ne: np.ndarray
    nubar: np.ndarray
    src_node: int
    src_amp: float
    src_f: float
    src_tau: float
    src_t0: float
    steps: int
    dx: float = DX_REF
    courant: float = COURANT_1D
    te_ev: float = 2.0
    vmax_over_vth: float = 6.0
    nu_model: str = "hard_sphere"
    bc: str = "mur"
    meta: dict = field(default_factory=dict)
    kinetic: str = "linear"     # "linear" (F0 frozen), "full" (the whole f evolves) or
                                # "two_term" (speed grid: F1 and an evolving F0)
    f0_model: str = "maxwell"   # two-term model: "maxwell" or "druyvesteyn"

    @property
    def plasma_cells(self) -> int:
        return int(np.count_nonzero(self.ne > 0))


@dataclass
class Run2D:
    """One 2D TEz run with a 2V kinetic plasma: per-cell inputs of shape (ny, nx)."""
    name: str
    nx: int
    ny: int
    nv: int
    ne: np.ndarray
    nubar: np.ndarray
    src_kind: int
    src_i: int
    src_j: int
    src_amp: float
    src_f: float
    src_tau: float
    src_t0: float
    steps: int
    dx: float = DX_REF
    courant: float = COURANT_2D
    te_ev: float = 5.0
    vmax_over_vth: float = 6.0
    nu_model: str = "hard_sphere"
    ncpml: int = 8
    meta: dict = field(default_factory=dict)

    @property
    def plasma_cells(self) -> int:
        return int(np.count_nonzero(self.ne > 0))


def slab_1d(nx, nv, lo, hi, ratio, nu_ratio, f_src, src_node, steps, name="slab",
            te_ev=2.0, nu_model="hard_sphere", bc="mur", f_grid=F_REF) -> Run1D:
    ne = np.zeros(nx + 1)
    nub = np.zeros(nx + 1)
    ne[lo:hi] = density_from_ratio(ratio, f_src)
    nub[lo:hi] = nu_ratio * 2.0 * math.pi * f_src
    return Run1D(name=name, nx=nx, nv=nv, ne=ne, nubar=nub, src_node=src_node,
                 steps=steps, te_ev=te_ev, nu_model=nu_model, bc=bc,
                 dx=_C / f_grid / 40.0, **pulse(f_src))


def c0() -> Run1D:
    """Small FP64 case: Nx=1000, slab [400, 600), omega_p/omega=0.8, nu/omega=0.1,
    Nv=64 on +-6 v_th, Te=2 eV, source at node 100, Mur ends, 1000 steps."""
    return slab_1d(1000, 64, 400, 600, 0.8, 0.1, F_REF, 100, 1000, name="c0")


def smoothed_uniform(g: np.random.Generator, n: int, sigma: float) -> np.ndarray:
    """White noise -> periodic Gaussian filter (width ``sigma`` samples) -> map through
    the normal CDF of its own spread, giving a smooth field with uniform marginals."""
    from scipy.ndimage import gaussian_filter1d
    from scipy.special import ndtr
    w = gaussian_filter1d(g.standard_normal(n), sigma, mode="wrap")
    return ndtr(w / w.std())


def c1(nx: int = 65536, steps: int = 20000, name: str = "c1", stream: str = "c1") -> Run1D:
    """Large 1D case: Nx=65536, Nv=512, plasma over nodes [400, Nx-100) with a smoothed
    random profile omega_p/omega in [0.2, 2] and log-uniform nu/omega in [0.01, 1]."""
    g = rng(stream)
    lo, hi = 400, nx - 100
    u = smoothed_uniform(g, hi - lo, 64.0)
    u2 = smoothed_uniform(g, hi - lo, 64.0)
    w = 2.0 * math.pi * F_REF
    ne = np.zeros(nx + 1)
    nub = np.zeros(nx + 1)
    ne[lo:hi] = density_from_ratio(0.2 + 1.8 * u, F_REF)
    nub[lo:hi] = 10.0 ** (-2.0 + 2.0 * u2) * w
    return Run1D(name=name, nx=nx, nv=512, ne=ne, nubar=nub, src_node=100, steps=steps,
                 **pulse(F_REF))


def c1_large() -> Run1D:
    """C1 with Nx = 2^20 and 2000 steps: F1 (1.07 GB half grid in FP32) exceeds every cache."""
    return c1(nx=1 << 20, steps=2000, name="c1l", stream="c1l")


def c2(n: int = 512, radius: float = 100.0, steps: int = 4000) -> Run2D:
    """2D TEz 512x512, 32x32 velocity grid, CPML 8, plasma column of radius 100 cells
    at the centre (omega_p/omega=1.2, nu/omega=0.05, Te=5 eV), Ey line source at i=20."""
    ii, jj = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5)
    inside = (ii - n / 2) ** 2 + (jj - n / 2) ** 2 < radius ** 2
    ne = np.where(inside, density_from_ratio(1.2, F_REF), 0.0)
    nub = np.where(inside, 0.05 * 2.0 * math.pi * F_REF, 0.0)
    return Run2D(name="c2", nx=n, ny=n, nv=32, ne=ne, nubar=nub, src_kind=1, src_i=20,
                 src_j=0, steps=steps, **pulse(F_REF))


def c3(nruns: int = 256) -> list:
    """Batched set: Nx ~ U[500, 20000], Nv in {64, 128, 256}, slab [0.4 Nx, 0.6 Nx) with
    omega_p/omega ~ U[0.2, 2], nu/omega log-U[0.01, 1], f_src = f_ref (1 + U[-0.3, 0.3])
    on the fixed f_ref grid, source at 0.1 Nx, 2 Nx steps per run."""
    g = rng("c3")
    runs = []
    for r in range(nruns):
        nx = int(g.integers(500, 20001))
        nv = int(g.choice([64, 128, 256]))
        ratio = float(g.uniform(0.2, 2.0))
        nu_ratio = float(10.0 ** g.uniform(-2.0, 0.0))
        f_src = F_REF * (1.0 + float(g.uniform(-0.3, 0.3)))
        run = slab_1d(nx, nv, int(0.4 * nx), int(0.6 * nx), ratio, nu_ratio, f_src,
                      int(0.1 * nx), 2 * nx, name=f"c3_{r}")
        run.meta = dict(ratio=ratio, nu_ratio=nu_ratio, f_src=f_src)
        runs.append(run)
    return runs


def blobs_2d(n: int, nblobs: int, g: np.random.Generator, ratio_lo=0.2, ratio_hi=1.5,
             r_lo=40.0, r_hi=200.0, margin=208, extra_hot: int = 0):
    """Random circular plasma blobs; where blobs overlap the one with the larger
    omega_p wins (with its own nu)."""
    ratio = np.zeros((n, n))
    nur = np.zeros((n, n))
    specs = []
    for b in range(nblobs + extra_hot):
        cx, cy = g.uniform(margin, n - margin, size=2)
        rad = g.uniform(r_lo, r_hi) * n / 4096.0
        rr = g.uniform(ratio_lo, ratio_hi) if b < nblobs else g.uniform(2.0, 2.5)
        nn = 10.0 ** g.uniform(-2.0, 0.0)
        specs.append((cx, cy, rad, rr, nn))
    for (cx, cy, rad, rr, nn) in specs:
        i0, i1 = max(0, int(cx - rad) - 1), min(n, int(cx + rad) + 2)
        j0, j1 = max(0, int(cy - rad) - 1), min(n, int(cy + rad) + 2)
        ii, jj = np.meshgrid(np.arange(i0, i1) + 0.5, np.arange(j0, j1) + 0.5)
        m = (ii - cx) ** 2 + (jj - cy) ** 2 < rad ** 2
        sub_r = ratio[j0:j1, i0:i1]
        sub_n = nur[j0:j1, i0:i1]
        take = m & (rr > sub_r)
        sub_r[take] = rr
        sub_n[take] = nn
    return ratio, nur, specs


def c4(n: int = 4096, nblobs: int = 48, extra_hot: int = 0, steps: int = 2000) -> Run2D:
    """2D TEz 4096x4096 with 48 random plasma blobs (omega_p/omega in [0.2, 1.5],
    nu/omega log-U[0.01, 1], radii U[40, 200] cells), Te=5 eV, Ey line source."""
    g = rng("c4")
    ratio, nur, specs = blobs_2d(n, nblobs, g, extra_hot=extra_hot)
    ne = np.where(ratio > 0, density_from_ratio(ratio, F_REF), 0.0)
    nub = nur * 2.0 * math.pi * F_REF
    return Run2D(name="c4", nx=n, ny=n, nv=32, ne=ne, nubar=nub, src_kind=1, src_i=20,
                 src_j=0, steps=steps, meta=dict(blobs=specs), **pulse(F_REF))


COURANT_3D = 0.5

# The paper's 3D Argon experiment (section 5.3 table): n = 1e19 m^-3, neutral density
# N = 1e23 m^-3, Te = 1 eV, a 4 mm plasma slab along z between air, a 20 GHz Gaussian-
# modulated plane wave (tau 48 ps, t0 217 ps).  Its elastic cross section s is not given:
# a constant s = 1e-19 m^2 stands in (nu = N s v).
ARGON_NE = 1e19
ARGON_N = 1e23
ARGON_S = 1e-19
ARGON_TE = 1.0


@dataclass
class Run3D:
    """One 3D run (Yee cube, CPML on all faces) with the speed-grid F1 in every plasma
    point: per-cell inputs of shape (nz, ny, nx)."""
    name: str
    nx: int
    ny: int
    nz: int
    nv: int            # speeds of the grid (the paper's v_dim)
    ne: np.ndarray
    nubar: np.ndarray
    src_kind: int      # 1 sheet of Ex on plane src_k (plane wave along z), 2 point
    src_i: int
    src_j: int
    src_k: int
    src_amp: float
    src_f: float
    src_tau: float
    src_t0: float
    steps: int
    dx: float = DX_REF
    courant: float = COURANT_3D
    te_ev: float = ARGON_TE
    vmax_over_vth: float = 5.0
    nu_model: str = "hard_sphere"
    f0_model: str = "druyvesteyn"
    ncpml: int = 8
    kinetic: str = "linear"   # or "two_term" (F0 of every plasma cell evolving)
    meta: dict = field(default_factory=dict)

    @property
    def plasma_cells(self) -> int:
        return int(np.count_nonzero(self.ne > 0))


def argon_nubar(te_ev=ARGON_TE, f0="druyvesteyn"):
    """Mean collision frequency N s <v> of the argon stand-in, with <v> the mean speed of
    the F0 (continuous): Maxwellian sqrt(8 e Te / (pi m)); Druyvesteyn with the same mean
    energy, vD Gamma(1) / Gamma(3/4), vD^2 = 3 (e Te / m) Gamma(3/4) / Gamma(5/4)."""
    vth2 = _QE * te_ev / _ME
    if f0 == "maxwell":
        vbar = math.sqrt(8.0 * vth2 / math.pi)
    else:
        vd = math.sqrt(3.0 * vth2 * math.gamma(0.75) / math.gamma(1.25))
        vbar = vd * math.gamma(1.0) / math.gamma(0.75)
    return ARGON_N * ARGON_S * vbar


def argon_slab_3d(nx=64, ny=64, nz=256, nv=31, steps=1200, slab_mm=4.0, ncpml=8,
                  f0="druyvesteyn", name="argon3d", kinetic="linear",
                  plasma_in_cpml=None) -> Run3D:
    """The paper's 3D slab: air, a slab_mm plasma slab along z starting at the middle of
    the box, air; a sheet source of Ex (a plane wave along z) 12 cells inside the low z
    layer; CPML on all faces; density 1e19 m^-3 with +-5 % seeded cell-to-cell texture.

    plasma_in_cpml: whether the slab runs on through the x and y absorbing layers (default:
    yes for the linear model, no for the two-term one).  With its point set (E points whose
    four cells all hold plasma) the two-term model has a mode that grows by about 6x per
    500 steps once plasma lies inside those layers (the FP64 oracle grows alike, and so
    does the linear model restricted to that point set); with the slab ending where the
    layers begin it decays."""
    g = rng("misc")
    ne = np.zeros((nz, ny, nx))
    nu = np.zeros((nz, ny, nx))
    k0 = nz // 2
    k1 = k0 + max(1, int(round(slab_mm * 1e-3 / DX_REF)))
    ne[k0:k1] = ARGON_NE * (1.0 + 0.05 * (2.0 * g.random((k1 - k0, ny, nx)) - 1.0))
    nu[k0:k1] = argon_nubar(f0=f0)
    if plasma_in_cpml is None:
        plasma_in_cpml = kinetic != "two_term"
    if not plasma_in_cpml and ncpml > 0:
        for a in (ne, nu):
            a[:, :, :ncpml] = 0.0
            a[:, :, nx - ncpml:] = 0.0
            a[:, :ncpml, :] = 0.0
            a[:, ny - ncpml:, :] = 0.0
    p = dict(src_amp=1.0, src_f=20e9, src_tau=48e-12, src_t0=217e-12)
    return Run3D(name=name, nx=nx, ny=ny, nz=nz, nv=nv, ne=ne, nubar=nu, src_kind=1, src_i=0,
                 src_j=0, src_k=ncpml + 4, steps=steps, ncpml=ncpml, f0_model=f0,
                 kinetic=kinetic, meta=dict(slab=(k0, k1)), **p)


def argon_line_1d(nv=31, kinetic="two_term", f0="druyvesteyn", slab_mm=4.0,
                  cells_per_mm=5, steps=4000) -> Run1D:
    """The paper's argon experiment along its propagation axis (the plane wave sees only z):
    air, a slab_mm slab of 1e19 m^-3 argon plasma (Te = 1 eV, nu = N s <v> of the stand-in
    cross section), air; Mur ends; the section 5.3 pulse (20 GHz, tau 48 ps, t0 217 ps)
    from a soft source 100 cells before the slab.  The ports of the scattering parameters
    sit at the two faces of the slab (the paper's z = 0 and z = 4 mm)."""
    dx = 1e-3 / cells_per_mm
    n_slab = int(round(slab_mm * cells_per_mm))
    lo = 400
    hi = lo + n_slab
    nx = hi + 400
    ne = np.zeros(nx + 1)
    nub = np.zeros(nx + 1)
    ne[lo:hi] = ARGON_NE
    nub[lo:hi] = argon_nubar(f0=f0)
    run = Run1D(name="argon1d", nx=nx, nv=nv, ne=ne, nubar=nub, src_node=lo - 100,
                src_amp=1.0, src_f=20e9, src_tau=48e-12, src_t0=217e-12, steps=steps, dx=dx,
                te_ev=ARGON_TE, vmax_over_vth=5.0, kinetic=kinetic, f0_model=f0,
                meta=dict(ports=(lo - 1, hi)))
    return run
