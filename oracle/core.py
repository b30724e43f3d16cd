"""ctypes front-end of the FP64 oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  State lives in numpy arrays
owned by the caller, so a run can be continued, inspected step by step, or saved.

Each class follows the step order of the paper's coupled model (section 5.2):
H update -> F1 update driven by E^n -> current moment J -> E update (Ampere's
law with -J, eq. (1)) -> absorbing boundary -> soft source at t^{n+1}.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.oracle_vgrid.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp]
        L.oracle_nu_shape.argtypes = [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_int, _dp]
        L.oracle_collision1v.argtypes = [C.c_int, _dp, _dp, _dp]
        L.oracle_constants.argtypes = [_dp]
        L.oracle_threads.argtypes = []
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_cpml_profile.argtypes = [C.c_int, C.c_int] + [C.c_double] * 7 + [_dp] * 6
        L.oracle_run1d.argtypes = (
            [C.c_int, C.c_double, C.c_double, C.c_int,
             C.c_int, C.c_double, C.c_double, C.c_int,
             _dp, _dp,
             C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
             C.c_longlong, C.c_longlong,
             _dp, _dp, _dp, _dp,
             C.c_int, _ip, _dp, C.c_int, _dp, C.c_int])
        L.oracle_run2d.argtypes = (
            [C.c_int, C.c_int, C.c_double, C.c_double,
             C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
             C.c_int, C.c_double, C.c_double, C.c_int,
             _dp, _dp,
             C.c_int, C.c_int, C.c_int,
             C.c_double, C.c_double, C.c_double, C.c_double,
             C.c_longlong, C.c_longlong,
             _dp, _dp, _dp, _dp, _dp, _dp, _dp,
             C.c_int, _ip, _dp,
             _ip, _dp, _dp, C.c_int, _dp, _dp])
        L.oracle_mlp.argtypes = [_dp, _dp, C.c_int]
        L.oracle_mlp.restype = C.c_double
        L.oracle_replay1v.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                      C.c_double, C.c_double, C.c_longlong, _dp, _dp]
        L.oracle_full1v.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                    C.c_double, C.c_double, C.c_longlong, _dp, _dp, _dp]
        L.oracle_sgrid.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, _dp, _dp, _dp, _dp, _dp]
        L.oracle_snu_shape.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_int, _dp]
        L.oracle_plasma3d_count.argtypes = [C.c_int, C.c_int, C.c_int, _dp]
        L.oracle_plasma3d_count_strict.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _ip]
        L.oracle_plasma3d_map.argtypes = [C.c_int, C.c_int, C.c_int, _dp, C.c_int, _ip, _ip]
        L.oracle_run3d.argtypes = (
            [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
             C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
             C.c_int, C.c_double, C.c_double, C.c_int, C.c_int,
             _dp, _dp,
             C.c_int, C.c_int, C.c_int, C.c_int,
             C.c_double, C.c_double, C.c_double, C.c_double,
             C.c_longlong, C.c_longlong,
             _dp, _dp, _dp, _dp, _dp,
             C.c_int, _ip, _dp, C.c_int])
        L.oracle_run1d_twoterm.argtypes = (
            [C.c_int, C.c_double, C.c_double, C.c_int,
             C.c_int, C.c_double, C.c_double, C.c_int, C.c_int,
             _dp, _dp,
             C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
             C.c_longlong, C.c_longlong,
             _dp, _dp, _dp, _dp,
             C.c_int, _ip, _dp, C.c_int])
        L.oracle_replay2v.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double,
                                      C.c_double, C.c_double, C.c_longlong, _dp, _dp, _dp, _dp]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_ip)
    raise TypeError(a.dtype)


def threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def set_threads(n):
    """Use n threads in the oracle's parallel loops from now on; returns the count."""
    return int(lib().oracle_set_threads(int(n)))


def constants():
    out = np.zeros(4)
    lib().oracle_constants(_p(out))
    return dict(c=out[0], eps0=out[1], e=out[2], me=out[3])


def vgrid(nv, vmax_over_vth, te_ev):
    """Velocity grid and Maxwellian tables (see ``oracle_vgrid``)."""
    v, fh, gh = np.zeros(nv), np.zeros(nv), np.zeros(nv)
    dv, vth = C.c_double(), C.c_double()
    rc = lib().oracle_vgrid(nv, vmax_over_vth, te_ev, _p(v), _p(fh), _p(gh), C.byref(dv), C.byref(vth))
    if rc:
        raise ValueError("bad velocity grid")
    return v, fh, gh, dv.value, vth.value


def sgrid(vdim, vmax_over_vth, te_ev, f0_model=0):
    """Speed grid and isotropic F0 tables of the 3D model (see ``oracle_sgrid``):
    (v, F0, dF0/dv, gam, v_th); f0_model 0 Maxwellian, 1 Druyvesteyn."""
    v, F0, dF0 = np.zeros(vdim), np.zeros(vdim), np.zeros(vdim)
    gam, vth = C.c_double(), C.c_double()
    rc = lib().oracle_sgrid(vdim, vmax_over_vth, te_ev, f0_model, _p(v), _p(F0), _p(dF0),
                            C.byref(gam), C.byref(vth))
    if rc:
        raise ValueError("bad speed grid")
    return v, F0, dF0, gam.value, vth.value


def snu_shape(vdim, vmax_over_vth, te_ev, f0_model, model):
    v, F0, dF0, gam, vth = sgrid(vdim, vmax_over_vth, te_ev, f0_model)
    s = np.zeros(vdim)
    lib().oracle_snu_shape(vdim, _p(v), _p(F0), gam, model, _p(s))
    return s


def nu_shape(dims, nv, vmax_over_vth, te_ev, model):
    v, fh, gh, dv, vth = vgrid(nv, vmax_over_vth, te_ev)
    s = np.zeros(nv if dims == 1 else nv * nv)
    lib().oracle_nu_shape(dims, nv, _p(v), _p(fh), dv, model, _p(s))
    return s


def collision1v(nu, f):
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    lib().oracle_collision1v(len(f), _p(nu), _p(f), _p(out))
    return out


def cpml_profile(n, ncpml, dx, dt, order=3.0, sigma_factor=1.0, kappa_max=5.0,
                 alpha_min=0.0, alpha_max=0.05):
    be, ae, ke = np.zeros(n + 1), np.zeros(n + 1), np.zeros(n + 1)
    bh, ah, kh = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().oracle_cpml_profile(n, ncpml, dx, dt, order, sigma_factor, kappa_max, alpha_min,
                              alpha_max, _p(be), _p(ae), _p(ke), _p(bh), _p(ah), _p(kh))
    return dict(be=be, ae=ae, ke=ke, bh=bh, ah=ah, kh=kh)


def mlp(params, x, emulate_bf16=False):
    """The closure network on one feature row (plain C, FP64)."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().oracle_mlp(_p(params), _p(x), int(bool(emulate_bf16)))


def replay1v(E, ne, nubar, dt, nv=64, vmax_over_vth=6.0, te_ev=2.0, nu_model="hard_sphere"):
    """One isolated 1V cell driven by the series E[n] = E^n; returns J^{n+1/2} (A/m^2)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    J = np.zeros_like(E)
    rc = lib().oracle_replay1v(nv, vmax_over_vth, te_ev, {"hard_sphere": 0, "const": 1}[nu_model],
                               ne, nubar, dt, len(E), _p(E), _p(J))
    if rc:
        raise ValueError("bad replay arguments")
    return J


def full1v(E, ne, nubar, dt, delta=None, nv=64, vmax_over_vth=6.0, te_ev=2.0,
           nu_model="hard_sphere"):
    """One isolated node of the full-distribution model driven by E[n] = E^n.

    ``delta`` (nv values, f = ne fhat + delta) is advanced in place when given (zeros
    otherwise); returns (J^{n+1/2} series in A/m^2, delta)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    J = np.zeros_like(E)
    d = np.zeros(nv) if delta is None else delta
    assert d.dtype == np.float64 and d.shape == (nv,) and d.flags["C_CONTIGUOUS"]
    rc = lib().oracle_full1v(nv, vmax_over_vth, te_ev, {"hard_sphere": 0, "const": 1}[nu_model],
                             ne, nubar, dt, len(E), _p(E), _p(d), _p(J))
    if rc == -2:
        raise ValueError("field too strong for the velocity grid: |a dt / dv| > 1")
    if rc:
        raise ValueError("bad arguments")
    return J, d


def replay2v(Ex, Ey, ne, nubar, dt, nv=32, vmax_over_vth=6.0, te_ev=5.0, nu_model="hard_sphere"):
    """One isolated 2V cell driven by (Ex, Ey)[n]; returns (Jx, Jy)^{n+1/2} (A/m^2)."""
    Ex = np.ascontiguousarray(Ex, dtype=np.float64)
    Ey = np.ascontiguousarray(Ey, dtype=np.float64)
    Jx, Jy = np.zeros_like(Ex), np.zeros_like(Ex)
    rc = lib().oracle_replay2v(nv, vmax_over_vth, te_ev, {"hard_sphere": 0, "const": 1}[nu_model],
                               ne, nubar, dt, len(Ex), _p(Ex), _p(Ey), _p(Jx), _p(Jy))
    if rc:
        raise ValueError("bad replay arguments")
    return Jx, Jy


class Oracle1D:
    """1D (Ez, Hy) Yee grid coupled to a 1V kinetic F1 in every plasma node.

    ``ne``/``nubar`` are per E node (nx+1 values).  ``bc`` is ``"mur"`` or ``"pec"``.
    ``kinetic`` is ``"linear"`` (F1 against the frozen F0) or ``"full"`` (the whole f
    evolves; ``df`` then holds f - ne fhat per node) on the signed grid of ``nv`` bins, or
    ``"two_term"`` (F1 and an evolving F0 on a speed grid of ``nv`` speeds; ``df`` rows
    hold [F1 | F0 - ne F0hat]) / ``"two_term_frozen"`` (the same with F0 held), with
    ``f0_model`` ``"maxwell"`` or ``"druyvesteyn"``.
    """

    def __init__(self, nx, dx, courant, ne, nubar, nv=64, vmax_over_vth=6.0, te_ev=2.0,
                 nu_model="hard_sphere", bc="mur", src_node=0, src_amp=0.0, src_f=0.0,
                 src_tau=1.0, src_t0=0.0, kinetic="linear", f0_model="maxwell"):
        self.model = {"linear": 0, "full": 1, "two_term": 2, "two_term_frozen": 3}[kinetic]
        self.f0_model = {"maxwell": 0, "druyvesteyn": 1}[f0_model]
        self.nx, self.dx, self.courant = int(nx), float(dx), float(courant)
        self.ne = np.ascontiguousarray(ne, dtype=np.float64)
        self.nubar = np.ascontiguousarray(nubar, dtype=np.float64)
        assert self.ne.shape == (nx + 1,) and self.nubar.shape == (nx + 1,)
        self.nv, self.vmax, self.te = int(nv), float(vmax_over_vth), float(te_ev)
        self.nu_model = {"hard_sphere": 0, "const": 1}[nu_model]
        self.bc = {"pec": 0, "mur": 1}[bc]
        self.src = (int(src_node), float(src_amp), float(src_f), float(src_tau), float(src_t0))
        self.cells = np.nonzero(self.ne > 0)[0].astype(np.int32)
        self.E = np.zeros(nx + 1)
        self.H = np.zeros(nx)
        self.J = np.zeros(nx + 1)
        self.row = self.nv * (2 if self.model >= 2 else 1)
        self.df = np.zeros(len(self.cells) * self.row)
        self.step = 0
        self.dt = self.courant * self.dx / constants()["c"]

    def run(self, nsteps, probes=(), snap_every=0):
        probes = np.ascontiguousarray(probes, dtype=np.int32)
        if self.model >= 2:
            pout = np.zeros(max(1, nsteps * len(probes)))
            rc = lib().oracle_run1d_twoterm(
                self.nx, self.dx, self.courant, self.bc,
                self.nv, self.vmax, self.te, self.nu_model, self.f0_model,
                _p(self.ne), _p(self.nubar), *self.src,
                self.step, int(nsteps),
                _p(self.E), _p(self.H), _p(self.J), _p(self.df),
                len(probes), _p(probes) if len(probes) else None, _p(pout),
                int(self.model == 2))
            if rc:
                raise ValueError("oracle_run1d_twoterm rejected its arguments")
            self.step += int(nsteps)
            return pout[: nsteps * len(probes)].reshape(nsteps, len(probes)), np.zeros((0, self.nx + 1))
        pout = np.zeros(max(1, nsteps * len(probes)))
        nsnap = nsteps // snap_every if snap_every > 0 else 0
        sout = np.zeros(max(1, nsnap * (self.nx + 1)))
        rc = lib().oracle_run1d(
            self.nx, self.dx, self.courant, self.bc,
            self.nv, self.vmax, self.te, self.nu_model,
            _p(self.ne), _p(self.nubar),
            *self.src,
            self.step, int(nsteps),
            _p(self.E), _p(self.H), _p(self.J), _p(self.df),
            len(probes), _p(probes) if len(probes) else None, _p(pout),
            int(snap_every), _p(sout), self.model)
        if rc == -2:
            raise ValueError("field too strong for the velocity grid: |a dt / dv| > 1")
        if rc:
            raise ValueError("oracle_run1d rejected its arguments")
        self.step += int(nsteps)
        return (pout[: nsteps * len(probes)].reshape(nsteps, len(probes)),
                sout[: nsnap * (self.nx + 1)].reshape(nsnap, self.nx + 1))

    def df_rows(self):
        return self.df.reshape(len(self.cells), self.row)


class Oracle2D:
    """2D TEz (Ex, Ey, Hz) Yee grid with CPML and a 2V kinetic F1 per plasma cell.

    ``ne``/``nubar`` are per cell, shape (ny, nx).  ``src_kind``: 0 none, 1 Ey line at
    column ``src_i``, 2 Ey point at (src_i, src_j).
    """

    def __init__(self, nx, ny, dx, courant, ne, nubar, nv=32, vmax_over_vth=6.0, te_ev=5.0,
                 nu_model="hard_sphere", ncpml=8, cpml_order=3.0, sigma_factor=1.0,
                 kappa_max=5.0, alpha_min=0.0, alpha_max=0.05,
                 src_kind=0, src_i=0, src_j=0, src_amp=0.0, src_f=0.0, src_tau=1.0, src_t0=0.0):
        self.nx, self.ny, self.dx, self.courant = int(nx), int(ny), float(dx), float(courant)
        self.ne = np.ascontiguousarray(ne, dtype=np.float64).reshape(-1)
        self.nubar = np.ascontiguousarray(nubar, dtype=np.float64).reshape(-1)
        assert self.ne.shape == (nx * ny,)
        self.nv, self.vmax, self.te = int(nv), float(vmax_over_vth), float(te_ev)
        self.nu_model = {"hard_sphere": 0, "const": 1}[nu_model]
        self.cpml = (int(ncpml), float(cpml_order), float(sigma_factor), float(kappa_max),
                     float(alpha_min), float(alpha_max))
        self.src = (int(src_kind), int(src_i), int(src_j), float(src_amp), float(src_f),
                    float(src_tau), float(src_t0))
        self.cells = np.nonzero(self.ne > 0)[0].astype(np.int32)
        self.Ex = np.zeros((ny + 1, nx))
        self.Ey = np.zeros((ny, nx + 1))
        self.Hz = np.zeros((ny, nx))
        self.Jx = np.zeros((ny + 1, nx))
        self.Jy = np.zeros((ny, nx + 1))
        self.psi = np.zeros(self.Ex.size + self.Ey.size + 2 * self.Hz.size)
        self.df = np.zeros(len(self.cells) * self.nv * self.nv)
        self.step = 0
        self.dt = self.courant * self.dx / constants()["c"]
        self.closure = None

    def set_closure(self, mode, coef, params, emulate_bf16=True):
        """Learned closure on the plasma cells with mode 1: coef [ncell][4] = (alpha, beta,
        q1, q2), params the 19073 network parameters (FP64)."""
        n = len(self.cells)
        self.closure = dict(mode=np.ascontiguousarray(mode, dtype=np.int32),
                            coef=np.ascontiguousarray(coef, dtype=np.float64).reshape(n * 4),
                            params=np.ascontiguousarray(params, dtype=np.float64),
                            bf=int(bool(emulate_bf16)), hist=np.zeros(n * 32), J=np.zeros(n * 2))

    def run(self, nsteps, probes=()):
        """``probes`` are (i, j) Ey indices; returns Ey at them after every step."""
        idx = np.ascontiguousarray([j * (self.nx + 1) + i for (i, j) in probes], dtype=np.int32)
        pout = np.zeros(max(1, nsteps * len(idx)))
        rc = lib().oracle_run2d(
            self.nx, self.ny, self.dx, self.courant, *self.cpml,
            self.nv, self.vmax, self.te, self.nu_model,
            _p(self.ne), _p(self.nubar), *self.src,
            self.step, int(nsteps),
            _p(self.Ex), _p(self.Ey), _p(self.Hz), _p(self.Jx), _p(self.Jy),
            _p(self.psi), _p(self.df),
            len(idx), _p(idx) if len(idx) else None, _p(pout),
            *((_p(self.closure["mode"]), _p(self.closure["coef"]), _p(self.closure["params"]),
               self.closure["bf"], _p(self.closure["hist"]), _p(self.closure["J"]))
              if self.closure else (None, None, None, 0, None, None)))
        if rc:
            raise ValueError("oracle_run2d rejected its arguments")
        self.step += int(nsteps)
        return pout[: nsteps * len(idx)].reshape(nsteps, len(idx))

    def df_cells(self):
        return self.df.reshape(len(self.cells), self.nv, self.nv)


class Oracle3D:
    """3D Yee cube with CPML on all faces and, at every plasma E point, the F1 component
    of that E on a speed grid of ``vdim`` speeds (the paper's production model).

    ``kinetic``: "linear" (F0 held, F1 on every E point touching plasma), "two_term"
    (F0 per plasma cell evolving under the l = 0 equation, F1 on the E points whose four
    cells are all plasma) or "two_term_frozen" (that model with F0 held).  ``df`` holds
    the F1 rows of the points, then for the two-term models the F0 - n F0hat rows of
    the plasma cells (cells with ne > 0 in storage order).

    ``ne``/``nubar`` are per cell, shape (nz, ny, nx).  Fields are kept as flat arrays in
    the library's layout; ``Ex``/``Ey``/``Ez`` (and H, J) give shaped views.
    ``src_kind``: 0 none, 1 Ex sheet on plane ``src_k``, 2 Ex point (src_i, src_j, src_k).
    """

    def __init__(self, nx, ny, nz, dx, courant, ne, nubar, vdim=31, vmax_over_vth=4.0,
                 te_ev=1.0, nu_model="hard_sphere", f0_model="maxwell", ncpml=8,
                 cpml_order=3.0, sigma_factor=1.0, kappa_max=5.0, alpha_min=0.0,
                 alpha_max=0.05, src_kind=0, src_i=0, src_j=0, src_k=0, src_amp=0.0,
                 src_f=0.0, src_tau=1.0, src_t0=0.0, kinetic="linear"):
        self.model = {"linear": 0, "two_term": 1, "two_term_frozen": 2}[kinetic]
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.courant = float(dx), float(courant)
        self.ne = np.ascontiguousarray(ne, dtype=np.float64).reshape(-1)
        self.nubar = np.ascontiguousarray(nubar, dtype=np.float64).reshape(-1)
        assert self.ne.shape == (nx * ny * nz,) and self.nubar.shape == self.ne.shape
        self.vdim, self.vmax, self.te = int(vdim), float(vmax_over_vth), float(te_ev)
        self.nu_model = {"hard_sphere": 0, "const": 1}[nu_model]
        self.f0_model = {"maxwell": 0, "druyvesteyn": 1}[f0_model]
        self.cpml = (int(ncpml), float(cpml_order), float(sigma_factor), float(kappa_max),
                     float(alpha_min), float(alpha_max))
        self.src = (int(src_kind), int(src_i), int(src_j), int(src_k), float(src_amp),
                    float(src_f), float(src_tau), float(src_t0))
        X, Y, Z = self.nx, self.ny, self.nz
        self.shapes_e = [(Z + 1, Y + 1, X), (Z + 1, Y, X + 1), (Z, Y + 1, X + 1)]
        self.shapes_h = [(Z, Y, X + 1), (Z, Y + 1, X), (Z + 1, Y, X)]
        ne_ = int(sum(np.prod(s) for s in self.shapes_e))
        nh_ = int(sum(np.prod(s) for s in self.shapes_h))
        self.E = np.zeros(ne_)
        self.H = np.zeros(nh_)
        self.J = np.zeros(ne_)
        self.psi = np.zeros(2 * ne_ + 2 * nh_)
        strict = int(self.model != 0)
        np_ = int(lib().oracle_plasma3d_map(X, Y, Z, _p(self.ne), strict, None, None))
        self.pidx = np.zeros(max(np_, 1), dtype=np.int32)
        self.pcell = np.zeros(4 * max(np_, 1), dtype=np.int32)
        lib().oracle_plasma3d_map(X, Y, Z, _p(self.ne), strict, _p(self.pidx), _p(self.pcell))
        self.npoints = np_
        self.pidx, self.pcell = self.pidx[:np_], self.pcell[:4 * np_].reshape(np_, 4)
        self.cells = np.flatnonzero(self.ne > 0) if strict else np.zeros(0, dtype=np.int64)
        self.ncells = len(self.cells)
        self.df = np.zeros((self.npoints + self.ncells) * self.vdim)
        self.step = 0
        self.dt = self.courant * self.dx / constants()["c"]

    def _views(self, flat, shapes):
        out, o = [], 0
        for s in shapes:
            n = int(np.prod(s))
            out.append(flat[o:o + n].reshape(s))
            o += n
        return out

    def fields(self):
        """dict of shaped views: Ex, Ey, Ez, Hx, Hy, Hz, Jx, Jy, Jz."""
        ex, ey, ez = self._views(self.E, self.shapes_e)
        hx, hy, hz = self._views(self.H, self.shapes_h)
        jx, jy, jz = self._views(self.J, self.shapes_e)
        return dict(Ex=ex, Ey=ey, Ez=ez, Hx=hx, Hy=hy, Hz=hz, Jx=jx, Jy=jy, Jz=jz)

    def run(self, nsteps, probes=()):
        """``probes``: flat indices into E; returns E there after every step."""
        idx = np.ascontiguousarray(probes, dtype=np.int32)
        pout = np.zeros(max(1, nsteps * len(idx)))
        rc = lib().oracle_run3d(
            self.nx, self.ny, self.nz, self.dx, self.courant, *self.cpml,
            self.vdim, self.vmax, self.te, self.nu_model, self.f0_model,
            _p(self.ne), _p(self.nubar), *self.src,
            self.step, int(nsteps),
            _p(self.E), _p(self.H), _p(self.J), _p(self.psi), _p(self.df),
            len(idx), _p(idx) if len(idx) else None, _p(pout), self.model)
        if rc:
            raise ValueError("oracle_run3d rejected its arguments")
        self.step += int(nsteps)
        return pout[: nsteps * len(idx)].reshape(nsteps, len(idx))

    def df_rows(self):
        """F1 rows of the plasma points."""
        return self.df[: self.npoints * self.vdim].reshape(self.npoints, self.vdim)

    def f0_rows(self):
        """F0 - n F0hat rows of the plasma cells (two-term models)."""
        return self.df[self.npoints * self.vdim:].reshape(self.ncells, self.vdim)
