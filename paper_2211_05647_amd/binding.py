"""ctypes binding of ``libfdtdplasma.so`` (the C ABI of ``include/fdtd_plasma.h``).

Argument marshalling only: every step of the method runs in the HIP kernels.  PyTorch
supplies the device workspace (a uint8 tensor) and the stream.  The library must be
built in-tree (``paper_2211_05647_amd/build.py``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtdplasma.so")

FP64, FP32 = 0, 1
BC_PEC, BC_MUR1, BC_CPML = 0, 1, 2
NU_HARD_SPHERE, NU_CONST = 0, 1
CLOSURE_KINETIC, CLOSURE_MLP = 0, 1
KINETIC_LINEAR, KINETIC_FULL, KINETIC_TWO_TERM = 0, 1, 2
F0_MAXWELL, F0_DRUYVESTEYN = 0, 1
SRC_NONE, SRC_LINE, SRC_POINT = 0, 1, 2
F_E, F_H, F_J, F_DF, F_EX, F_EY, F_HZ, F_JX, F_JY, F_JCX, F_JCY, F_EZ, F_HX, F_HY, F_JZ = range(15)

OK, EINVAL, ENOMEM, EDEVICE, ERANGE, ENUMERIC, ESTATE = 0, -1, -2, -3, -4, -5, -6

_dp = C.POINTER(C.c_double)


class Grid(C.Structure):
    _fields_ = [("dims", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("dx", C.c_double), ("courant", C.c_double),
                ("precision", C.c_int32), ("boundary", C.c_int32),
                ("cpml_cells", C.c_int32), ("cpml_order", C.c_double),
                ("cpml_sigma_factor", C.c_double), ("cpml_kappa_max", C.c_double),
                ("cpml_alpha_min", C.c_double), ("cpml_alpha_max", C.c_double),
                ("nz", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("ne", _dp), ("nu_mean", _dp), ("te_ev", C.c_double), ("nv", C.c_int32),
                ("vmax_over_vth", C.c_double), ("nu_model", C.c_int32),
                ("closure", C.c_int32), ("mlp", C.c_void_p), ("kinetic", C.c_int32),
                ("f0_model", C.c_int32)]


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("i", C.c_int32), ("j", C.c_int32),
                ("amplitude", C.c_double), ("f_hz", C.c_double), ("tau_s", C.c_double),
                ("t0_s", C.c_double), ("k", C.c_int32)]


class Device(C.Structure):
    _fields_ = [("device", C.c_int32), ("hip_stream", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("max_probes", C.c_int32),
                ("probe_capacity", C.c_int32)]


# every symbol the header declares, with its ctypes signature
_SIGS = {
    "fdtd_plasma_workspace_size": ([C.POINTER(Grid), C.POINTER(Profile), C.POINTER(Device), C.POINTER(C.c_size_t)], C.c_int),
    "fdtd_plasma_create": ([C.POINTER(Grid), C.POINTER(Profile), C.POINTER(Source), C.POINTER(Device), C.POINTER(C.c_void_p)], C.c_int),
    "fdtd_plasma_workspace_size_batch": ([C.c_int32, C.POINTER(Grid), C.POINTER(Profile), C.POINTER(C.c_int64), C.c_int32, C.POINTER(Device), C.POINTER(C.c_size_t)], C.c_int),
    "fdtd_plasma_create_batch": ([C.c_int32, C.POINTER(Grid), C.POINTER(Profile), C.POINTER(Source), C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32), C.POINTER(Device), C.POINTER(C.c_void_p)], C.c_int),
    "fdtd_plasma_set_batch_mode": ([C.c_void_p, C.c_int32, C.c_int32], C.c_int),
    "fdtd_plasma_read_taps": ([C.c_void_p, C.c_int32, _dp, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
    "fdtd_plasma_run_status": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "fdtd_plasma_closure_counts": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "fdtd_plasma_set_time_block": ([C.c_void_p, C.c_int32], C.c_int),
    "fdtd_plasma_time_block": ([C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int),
    "fdtd_plasma_step": ([C.c_void_p], C.c_int),
    "fdtd_plasma_run": ([C.c_void_p, C.c_int64], C.c_int),
    "fdtd_plasma_steps": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "fdtd_plasma_field_size": ([C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
    "fdtd_plasma_read_fields": ([C.c_void_p, C.c_int32, C.c_int32, _dp, C.c_size_t, C.POINTER(C.c_int64)], C.c_int),
    "fdtd_plasma_write_fields": ([C.c_void_p, C.c_int32, C.c_int32, _dp, C.c_size_t], C.c_int),
    "fdtd_plasma_add_probe": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "fdtd_plasma_add_probe3d": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "fdtd_plasma_read_probe": ([C.c_void_p, C.c_int32, _dp, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
    "fdtd_plasma_state_size": ([C.c_void_p, C.POINTER(C.c_size_t)], C.c_int),
    "fdtd_plasma_save_state": ([C.c_void_p, C.c_void_p, C.c_size_t], C.c_int),
    "fdtd_plasma_load_state": ([C.c_void_p, C.c_void_p, C.c_size_t], C.c_int),
    "fdtd_plasma_set_tiling": ([C.c_void_p, C.c_int32, C.c_int32], C.c_int),
    "fdtd_plasma_last_run_ms": ([C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "fdtd_plasma_destroy": ([C.c_void_p], None),
    "fdtd_plasma_tap_buffer": ([C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_int32)], C.c_int),
    "fdtd_closure_workspace_size": ([C.c_int32, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
    "fdtd_closure_create": ([C.POINTER(Device), C.c_int32, C.c_int32, C.POINTER(C.c_void_p)], C.c_int),
    "fdtd_closure_set_params": ([C.c_void_p, C.POINTER(C.c_float), C.c_size_t], C.c_int),
    "fdtd_closure_get_params": ([C.c_void_p, C.POINTER(C.c_float), C.c_size_t], C.c_int),
    "fdtd_closure_forward": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "fdtd_closure_grad": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float)], C.c_int),
    "fdtd_closure_adam": ([C.c_void_p, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
    "fdtd_closure_train_step": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.POINTER(C.c_float)], C.c_int),
    "fdtd_closure_single_pole": ([C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "fdtd_closure_replay2v": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_int64, _dp, _dp, C.c_double, C.c_double, C.c_int32, C.c_double, C.c_void_p, C.c_int64], C.c_int),
    "fdtd_closure_make_pairs": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_int64), C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "fdtd_closure_grad_static": ([C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "fdtd_closure_destroy": ([C.c_void_p], None),
    "fdtd_plasma_strerror": ([C.c_int], C.c_char_p),
    "fdtd_plasma_last_error": ([], C.c_char_p),
}

_lib = None


def lib():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2211_05647_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class FdtdError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        msg = lib().fdtd_plasma_last_error().decode()
        super().__init__(f"{what}: {lib().fdtd_plasma_strerror(code).decode()} ({code}): {msg}")


def check(rc, what):
    if rc != OK:
        raise FdtdError(rc, what)


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def make_grid(dims, nx, ny, dx, courant, precision, boundary, cpml_cells=8, cpml_order=3.0,
              sigma_factor=1.0, kappa_max=5.0, alpha_min=0.0, alpha_max=0.05, nz=1):
    return Grid(dims, nx, ny, dx, courant, precision, boundary, cpml_cells, cpml_order,
                sigma_factor, kappa_max, alpha_min, alpha_max, nz)


class Sim:
    """One run (or a batch of 1D runs) on the GPU through the C ABI.

    ``workload``: a ``workloads.Run1D`` / ``Run2D`` (or a list of Run1D for a batch).
    The workspace is a torch uint8 tensor on ``cuda:device``; work goes on torch's
    current stream of that device.
    """

    def __init__(self, workload, precision=FP32, device=0, max_probes=0, probe_capacity=0,
                 closure=CLOSURE_KINETIC, mlp_blob=None, tile=0, cells_per_group=0,
                 taps=None, batch_mode=None, groups=0, time_block=None):
        import torch
        self.torch = torch
        L = lib()
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self.batch = isinstance(workload, (list, tuple))
        runs = list(workload) if self.batch else [workload]
        self.runs = runs
        self._keep = []
        grids, profs, srcs = [], [], []
        for w in runs:
            if hasattr(w, "nz"):
                g = make_grid(3, w.nx, w.ny, w.dx, w.courant, precision,
                              BC_CPML if w.ncpml > 0 else BC_PEC, max(w.ncpml, 0), nz=w.nz)
                src = Source(w.src_kind if w.src_amp != 0 else SRC_NONE, w.src_i, w.src_j,
                             w.src_amp, w.src_f, w.src_tau, w.src_t0, w.src_k)
            elif hasattr(w, "ny"):
                g = make_grid(2, w.nx, w.ny, w.dx, w.courant, precision, BC_CPML, w.ncpml)
                if w.ncpml == 0:
                    g.boundary = BC_PEC
                src = Source(w.src_kind, w.src_i, w.src_j, w.src_amp, w.src_f, w.src_tau, w.src_t0)
            else:
                g = make_grid(1, w.nx, 1, w.dx, w.courant, precision,
                              BC_MUR1 if w.bc == "mur" else BC_PEC, 0)
                src = Source(SRC_POINT if w.src_amp != 0 else SRC_NONE, w.src_node, 0,
                             w.src_amp, w.src_f, w.src_tau, w.src_t0)
            ne, pne = _arr(w.ne)
            nu, pnu = _arr(w.nubar)
            self._keep += [ne, nu]
            mlp_ptr = None
            if mlp_blob is not None:
                self._keep.append(mlp_blob)
                mlp_ptr = mlp_blob.ctypes.data_as(C.c_void_p)
            p = Profile(pne, pnu, w.te_ev, w.nv, w.vmax_over_vth,
                        NU_HARD_SPHERE if w.nu_model == "hard_sphere" else NU_CONST,
                        closure, mlp_ptr,
                        {"linear": KINETIC_LINEAR, "full": KINETIC_FULL,
                         "two_term": KINETIC_TWO_TERM}[getattr(w, "kinetic", "linear")],
                        F0_DRUYVESTEYN if getattr(w, "f0_model", "maxwell") == "druyvesteyn"
                        else F0_MAXWELL)
            grids.append(g)
            profs.append(p)
            srcs.append(src)
        dev = Device(device, C.c_void_p(self.stream.cuda_stream), None, 0, max_probes, probe_capacity)
        nbytes = C.c_size_t()
        if self.batch:
            GA, PA = Grid * len(runs), Profile * len(runs)
            self._ga, self._pa = GA(*grids), PA(*profs)
            self._sa = (Source * len(runs))(*srcs)
            self._steps = (C.c_int64 * len(runs))(*[int(w.steps) for w in runs])
            self.ntap = 0 if taps is None else int(np.asarray(taps).shape[1])
            self._taps = None
            if self.ntap:
                self._taps = np.ascontiguousarray(taps, dtype=np.int32)
            check(L.fdtd_plasma_workspace_size_batch(len(runs), self._ga, self._pa, self._steps, self.ntap,
                                                     C.byref(dev), C.byref(nbytes)),
                  "workspace_size_batch")
        else:
            check(L.fdtd_plasma_workspace_size(C.byref(grids[0]), C.byref(profs[0]), C.byref(dev), C.byref(nbytes)),
                  "workspace_size")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=f"cuda:{device}")
        dev.workspace = C.c_void_p(self.workspace.data_ptr())
        dev.workspace_bytes = self.workspace.numel()
        h = C.c_void_p()
        if self.batch:
            tp = self._taps.ctypes.data_as(C.POINTER(C.c_int32)) if self.ntap else None
            check(L.fdtd_plasma_create_batch(len(runs), self._ga, self._pa, self._sa, self._steps, self.ntap, tp,
                                             C.byref(dev), C.byref(h)),
                  "create_batch")
        else:
            check(L.fdtd_plasma_create(C.byref(grids[0]), C.byref(profs[0]), C.byref(srcs[0]), C.byref(dev), C.byref(h)),
                  "create")
        self.h = h
        if self.batch and (batch_mode is not None or groups):
            mode = 1 if batch_mode is None else batch_mode
            check(L.fdtd_plasma_set_batch_mode(self.h, mode, groups), "set_batch_mode")
        if tile or cells_per_group:
            check(L.fdtd_plasma_set_tiling(self.h, tile, cells_per_group), "set_tiling")
        if time_block is not None:
            self.set_time_block(time_block)

    def close(self):
        if getattr(self, "h", None):
            lib().fdtd_plasma_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, nsteps):
        check(lib().fdtd_plasma_run(self.h, int(nsteps)), "run")

    def step(self):
        check(lib().fdtd_plasma_step(self.h), "step")

    @property
    def steps(self):
        s = C.c_int64()
        check(lib().fdtd_plasma_steps(self.h, C.byref(s)), "steps")
        return s.value

    def read(self, field, run=0):
        n = C.c_size_t()
        check(lib().fdtd_plasma_field_size(self.h, run, field, C.byref(n)), "field_size")
        out = np.empty(n.value, dtype=np.float64)
        st = C.c_int64()
        check(lib().fdtd_plasma_read_fields(self.h, run, field, out.ctypes.data_as(_dp), out.size, C.byref(st)),
              "read_fields")
        return out

    def write(self, field, values, run=0):
        """Overwrite a field (SI units, read_fields layout) of the current state."""
        v = np.ascontiguousarray(values, dtype=np.float64).ravel()
        check(lib().fdtd_plasma_write_fields(self.h, run, field, v.ctypes.data_as(_dp), v.size),
              "write_fields")

    def add_probe(self, field, i, j=0, run=0):
        pid = C.c_int32()
        check(lib().fdtd_plasma_add_probe(self.h, run, field, i, j, C.byref(pid)), "add_probe")
        return pid.value

    def add_probe3d(self, field, i, j, k):
        """3D handles: E component ``field`` (F_EX, F_EY, F_EZ) at storage index (i, j, k)."""
        pid = C.c_int32()
        check(lib().fdtd_plasma_add_probe3d(self.h, field, i, j, k, C.byref(pid)), "add_probe3d")
        return pid.value

    def read_probe(self, pid, n):
        out = np.empty(n, dtype=np.float64)
        got = C.c_size_t()
        check(lib().fdtd_plasma_read_probe(self.h, pid, out.ctypes.data_as(_dp), n, C.byref(got)), "read_probe")
        return out[: got.value]

    def save_state(self):
        n = C.c_size_t()
        check(lib().fdtd_plasma_state_size(self.h, C.byref(n)), "state_size")
        buf = np.empty(n.value, dtype=np.uint8)
        check(lib().fdtd_plasma_save_state(self.h, buf.ctypes.data_as(C.c_void_p), buf.size), "save_state")
        return buf

    def load_state(self, buf):
        check(lib().fdtd_plasma_load_state(self.h, buf.ctypes.data_as(C.c_void_p), buf.size), "load_state")

    def read_taps(self, run):
        """(ntap, steps, 2) array of (E^n in V/m, J^{n+1/2} in A/m^2) at the run's taps."""
        n = self.ntap * max(0, min(self.steps, int(self.runs[run].steps))) * 2
        out = np.empty(max(n, 1), dtype=np.float64)
        got = C.c_size_t()
        check(lib().fdtd_plasma_read_taps(self.h, run, out.ctypes.data_as(_dp), out.size, C.byref(got)), "read_taps")
        return out[: got.value].reshape(self.ntap, -1, 2)

    def run_status(self, run):
        st = C.c_int32()
        check(lib().fdtd_plasma_run_status(self.h, run, C.byref(st)), "run_status")
        return st.value

    def set_time_block(self, steps):
        """Steps per launch of a single FP32 1D run (1 = one step per launch)."""
        check(lib().fdtd_plasma_set_time_block(self.h, int(steps)), "set_time_block")

    def time_block(self, rows=False):
        """Steps per launch in effect; with rows=True also the F1 rows one launch reads."""
        v, r = C.c_int32(), C.c_int64()
        check(lib().fdtd_plasma_time_block(self.h, C.byref(v), C.byref(r)), "time_block")
        return (v.value, r.value) if rows else v.value

    def closure_counts(self):
        """(closure cells, kinetic cells) of a 2D run with the learned closure."""
        a, b = C.c_int64(), C.c_int64()
        check(lib().fdtd_plasma_closure_counts(self.h, C.byref(a), C.byref(b)), "closure_counts")
        return a.value, b.value

    def tap_buffer(self, run):
        """(device pointer, capacity, ntap) of a batch run's tap buffer [ntap][cap][2] FP32."""
        ptr, cap, nt = C.c_void_p(), C.c_int64(), C.c_int32()
        check(lib().fdtd_plasma_tap_buffer(self.h, run, C.byref(ptr), C.byref(cap), C.byref(nt)), "tap_buffer")
        return ptr.value, cap.value, nt.value

    def last_run_ms(self):
        ms = C.c_double()
        check(lib().fdtd_plasma_last_run_ms(self.h, C.byref(ms)), "last_run_ms")
        return ms.value


NPARAM = 19073
NIN = 18


def single_pole(dims, nv, te_ev, nu_model, ne, nu_mean, dt, vmax_over_vth=6.0):
    """(alpha, beta) of the single-pole recurrence of a kinetic cell (library routine)."""
    a, b = C.c_double(), C.c_double()
    check(lib().fdtd_closure_single_pole(dims, nv, vmax_over_vth, te_ev,
                                         NU_HARD_SPHERE if nu_model == "hard_sphere" else NU_CONST,
                                         ne, nu_mean, dt, C.byref(a), C.byref(b)), "single_pole")
    return a.value, b.value


class Closure:
    """The learned closure's trainer/evaluator on the GPU (argument marshalling only).
    Feature rows, targets and outputs are torch float32 tensors on the device."""

    def __init__(self, max_rows=4096, max_series=4096, device=0):
        import torch
        self.torch = torch
        self.stream = torch.cuda.current_stream(device)
        n = C.c_size_t()
        check(lib().fdtd_closure_workspace_size(max_rows, max_series, C.byref(n)), "closure_workspace_size")
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=f"cuda:{device}")
        dev = Device(device, C.c_void_p(self.stream.cuda_stream), C.c_void_p(self.workspace.data_ptr()),
                     self.workspace.numel(), 0, 0)
        h = C.c_void_p()
        check(lib().fdtd_closure_create(C.byref(dev), max_rows, max_series, C.byref(h)), "closure_create")
        self.h = h
        self.max_rows = max_rows

    def close(self):
        if getattr(self, "h", None):
            lib().fdtd_closure_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        check(lib().fdtd_closure_set_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size), "set_params")

    def get_params(self):
        p = np.empty(NPARAM, dtype=np.float32)
        check(lib().fdtd_closure_get_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size), "get_params")
        return p

    def forward(self, X):
        Y = self.torch.empty(X.shape[0], dtype=self.torch.float32, device=X.device)
        check(lib().fdtd_closure_forward(self.h, X.data_ptr(), X.shape[0], Y.data_ptr()), "forward")
        return Y

    def grad(self, X, T):
        g = np.empty(NPARAM, dtype=np.float32)
        loss = C.c_float()
        check(lib().fdtd_closure_grad(self.h, X.data_ptr(), T.data_ptr(), X.shape[0],
                                      g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss)), "grad")
        return loss.value, g

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        check(lib().fdtd_closure_adam(self.h, lr, beta1, beta2, eps), "adam")

    def train_step(self, X, T, lr, want_loss=False):
        loss = C.c_float()
        check(lib().fdtd_closure_train_step(self.h, X.data_ptr(), T.data_ptr(), X.shape[0], lr,
                                            C.byref(loss) if want_loss else None), "train_step")
        return loss.value if want_loss else None

    def replay2v(self, E_ptr, e_stride, e_series_stride, nseries, nsteps, ne, nu, te_ev, dt, J,
                 j_series_stride, nu_model="hard_sphere", vmax_over_vth=6.0):
        ne, pne = _arr(ne)
        nu, pnu = _arr(nu)
        check(lib().fdtd_closure_replay2v(self.h, E_ptr, e_stride, e_series_stride, nseries, nsteps,
                                          pne, pnu, te_ev, vmax_over_vth,
                                          NU_HARD_SPHERE if nu_model == "hard_sphere" else NU_CONST,
                                          dt, J.data_ptr(), j_series_stride), "replay2v")

    def make_pairs(self, E_ptr, e_stride, e_series_stride, J, j_series_stride, series4, idx):
        series4 = np.ascontiguousarray(series4, dtype=np.float32)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        n = idx.size
        X = self.torch.empty((n, NIN), dtype=self.torch.float32, device=J.device)
        T = self.torch.empty(n, dtype=self.torch.float32, device=J.device)
        check(lib().fdtd_closure_make_pairs(self.h, E_ptr, e_stride, e_series_stride, J.data_ptr(),
                                            j_series_stride, series4.shape[0],
                                            series4.ctypes.data_as(C.POINTER(C.c_float)),
                                            idx.ctypes.data_as(C.POINTER(C.c_int64)), n,
                                            X.data_ptr(), T.data_ptr()), "make_pairs")
        return X, T
