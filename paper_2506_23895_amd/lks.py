"""Python binding of the C ABI in include/lks.h (argument marshalling only).

Every step of the forward sweep, the reverse sweep and the sensitivity runs inside liblks.so
(HIP kernels for gfx950).  There is no CPU fallback: if the library is missing, importing the
binding raises.

Workloads are the plain dictionaries of ``lks_inputs``.  Host buffers are numpy arrays in the
context precision; with ``io_on_device=True`` the caller passes torch CUDA tensors instead and
their device pointers go straight to the library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblks.so")

LKS_OK, LKS_EINVAL, LKS_ENOMEM, LKS_ESTATE, LKS_ENONFINITE, LKS_EDEVICE, LKS_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
STATE_FINAL = -1

_LATTICE = {"D2Q9": 0, "D3Q15": 1, "D3Q19": 2}
_INTERP = {"PAPER": 0, "FLUID_ONE": 1}
_WEIGHT = {"COS4": 0, "LIN": 1}
_BC = {"PERIODIC": 0, "VELOCITY": 1, "PRESSURE": 2, "ZERO_GRADIENT": 3, "NOSLIP": 4}
_OBJ = {"NONE": -1, "POWER": 0, "DRAG": 1, "TORQUE": 2, "J1": 3, "J2": 4, "MASS": 5}
_PREC = {"F32": 0, "F64": 1}
_ADJ = {"EXACT": 0, "PAPER": 1}

EXPORTS = ["lks_query_bytes", "lks_create", "lks_destroy", "lks_forward", "lks_adjoint",
           "lks_sensitivity", "lks_read_state", "lks_read_objective_steps", "lks_set_timing",
           "lks_kernel_timing", "lks_last_error", "lks_strerror", "lks_batch_create",
           "lks_batch_destroy", "lks_begin", "lks_batch_round", "lks_batch_error", "lks_poll",
           "lks_finish", "lks_forward_noalloc"]


class LksBc(C.Structure):
    _fields_ = [("kind", C.c_int), ("rho", C.c_double), ("u", C.c_double * 3)]


class LksMotion(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("omega", C.c_double * 3), ("xG", C.c_double * 3),
                ("uG", C.c_double * 3)]


class LksObjective(C.Structure):
    _fields_ = [("kind", C.c_int), ("n0", C.c_int), ("n1", C.c_int), ("normalize", C.c_int),
                ("centre", C.c_double * 3), ("dir", C.c_double * 3),
                ("mask", C.POINTER(C.c_uint8))]


class LksDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("lattice", C.c_int), ("n", C.c_int * 3), ("nd", C.c_int * 3),
        ("xi_G", C.c_double * 3), ("nu", C.c_double), ("interp", C.c_int),
        ("kappa_max", C.c_double), ("q", C.c_double), ("weight", C.c_int), ("bc", LksBc * 6),
        ("rho0", C.c_double), ("u0", C.c_double * 3), ("rho_init", C.POINTER(C.c_double)),
        ("u_init", C.POINTER(C.c_double)), ("kappa_static", C.POINTER(C.c_double)),
        ("body_force", C.c_double * 3), ("nsteps", C.c_int), ("motion", C.POINTER(LksMotion)),
        ("objective", LksObjective), ("precision", C.c_int), ("checkpoint_every", C.c_int),
        ("io_on_device", C.c_int), ("stream", C.c_void_p), ("hbm_budget_bytes", C.c_size_t),
        ("adjoint_form", C.c_int), ("zchunk", C.c_int),
    ]


class LksError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def lib():
    """Load liblks.so (raises if it has not been built: there is no fallback path)."""
    global _lib
    if _lib is None:
        # When torch is present, load its HIP runtime first: liblks.so then binds to the same
        # libamdhip64 (matching SONAME), so torch tensors and the library share one runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with paper_2506_23895_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.lks_query_bytes.argtypes = [C.POINTER(LksDesc), C.POINTER(C.c_size_t)]
        L.lks_create.argtypes = [C.POINTER(LksDesc), C.POINTER(P)]
        L.lks_destroy.argtypes = [P]
        L.lks_destroy.restype = None
        L.lks_forward.argtypes = [P, P, C.POINTER(C.c_double)]
        L.lks_adjoint.argtypes = [P]
        L.lks_sensitivity.argtypes = [P, P]
        L.lks_read_state.argtypes = [P, C.c_int, P, P]
        L.lks_read_objective_steps.argtypes = [P, C.POINTER(C.c_double)]
        L.lks_set_timing.argtypes = [P, C.c_int]
        L.lks_kernel_timing.argtypes = [P, C.c_int, C.POINTER(C.c_long), C.POINTER(C.c_double)]
        L.lks_last_error.argtypes = [P]
        L.lks_last_error.restype = C.c_char_p
        L.lks_strerror.argtypes = [C.c_int]
        L.lks_strerror.restype = C.c_char_p
        L.lks_batch_create.argtypes = [P, C.POINTER(P)]
        L.lks_batch_destroy.argtypes = [P]
        L.lks_batch_destroy.restype = None
        L.lks_begin.argtypes = [P, P, P]
        L.lks_batch_round.argtypes = [P, C.POINTER(P), C.c_int, C.POINTER(C.c_int)]
        L.lks_batch_error.argtypes = [P]
        L.lks_batch_error.restype = C.c_char_p
        L.lks_poll.argtypes = [P]
        L.lks_finish.argtypes = [P, C.POINTER(C.c_double)]
        L.lks_forward_noalloc.argtypes = [C.POINTER(LksDesc), P, C.POINTER(C.c_double), P, P]
        _lib = L
    return _lib


class _DescHolder:
    """An LksDesc plus the arrays it points into (kept alive while the descriptor is used)."""

    def __init__(self, cfg: dict, io_on_device: bool = False, stream: Optional[int] = None,
                 hbm_budget: int = 0):
        d = LksDesc()
        self.keep = []
        d.dim = cfg["dim"]
        d.lattice = _LATTICE[cfg["lattice"]]
        for a in range(3):
            d.n[a] = cfg["n"][a]
            d.nd[a] = cfg["nd"][a]
            d.xi_G[a] = cfg["xi_G"][a]
            d.u0[a] = cfg["u0"][a]
            d.body_force[a] = cfg["body_force"][a]
        d.nu = cfg["nu"]
        d.interp = _INTERP[cfg["interp"]]
        d.kappa_max = cfg["kappa_max"]
        d.q = cfg["q"]
        d.weight = _WEIGHT[cfg["weight"]]
        for f, bc in enumerate(cfg["bc"]):
            d.bc[f].kind = _BC[bc["kind"]]
            d.bc[f].rho = bc["rho"]
            for a in range(3):
                d.bc[f].u[a] = bc["u"][a]
        d.rho0 = cfg["rho0"]
        self.ncell = int(np.prod(cfg["n"]))

        def dptr(x, size):
            if x is None:
                return None
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
            if a.size != size:
                raise ValueError("field has the wrong size")
            self.keep.append(a)
            return a.ctypes.data_as(C.POINTER(C.c_double))

        d.rho_init = dptr(cfg.get("rho_init"), self.ncell)
        d.u_init = dptr(cfg.get("u_init"), 3 * self.ncell)
        d.kappa_static = dptr(cfg.get("kappa_static"), self.ncell)
        d.nsteps = cfg["nsteps"]
        mot = np.ascontiguousarray(cfg["motion"], dtype=np.float64)
        if mot.shape != (cfg["nsteps"] + 1, 18):
            raise ValueError("motion table must be (nsteps + 1, 18)")
        self.keep.append(mot)
        d.motion = C.cast(mot.ctypes.data, C.POINTER(LksMotion))
        ob = cfg["objective"]
        d.objective.kind = _OBJ[ob["kind"]]
        d.objective.n0, d.objective.n1, d.objective.normalize = ob["n0"], ob["n1"], ob["norm"]
        for a in range(3):
            d.objective.centre[a] = ob["centre"][a]
            d.objective.dir[a] = ob["dir"][a]
        if ob.get("mask") is not None:
            m = np.ascontiguousarray(np.asarray(ob["mask"], dtype=np.uint8).reshape(-1))
            self.keep.append(m)
            d.objective.mask = m.ctypes.data_as(C.POINTER(C.c_uint8))
        d.precision = _PREC[cfg["precision"]]
        d.checkpoint_every = cfg["checkpoint_every"]
        d.io_on_device = 1 if io_on_device else 0
        d.stream = stream
        d.hbm_budget_bytes = int(hbm_budget)
        d.adjoint_form = _ADJ[cfg.get("adjoint", "EXACT")]
        d.zchunk = int(cfg.get("zchunk", 0))
        self.d = d


def _check(rc: int, ctx=None):
    if rc != LKS_OK:
        msg = lib().lks_last_error(ctx).decode() if ctx is not None else lib().lks_last_error(None).decode()
        raise LksError(rc, msg or lib().lks_strerror(rc).decode())


def _addr(x):
    """Address of a torch tensor's or numpy array's data (None stays NULL)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return C.c_void_p(int(x.data_ptr()))
    return C.c_void_p(x.ctypes.data)


def forward_noalloc(cfg: dict, gamma, drho=None, u=None, stream: Optional[int] = None) -> float:
    """lks_forward_noalloc: the forward sweep with every kernel buffer in the library's static
    device scratch.  gamma [nd], drho [ncell] and u [dim, ncell] in the workload precision (torch
    tensors or numpy arrays; the outputs may be None).  Returns J."""
    h = _DescHolder(cfg, io_on_device=True, stream=stream)
    J = C.c_double(0.0)
    _check(lib().lks_forward_noalloc(C.byref(h.d), _addr(gamma), C.byref(J), _addr(drho), _addr(u)))
    return J.value


def query_bytes(cfg: dict, hbm_budget: int = 0) -> int:
    h = _DescHolder(cfg, hbm_budget=hbm_budget)
    out = C.c_size_t(0)
    _check(lib().lks_query_bytes(C.byref(h.d), C.byref(out)))
    return int(out.value)


class Solver:
    """One lks_ctx: forward, adjoint and sensitivity of a workload dictionary."""

    def __init__(self, cfg: dict, io_on_device: bool = False, stream: Optional[int] = None,
                 hbm_budget: int = 0):
        self.cfg = cfg
        self.dtype = np.float64 if cfg["precision"] == "F64" else np.float32
        self.io_on_device = io_on_device
        self.dim = cfg["dim"]
        self.ncell = int(np.prod(cfg["n"]))
        self.nd = int(np.prod(cfg["nd"]))
        h = _DescHolder(cfg, io_on_device=io_on_device, stream=stream, hbm_budget=hbm_budget)
        self._ctx = C.c_void_p(None)
        _check(lib().lks_create(C.byref(h.d), C.byref(self._ctx)))

    # -- buffers ----------------------------------------------------------------------------
    def _in(self, x, size):
        if self.io_on_device:
            return C.c_void_p(int(x.data_ptr())), x
        a = np.ascontiguousarray(np.asarray(x, dtype=self.dtype).reshape(-1))
        if a.size != size:
            raise ValueError("wrong size")
        return C.c_void_p(a.ctypes.data), a

    def forward(self, gamma) -> float:
        p, keep = self._in(gamma, self.nd)
        J = C.c_double(0.0)
        _check(lib().lks_forward(self._ctx, p, C.byref(J)), self._ctx)
        del keep
        return J.value

    def adjoint(self) -> None:
        _check(lib().lks_adjoint(self._ctx), self._ctx)

    def sensitivity(self, out=None):
        if self.io_on_device:
            _check(lib().lks_sensitivity(self._ctx, C.c_void_p(int(out.data_ptr()))), self._ctx)
            return out
        o = np.empty(self.nd, dtype=self.dtype) if out is None else out
        _check(lib().lks_sensitivity(self._ctx, C.c_void_p(o.ctypes.data)), self._ctx)
        return o

    def read_state(self, which: int = STATE_FINAL) -> Tuple[np.ndarray, np.ndarray]:
        """(rho - 1 [ncell], u [dim, ncell]) on the host."""
        if self.io_on_device:
            raise RuntimeError("read_state_device() for io_on_device contexts")
        r = np.empty(self.ncell, dtype=self.dtype)
        u = np.empty((self.dim, self.ncell), dtype=self.dtype)
        _check(lib().lks_read_state(self._ctx, which, C.c_void_p(r.ctypes.data),
                                    C.c_void_p(u.ctypes.data)), self._ctx)
        return r, u

    def read_state_device(self, which: int, drho, u) -> None:
        _check(lib().lks_read_state(self._ctx, which, C.c_void_p(int(drho.data_ptr())),
                                    C.c_void_p(int(u.data_ptr()))), self._ctx)

    def objective_steps(self) -> np.ndarray:
        jn = np.empty(self.cfg["nsteps"] + 1)
        _check(lib().lks_read_objective_steps(self._ctx, jn.ctypes.data_as(C.POINTER(C.c_double))), self._ctx)
        return jn

    def set_timing(self, every: int) -> None:
        _check(lib().lks_set_timing(self._ctx, every), self._ctx)

    def kernel_timing(self, kind: int) -> Tuple[int, float]:
        cnt = C.c_long(0)
        ms = C.c_double(0.0)
        _check(lib().lks_kernel_timing(self._ctx, kind, C.byref(cnt), C.byref(ms)), self._ctx)
        return int(cnt.value), float(ms.value)

    # -- continuous batching (device IO) -----------------------------------------------------
    def begin(self, gamma, out) -> None:
        """Start an evaluation whose kernels run in Batch.round() calls; keep gamma/out alive."""
        self._begun = (gamma, out)
        _check(lib().lks_begin(self._ctx, C.c_void_p(int(gamma.data_ptr())),
                               C.c_void_p(int(out.data_ptr()))), self._ctx)

    def poll(self) -> bool:
        rc = lib().lks_poll(self._ctx)
        if rc < 0:
            _check(rc, self._ctx)
        return rc == 1

    def finish(self) -> float:
        J = C.c_double(0.0)
        _check(lib().lks_finish(self._ctx, C.byref(J)), self._ctx)
        self._begun = None
        return J.value

    def close(self) -> None:
        if self._ctx:
            lib().lks_destroy(self._ctx)
            self._ctx = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """lks_batch: advance many contexts one micro-step per round with shared kernel launches."""

    def __init__(self, stream: Optional[int] = None):
        self._b = C.c_void_p(None)
        _check(lib().lks_batch_create(stream, C.byref(self._b)))

    def round(self, solvers) -> np.ndarray:
        n = len(solvers)
        arr = (C.c_void_p * n)(*[s._ctx for s in solvers])
        done = (C.c_int * n)()
        rc = lib().lks_batch_round(self._b, arr, n, done)
        if rc != LKS_OK:
            raise LksError(rc, lib().lks_batch_error(self._b).decode())
        return np.frombuffer(done, dtype=np.int32).copy()

    def close(self) -> None:
        if self._b:
            lib().lks_batch_destroy(self._b)
            self._b = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
