"""ctypes wrapper of the FP64 CPU oracle (``lks_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline leg
of the benchmark, never by the HIP library or its binding.  It takes the plain workload
dictionaries of ``lks_inputs`` and converts them to the oracle's own C structure.

Arrays: scalar fields are flat [ncell] (x fastest), vector fields are [3, ncell].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblks_oracle.so")

_LATTICE = {"D2Q9": 0, "D3Q15": 1, "D3Q19": 2}
_INTERP = {"PAPER": 0, "FLUID_ONE": 1}
_WEIGHT = {"COS4": 0, "LIN": 1}
_BC = {"PERIODIC": 0, "VELOCITY": 1, "PRESSURE": 2, "ZERO_GRADIENT": 3, "NOSLIP": 4}
_OBJ = {"NONE": -1, "POWER": 0, "DRAG": 1, "TORQUE": 2, "J1": 3, "J2": 4, "MASS": 5}
_ADJ = {"EXACT": 0, "PAPER": 1}

_dp = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)


class OrDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("lattice", C.c_int), ("n", C.c_int * 3), ("nd", C.c_int * 3),
        ("xi_G", C.c_double * 3), ("nu", C.c_double), ("interp", C.c_int),
        ("kappa_max", C.c_double), ("q", C.c_double), ("weight", C.c_int),
        ("bc_kind", C.c_int * 6), ("bc_rho", C.c_double * 6), ("bc_u", (C.c_double * 3) * 6),
        ("rho0", C.c_double), ("u0", C.c_double * 3), ("rho_init", _dp), ("u_init", _dp),
        ("kappa_static", _dp), ("g", C.c_double * 3), ("nsteps", C.c_int), ("motion", _dp),
        ("obj_kind", C.c_int), ("obj_n0", C.c_int), ("obj_n1", C.c_int), ("obj_norm", C.c_int),
        ("obj_centre", C.c_double * 3), ("obj_dir", C.c_double * 3), ("obj_mask", _u8p),
        ("adj_form", C.c_int),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, optional OpenMP)."""
    src = os.path.join(_HERE, "lks_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER(OrDesc)
        L.or_validate.argtypes = [P]
        L.or_interp.argtypes = [P, _dp, _dp, _dp]
        L.or_transfer.argtypes = [P, C.c_int, _dp, _dp, _dp]
        L.or_transfer_T.argtypes = [P, C.c_int, _dp, _dp]
        L.or_step.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_apply_bc.argtypes = [P, _dp, _dp]
        L.or_step_T.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_step_T_paper.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_objective_step.argtypes = [P, _dp, _dp, _dp, _dp]
        L.or_objective_step.restype = C.c_double
        L.or_objective_partials.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_solve.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


class Desc:
    """Owns an OrDesc and the numpy arrays it points into."""

    def __init__(self, cfg: dict):
        self.cfg = cfg
        d = OrDesc()
        d.dim = cfg["dim"]
        d.lattice = _LATTICE[cfg["lattice"]]
        for a in range(3):
            d.n[a] = cfg["n"][a]
            d.nd[a] = cfg["nd"][a]
            d.xi_G[a] = cfg["xi_G"][a]
            d.u0[a] = cfg["u0"][a]
            d.g[a] = cfg["body_force"][a]
        d.nu = cfg["nu"]
        d.interp = _INTERP[cfg["interp"]]
        d.kappa_max = cfg["kappa_max"]
        d.q = cfg["q"]
        d.weight = _WEIGHT[cfg["weight"]]
        for f, bc in enumerate(cfg["bc"]):
            d.bc_kind[f] = _BC[bc["kind"]]
            d.bc_rho[f] = bc["rho"]
            for a in range(3):
                d.bc_u[f][a] = bc["u"][a]
        d.rho0 = cfg["rho0"]
        self._keep = []
        self.nc = int(np.prod(cfg["n"]))
        self.nd = int(np.prod(cfg["nd"]))

        def arr(x, size):
            if x is None:
                return None
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
            assert a.size == size
            self._keep.append(a)
            return _ptr(a)

        d.rho_init = arr(cfg.get("rho_init"), self.nc)
        d.u_init = arr(cfg.get("u_init"), 3 * self.nc)
        d.kappa_static = arr(cfg.get("kappa_static"), self.nc)
        d.nsteps = cfg["nsteps"]
        mot = np.ascontiguousarray(cfg["motion"], dtype=np.float64)
        assert mot.shape == (cfg["nsteps"] + 1, 18)
        self._keep.append(mot)
        d.motion = _ptr(mot)
        ob = cfg["objective"]
        d.obj_kind = _OBJ[ob["kind"]]
        d.obj_n0, d.obj_n1, d.obj_norm = ob["n0"], ob["n1"], ob["norm"]
        for a in range(3):
            d.obj_centre[a] = ob["centre"][a]
            d.obj_dir[a] = ob["dir"][a]
        if ob.get("mask") is not None:
            m = np.ascontiguousarray(np.asarray(ob["mask"], dtype=np.uint8).reshape(-1))
            assert m.size == self.nc
            self._keep.append(m)
            d.obj_mask = m.ctypes.data_as(_u8p)
        d.adj_form = _ADJ[cfg.get("adjoint", "EXACT")]
        self.d = d

    @property
    def ref(self):
        return C.byref(self.d)


def validate(cfg: dict) -> int:
    D = Desc(cfg)
    return lib().or_validate(D.ref)


def interp(cfg: dict, gamma: np.ndarray):
    D = Desc(cfg)
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    k = np.empty(D.nd)
    kp = np.empty(D.nd)
    lib().or_interp(D.ref, _ptr(g), _ptr(k), _ptr(kp))
    return k, kp


def transfer(cfg: dict, n: int, kref: np.ndarray):
    D = Desc(cfg)
    kr = np.ascontiguousarray(kref, dtype=np.float64)
    kappa = np.empty(D.nc)
    uS = np.empty((3, D.nc))
    rc = lib().or_transfer(D.ref, n, _ptr(kr), _ptr(kappa), _ptr(uS))
    if rc:
        raise ValueError("transfer footprint leaves the domain")
    return kappa, uS


def transfer_T(cfg: dict, n: int, kbar: np.ndarray) -> np.ndarray:
    D = Desc(cfg)
    kb = np.ascontiguousarray(kbar, dtype=np.float64)
    G = np.zeros(D.nd)
    rc = lib().or_transfer_T(D.ref, n, _ptr(kb), _ptr(G))
    if rc:
        raise ValueError("transfer footprint leaves the domain")
    return G


def apply_bc(cfg: dict, rho: np.ndarray, u: np.ndarray):
    D = Desc(cfg)
    r = np.array(rho, dtype=np.float64).reshape(-1)
    v = np.array(u, dtype=np.float64).reshape(3, -1)
    lib().or_apply_bc(D.ref, _ptr(r), _ptr(v))
    return r, v


def step(cfg: dict, kappa, uS, rho, u):
    D = Desc(cfg)
    k = np.ascontiguousarray(kappa, dtype=np.float64)
    us = np.ascontiguousarray(uS, dtype=np.float64).reshape(3, -1)
    r = np.ascontiguousarray(rho, dtype=np.float64)
    v = np.ascontiguousarray(u, dtype=np.float64).reshape(3, -1)
    ro = np.empty(D.nc)
    uo = np.empty((3, D.nc))
    lib().or_step(D.ref, _ptr(k), _ptr(us), _ptr(r), _ptr(v), _ptr(ro), _ptr(uo))
    return ro, uo


def step_T(cfg: dict, kappa, uS, u_prev, u_cur, P, V):
    D = Desc(cfg)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (kappa, uS, u_prev, u_cur, P, V)]
    Po = np.empty(D.nc)
    Vo = np.empty((3, D.nc))
    kb = np.empty(D.nc)
    lib().or_step_T(D.ref, *[_ptr(x) for x in a], _ptr(Po), _ptr(Vo), _ptr(kb))
    return Po, Vo, kb


def step_T_paper(cfg: dict, kappa, uS, u_prev, u_cur, P, V, U3):
    D = Desc(cfg)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (kappa, uS, u_prev, u_cur, P, V, U3)]
    Po = np.empty(D.nc)
    Vo = np.empty((3, D.nc))
    U3o = np.empty((3, D.nc))
    kb = np.empty(D.nc)
    lib().or_step_T_paper(D.ref, *[_ptr(x) for x in a], _ptr(Po), _ptr(Vo), _ptr(U3o), _ptr(kb))
    return Po, Vo, U3o, kb


def objective_step(cfg: dict, kappa, uS, rho, u) -> float:
    D = Desc(cfg)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (kappa, uS, rho, u)]
    return lib().or_objective_step(D.ref, *[_ptr(x) for x in a])


def objective_partials(cfg: dict, kappa, uS, rho, u):
    D = Desc(cfg)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (kappa, uS, rho, u)]
    dP = np.empty(D.nc)
    dV = np.empty((3, D.nc))
    dK = np.empty(D.nc)
    lib().or_objective_partials(D.ref, *[_ptr(x) for x in a], _ptr(dP), _ptr(dV), _ptr(dK))
    return dP, dV, dK


def solve(cfg: dict, gamma: np.ndarray, grad: bool = True, traj: bool = False) -> dict:
    """Forward (and reverse when ``grad``) solve; returns J, per-step j, dJ/dgamma, final state."""
    D = Desc(cfg)
    N = cfg["nsteps"]
    g = np.ascontiguousarray(gamma, dtype=np.float64).reshape(-1)
    assert g.size == D.nd
    J = C.c_double(0.0)
    jn = np.zeros(N + 1)
    gr = np.zeros(D.nd) if grad else None
    rho = np.empty(D.nc)
    u = np.empty((3, D.nc))
    rt = np.empty((N + 1, D.nc)) if traj else None
    ut = np.empty((N + 1, 3, D.nc)) if traj else None
    rc = lib().or_solve(D.ref, _ptr(g), C.byref(J), _ptr(jn), _ptr(gr), _ptr(rho), _ptr(u),
                        _ptr(rt), _ptr(ut))
    if rc:
        raise ValueError(f"oracle solve failed: {rc}")
    return {"J": J.value, "jn": jn, "grad": gr, "rho": rho, "u": u, "rho_traj": rt, "u_traj": ut}


def num_threads() -> int:
    return int(lib().or_num_threads())
