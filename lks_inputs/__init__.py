"""Seeded synthetic inputs for the moving-body LKS solver (no solver arithmetic here).

This module only *describes* workloads: design-density fields drawn from a seeded
generator, tables of prescribed rigid motion, boundary-condition lists and objective
settings.  Both the FP64 CPU oracle (``oracle/``) and the HIP library
(``paper_2506_23895_amd``) consume the plain-dict descriptions produced here; each
converts them to its own C structure.  Nothing in this file evaluates any step of the
lattice kinetic scheme, the grid transfer, the Brinkman interpolation or the adjoint.

Motion records follow the paper's rigid-body description (Sec. 2.3, equations for the
position and velocity of a design point): each step n carries the rotation matrix
R^n (row-major 3x3), the angular-velocity vector Omega^n, the position x_G^n of the
point that the design centre xi_G is mapped to, and its velocity u_G^n.  Record n is
used at time t_n = n (lattice units, dt = 1).
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np

MOTION_REC = 18  # R[9], Omega[3], xG[3], uG[3]


# ----------------------------------------------------------------------------------------
# design-density fields
# ----------------------------------------------------------------------------------------
def box_filter(g: np.ndarray) -> np.ndarray:
    """One 3^d box filter: mean over the in-bounds neighbours (the input recipe)."""
    g = np.asarray(g, dtype=np.float64)
    acc = np.zeros_like(g)
    cnt = np.zeros_like(g)
    offs = [(-1, 0, 1)] * g.ndim
    for d in np.array(np.meshgrid(*offs, indexing="ij")).reshape(g.ndim, -1).T:
        src = [slice(max(0, -o), g.shape[a] - max(0, o)) for a, o in enumerate(d)]
        dst = [slice(max(0, o), g.shape[a] - max(0, -o)) for a, o in enumerate(d)]
        acc[tuple(dst)] += g[tuple(src)]
        cnt[tuple(dst)] += 1.0
    return acc / cnt


def gamma_field(nd: Sequence[int], dim: int, seed: int, smooth: bool = True) -> np.ndarray:
    """gamma ~ U(0,1) on the design grid from ``seed``, optionally box-filtered once.

    Returned flat in x-fastest order (index = i + nd0*(j + nd1*k)).
    """
    shape = tuple(int(v) for v in nd[:dim])[::-1]  # (nz, ny, nx) / (ny, nx)
    g = np.random.default_rng(seed).random(shape)
    if smooth:
        g = box_filter(g)
    return np.ascontiguousarray(g.reshape(-1))


# ----------------------------------------------------------------------------------------
# motion tables
# ----------------------------------------------------------------------------------------
def _rot_z(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def motion_rotation(nsteps: int, centre: Sequence[float], omega: float, theta0: float = 0.0) -> np.ndarray:
    """Rotation about the z axis through ``centre`` at constant angular velocity."""
    out = np.zeros((nsteps + 1, MOTION_REC))
    for n in range(nsteps + 1):
        R = _rot_z(theta0 + omega * n)
        out[n, 0:9] = R.reshape(-1)
        out[n, 9:12] = (0.0, 0.0, omega)
        out[n, 12:15] = centre
        out[n, 15:18] = 0.0
    return out


def motion_rotation_axis(nsteps: int, centre: Sequence[float], omega: float,
                         axis: Sequence[float]) -> np.ndarray:
    """Rotation about a fixed unit ``axis`` through ``centre`` at constant angular velocity:
    R(t) from the axis-angle (Rodrigues) form, Omega = omega * axis."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    out = np.zeros((nsteps + 1, MOTION_REC))
    for n in range(nsteps + 1):
        th = omega * n
        R = np.eye(3) + math.sin(th) * K + (1.0 - math.cos(th)) * (K @ K)
        out[n, 0:9] = R.reshape(-1)
        out[n, 9:12] = omega * a
        out[n, 12:15] = centre
        out[n, 15:18] = 0.0
    return out


def motion_heave(nsteps: int, centre: Sequence[float], amp: float, omega: float,
                 theta_amp: float = 0.0) -> np.ndarray:
    """Vertical heave y_G = y_c + amp sin(omega t) with optional pitching theta = theta_amp sin(omega t)."""
    out = np.zeros((nsteps + 1, MOTION_REC))
    for n in range(nsteps + 1):
        s, c = math.sin(omega * n), math.cos(omega * n)
        th = theta_amp * s
        out[n, 0:9] = _rot_z(th).reshape(-1)
        out[n, 9:12] = (0.0, 0.0, theta_amp * omega * c)
        out[n, 12:15] = (centre[0], centre[1] + amp * s, centre[2] if len(centre) > 2 else 0.0)
        out[n, 15:18] = (0.0, amp * omega * c, 0.0)
    return out


def motion_static(nsteps: int, centre: Sequence[float]) -> np.ndarray:
    out = np.zeros((nsteps + 1, MOTION_REC))
    out[:, 0:9] = np.eye(3).reshape(-1)
    out[:, 12:15] = centre
    return out


# ----------------------------------------------------------------------------------------
# workload descriptions
# ----------------------------------------------------------------------------------------
def _bc(kind: str, rho: float = 1.0, u: Sequence[float] = (0.0, 0.0, 0.0)) -> dict:
    return {"kind": kind, "rho": float(rho), "u": tuple(float(v) for v in u)}


def channel_bcs(dim: int, u_in: float, walls: bool = True) -> List[dict]:
    """x- velocity inlet, x+ zero-gradient outlet; y (and z) no-slip walls or periodic."""
    side = _bc("NOSLIP") if walls else _bc("PERIODIC")
    bcs = [_bc("VELOCITY", 1.0, (u_in, 0.0, 0.0)), _bc("ZERO_GRADIENT"), dict(side), dict(side)]
    if dim == 3:
        bcs += [dict(side), dict(side)]
    else:
        bcs += [_bc("PERIODIC"), _bc("PERIODIC")]
    return bcs


def periodic_bcs() -> List[dict]:
    return [_bc("PERIODIC") for _ in range(6)]


def objective(kind: str, n0: int, n1: int, norm: int = 0, centre=(0.0, 0.0, 0.0),
              direction=(1.0, 0.0, 0.0), mask: Optional[np.ndarray] = None) -> dict:
    """Objective settings; norm bit 1 = divide by the number of steps, bit 2 = divide by |mask|."""
    return {"kind": kind, "n0": int(n0), "n1": int(n1), "norm": int(norm),
            "centre": tuple(float(v) for v in centre), "dir": tuple(float(v) for v in direction),
            "mask": mask}


def make_config(*, dim: int, lattice: str, n: Sequence[int], nd: Sequence[int], nu: float,
                nsteps: int, motion: np.ndarray, bcs: List[dict], obj: dict,
                interp: str = "FLUID_ONE", kappa_max: float = 0.1, q: float = 0.1,
                weight: str = "LIN", xi_G: Optional[Sequence[float]] = None,
                rho0: float = 1.0, u0=(0.0, 0.0, 0.0), body_force=(0.0, 0.0, 0.0),
                kappa_static: Optional[np.ndarray] = None, rho_init: Optional[np.ndarray] = None,
                u_init: Optional[np.ndarray] = None, precision: str = "F64",
                checkpoint_every: int = 0, name: str = "custom") -> dict:
    n3 = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    nd3 = tuple(int(v) for v in nd) + (1,) * (3 - len(nd))
    if xi_G is None:
        xi_G = tuple((nd3[a] - 1) / 2.0 if a < dim else 0.0 for a in range(3))
    return {
        "name": name, "dim": dim, "lattice": lattice, "n": n3, "nd": nd3,
        "xi_G": tuple(float(v) for v in xi_G), "nu": float(nu), "interp": interp,
        "kappa_max": float(kappa_max), "q": float(q), "weight": weight, "bc": bcs,
        "rho0": float(rho0), "u0": tuple(float(v) for v in u0),
        "body_force": tuple(float(v) for v in body_force), "kappa_static": kappa_static,
        "rho_init": rho_init, "u_init": u_init, "nsteps": int(nsteps),
        "motion": np.ascontiguousarray(motion, dtype=np.float64), "objective": obj,
        "precision": precision, "checkpoint_every": int(checkpoint_every),
    }


def ncell(cfg: dict) -> int:
    return int(cfg["n"][0] * cfg["n"][1] * cfg["n"][2])


def ndesign(cfg: dict) -> int:
    return int(cfg["nd"][0] * cfg["nd"][1] * cfg["nd"][2])


def nu_from_re(re: float, u: float, length: float) -> float:
    """Kinematic viscosity for Reynolds number ``re`` on velocity ``u`` and length ``length``."""
    return u * length / re


# ---- the five benchmark workloads, restated as seeded synthetic inputs -------------------
U_IN = 0.02


def config_c1(precision: str = "F64") -> dict:
    """64x64 D2Q9 channel, 24x24 design rotating at 2pi/400 about the centre, 400 steps, POWER."""
    n, nd, N = (64, 64), (24, 24), 400
    centre = ((n[0] - 1) / 2.0, (n[1] - 1) / 2.0, 0.0)
    mot = motion_rotation(N, centre, 2 * math.pi / 400)
    return make_config(name="c1_2d_64_fp64", dim=2, lattice="D2Q9", n=n, nd=nd,
                       nu=nu_from_re(40, U_IN, nd[0]), nsteps=N, motion=mot,
                       bcs=channel_bcs(2, U_IN), obj=objective("POWER", 1, N),
                       u0=(U_IN, 0, 0), precision=precision)


def config_c2(precision: str = "F32", nsteps: int = 20000, period: float = 2000.0) -> dict:
    """2048x1024 channel, 512^2 design under heave A=64 + pitch 0.5 sin(wt), w = 2pi/period
    (stated 2pi/2000), forward only."""
    n, nd = (2048, 1024), (512, 512)
    centre = ((n[0] - 1) / 2.0, (n[1] - 1) / 2.0, 0.0)
    w = 2 * math.pi / period
    mot = motion_heave(nsteps, centre, 64.0, w, theta_amp=0.5)
    return make_config(name="c2_2d_2048x1024_fwd", dim=2, lattice="D2Q9", n=n, nd=nd,
                       nu=nu_from_re(200, U_IN, nd[0]), nsteps=nsteps, motion=mot,
                       bcs=channel_bcs(2, U_IN), obj=objective("NONE", 1, 0),
                       u0=(U_IN, 0, 0), precision=precision)


def config_c3(n_side: int = 1024, nd_side: int = 256, precision: str = "F32",
              nsteps: int = 10000, checkpoint_every: int = 100, seed: int = 2,
              period: float = 1000.0) -> dict:
    """D2Q9 channel, rotating design (w = 2pi/period, stated 2pi/1000), time-averaged drag,
    checkpoint every 100 steps."""
    n, nd = (n_side, n_side), (nd_side, nd_side)
    centre = ((n[0] - 1) / 2.0, (n[1] - 1) / 2.0, 0.0)
    mot = motion_rotation(nsteps, centre, 2 * math.pi / period)
    return make_config(name=f"c3_2d_{n_side}_fwdadj", dim=2, lattice="D2Q9", n=n, nd=nd,
                       nu=nu_from_re(100, U_IN, 256), nsteps=nsteps, motion=mot,
                       bcs=channel_bcs(2, U_IN), obj=objective("DRAG", 1, nsteps, norm=1),
                       u0=(U_IN, 0, 0), precision=precision, checkpoint_every=checkpoint_every)


def config_c4(n_side: int = 256, nd_side: int = 96, precision: str = "F32", nsteps: int = 3000,
              checkpoint_every: int = 50, lattice: str = "D3Q19", nu: Optional[float] = None) -> dict:
    """D3Q19 box, x inflow / zero-gradient outflow, periodic y,z, design rotating about z (2pi/1500)."""
    n, nd = (n_side,) * 3, (nd_side,) * 3
    centre = tuple((v - 1) / 2.0 for v in n)
    mot = motion_rotation(nsteps, centre, 2 * math.pi / 1500)
    bcs = [_bc("VELOCITY", 1.0, (U_IN, 0, 0)), _bc("ZERO_GRADIENT"),
           _bc("PERIODIC"), _bc("PERIODIC"), _bc("PERIODIC"), _bc("PERIODIC")]
    return make_config(name=f"c4_3d_{n_side}_fwdadj", dim=3, lattice=lattice, n=n, nd=nd,
                       nu=nu if nu is not None else nu_from_re(100, U_IN, 96), nsteps=nsteps,
                       motion=mot, bcs=bcs,
                       obj=objective("TORQUE", 1, nsteps, centre=centre, direction=(0, 0, 1)),
                       u0=(U_IN, 0, 0), precision=precision, checkpoint_every=checkpoint_every)


def served_job(rng: np.random.Generator, precision: str = "F32") -> dict:
    """One request of the served mix: 2D 128^2..1024^2 or 3D 64^3..160^3, design at 40%,
    500..5000 steps, checkpoints every ceil(sqrt(steps)) steps.  Rotation at a tip speed of 0.1, or
    heave of amplitude 0.1 n at a peak speed of 0.1 (at a fixed period of 2000 steps the peak heave
    speed of the largest 2D grids reaches 0.32, and those jobs go non-finite)."""
    is3d = bool(rng.integers(0, 2))
    rotate = bool(rng.integers(0, 2))
    nsteps = int(rng.integers(500, 5001))
    if is3d:
        s = int(rng.integers(64, 161))
        dim, lat, n = 3, "D3Q19", (s, s, s)
    else:
        s = int(rng.integers(128, 1025))
        dim, lat, n = 2, "D2Q9", (s, s)
    d = int(round(0.4 * s))
    nd = (d,) * dim
    centre = tuple((v - 1) / 2.0 for v in n) + ((0.0,) if dim == 2 else ())
    if rotate:
        tip = (d / 2.0) * math.sqrt(2.0)
        mot = motion_rotation(nsteps, centre, 0.1 / tip)
        obj = objective("POWER", 1, nsteps)
    else:
        mot = motion_heave(nsteps, centre, 0.1 * s, 0.1 / (0.1 * s))
        obj = objective("DRAG", 1, nsteps, norm=1)
    bcs = channel_bcs(dim, U_IN, walls=(dim == 2))
    if dim == 3:
        bcs[2:] = [_bc("PERIODIC")] * 4
    return make_config(name=f"served_{dim}d_{s}", dim=dim, lattice=lat, n=n, nd=nd,
                       nu=nu_from_re(100, U_IN, d), nsteps=nsteps, motion=mot, bcs=bcs, obj=obj,
                       u0=(U_IN, 0, 0), precision=precision,
                       checkpoint_every=int(math.ceil(math.sqrt(nsteps))))
