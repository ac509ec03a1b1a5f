"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a closed form (shear-wave decay,
Poiseuille, Couette, Taylor-Couette), an invariant (mass conservation, uniform flow, rigid
isometry, mirror symmetry), a special case of the transfer (integer shift, quarter turn,
partition of unity, w(0)), a transpose identity, or central finite differences of J.  A
plausible slip anywhere in the oracle (a dropped term, a wrong sign, a transposed index) fails
at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import lks_inputs as I
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def setup_module(_m):
    O.build()


# ------------------------------------------------------------------------------------------
# helpers
# ------------------------------------------------------------------------------------------
def tiny_cfg(dim=2, lattice="D2Q9", weight="LIN", interp="FLUID_ONE", obj="DRAG", bcs=None,
             N=25, nu=0.05, kmax=None, mask=None, norm=1, n=None, nd=None, motion="rotate"):
    n = n or ((14, 12) if dim == 2 else (10, 9, 8))
    nd = nd or ((4, 4) if dim == 2 else (3, 3, 3))
    centre = tuple((v - 1) / 2 for v in n) + ((0.0,) if dim == 2 else ())
    if motion == "rotate":
        mot = I.motion_rotation(N, centre, 2 * math.pi / 60)
    elif motion == "heave":
        mot = I.motion_heave(N, centre, 0.7, 2 * math.pi / 40, theta_amp=0.3)
    elif motion == "tilt":
        mot = I.motion_rotation_axis(N, centre, 2 * math.pi / 60, (0.36, 0.48, 0.8))
    else:
        mot = I.motion_static(N, centre)
    if bcs is None:
        bcs = I.channel_bcs(dim, 0.03)
    if kmax is None:
        kmax = 0.8 if interp == "FLUID_ONE" else 5.0
    d = (0.6, 0.8, 0.0) if obj != "TORQUE" else (0.0, 0.0, 1.0)
    return I.make_config(dim=dim, lattice=lattice, n=n, nd=nd, nu=nu, nsteps=N, motion=mot,
                         bcs=bcs, obj=I.objective(obj, 3, N, norm=norm, centre=centre,
                                                  direction=d, mask=mask),
                         u0=(0.03, 0, 0), weight=weight, interp=interp, kappa_max=kmax)


def fd_grad(cfg, g, h=1e-6):
    fd = np.zeros_like(g)
    for i in range(g.size):
        gp, gm = g.copy(), g.copy()
        gp[i] += h
        gm[i] -= h
        fd[i] = (O.solve(cfg, gp, grad=False)["J"] - O.solve(cfg, gm, grad=False)["J"]) / (2 * h)
    return fd


def A_of(nu):
    return 4.5 * (1.0 / 6.0 - nu)


# ------------------------------------------------------------------------------------------
# P1: central finite differences of J pin the whole reverse sweep
# ------------------------------------------------------------------------------------------
def _bc(kind, rho=1.0, u=(0.0, 0.0, 0.0)):
    return {"kind": kind, "rho": rho, "u": u}


FD_CASES = {
    "lin_fluidone_drag": dict(),
    "cos4": dict(weight="COS4"),
    "paper_interp": dict(interp="PAPER"),
    "power": dict(obj="POWER"),
    "torque": dict(obj="TORQUE"),
    "j2": dict(obj="J2"),
    "heave_pitch": dict(motion="heave", obj="POWER"),
    "pressure_outlet": dict(bcs=[_bc("VELOCITY", 1.0, (0.03, 0, 0)), _bc("PRESSURE", 1.001, (0, 0.002, 0)),
                                 _bc("NOSLIP", 1.0, (0.01, 0, 0)), _bc("ZERO_GRADIENT"),
                                 _bc("PERIODIC"), _bc("PERIODIC")]),
    "periodic_x": dict(bcs=[_bc("PERIODIC"), _bc("PERIODIC"), _bc("NOSLIP"),
                            _bc("VELOCITY", 1.0, (0.02, 0, 0)), _bc("PERIODIC"), _bc("PERIODIC")]),
    "d3q19": dict(dim=3, lattice="D3Q19"),
    "d3q15_cos4_torque": dict(dim=3, lattice="D3Q15", weight="COS4", obj="TORQUE"),
    "d3q19_tilted_axis_cos4": dict(dim=3, lattice="D3Q19", weight="COS4", obj="TORQUE",
                                   motion="tilt", n=(12, 11, 11)),
    "d3q19_walls": dict(dim=3, lattice="D3Q19", obj="POWER",
                        bcs=[_bc("VELOCITY", 1.0, (0.03, 0, 0)), _bc("ZERO_GRADIENT"), _bc("NOSLIP"),
                             _bc("NOSLIP"), _bc("PRESSURE", 1.0), _bc("ZERO_GRADIENT")]),
}


@pytest.mark.parametrize("name", sorted(FD_CASES))
def test_P1_finite_differences(name):
    cfg = tiny_cfg(**FD_CASES[name])
    g = I.gamma_field(cfg["nd"], cfg["dim"], 5)
    r = O.solve(cfg, g)
    fd = fd_grad(cfg, g)
    assert np.abs(fd).max() > 1e-4  # the objective really depends on gamma
    rel = np.abs(fd - r["grad"]).max() / np.abs(fd).max()
    assert rel < 1e-6, rel


def test_P1_j1_on_boundary_mask():
    """J1 (mean pressure on a set of boundary nodes) seeds face nodes: the BC transpose matters."""
    n = (14, 12)
    mask = np.zeros(n[::-1], dtype=np.uint8)
    mask[0, :] = 1          # bottom wall
    mask[:, -1] = 1         # outlet
    cfg = tiny_cfg(obj="J1", mask=mask.reshape(-1), norm=3)
    g = I.gamma_field(cfg["nd"], 2, 7)
    r = O.solve(cfg, g)
    fd = fd_grad(cfg, g)
    assert np.abs(fd - r["grad"]).max() / np.abs(fd).max() < 1e-6


# ------------------------------------------------------------------------------------------
# P2: transpose identities, step by step
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dim,lattice", [(2, "D2Q9"), (3, "D3Q19"), (3, "D3Q15")])
def test_P2_step_transpose_state(dim, lattice):
    """<lam, dPhi/dX dX> == <Phi^T lam, dX>; Phi is quadratic in X so central FD is exact."""
    bcs = (I.channel_bcs(2, 0.03) if dim == 2 else
           [_bc("VELOCITY", 1.0, (0.03, 0, 0)), _bc("PRESSURE", 1.01, (0, 0.01, 0)), _bc("NOSLIP"),
            _bc("ZERO_GRADIENT"), _bc("PERIODIC"), _bc("PERIODIC")])
    cfg = tiny_cfg(dim=dim, lattice=lattice, bcs=bcs)
    nc = int(np.prod(cfg["n"]))
    rng = np.random.default_rng(3)
    kappa = rng.random(nc) * 0.5
    uS = rng.normal(size=(3, nc)) * 0.05
    rho = 1 + 0.01 * rng.normal(size=nc)
    u = 0.05 * rng.normal(size=(3, nc))
    if dim == 2:
        u[2] = 0
        uS[2] = 0
    rho, u = O.apply_bc(cfg, rho, u)
    dr = rng.normal(size=nc)
    du = rng.normal(size=(3, nc))
    if dim == 2:
        du[2] = 0
    P = rng.normal(size=nc)
    V = rng.normal(size=(3, nc))
    if dim == 2:
        V[2] = 0
    h = 1e-3
    rp, up = O.step(cfg, kappa, uS, rho + h * dr, u + h * du)
    rm, um = O.step(cfg, kappa, uS, rho - h * dr, u - h * du)
    lhs = (np.dot(P, rp - rm) + np.sum(V * (up - um))) / (2 * h)
    r1, u1 = O.step(cfg, kappa, uS, rho, u)
    Po, Vo, _ = O.step_T(cfg, kappa, uS, u, u1, P, V)
    rhs = np.dot(Po, dr) + np.sum(Vo * du)
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs)), (lhs, rhs)


def test_P2_step_transpose_kappa():
    cfg = tiny_cfg()
    nc = int(np.prod(cfg["n"]))
    rng = np.random.default_rng(4)
    kappa = rng.random(nc)
    uS = rng.normal(size=(3, nc)) * 0.05
    uS[2] = 0
    rho = 1 + 0.01 * rng.normal(size=nc)
    u = 0.05 * rng.normal(size=(3, nc))
    u[2] = 0
    dk = rng.normal(size=nc)
    P = rng.normal(size=nc)
    V = rng.normal(size=(3, nc))
    V[2] = 0
    h = 1e-5
    rp, up = O.step(cfg, kappa + h * dk, uS, rho, u)
    rm, um = O.step(cfg, kappa - h * dk, uS, rho, u)
    lhs = (np.dot(P, rp - rm) + np.sum(V * (up - um))) / (2 * h)
    r1, u1 = O.step(cfg, kappa, uS, rho, u)
    _, _, kb = O.step_T(cfg, kappa, uS, u, u1, P, V)
    assert abs(lhs - np.dot(kb, dk)) < 1e-8 * max(1, abs(lhs))


@pytest.mark.parametrize("weight", ["LIN", "COS4"])
@pytest.mark.parametrize("dim", [2, 3])
def test_P2_transfer_transpose(weight, dim):
    """<W a, b> over the analysis grid == <a, W^T b> over the design grid (exact to round-off)."""
    cfg = tiny_cfg(dim=dim, lattice="D2Q9" if dim == 2 else "D3Q19", weight=weight,
                   n=(20, 18) if dim == 2 else (14, 13, 12), motion="heave")
    rng = np.random.default_rng(5)
    nd = int(np.prod(cfg["nd"]))
    nc = int(np.prod(cfg["n"]))
    a = rng.normal(size=nd)
    b = rng.normal(size=nc)
    for n in (0, 7, 19):
        kap, _ = O.transfer(cfg, n, a)
        G = O.transfer_T(cfg, n, b)
        assert abs(np.dot(kap, b) - np.dot(a, G)) < 1e-12 * np.abs(kap).sum() * np.abs(b).max()


# ------------------------------------------------------------------------------------------
# P3, P7, P10: invariants
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dim,lattice", [(2, "D2Q9"), (3, "D3Q15"), (3, "D3Q19")])
def test_P3_mass_conserved_periodic_with_moving_body(dim, lattice):
    """Sum_i E_i = rho + (2A/3) div u and the periodic sum of a central divergence is 0, and the
    force leaves rho alone: total mass is constant even with the Brinkman body moving."""
    n = (16, 14) if dim == 2 else (10, 10, 9)
    cfg = tiny_cfg(dim=dim, lattice=lattice, bcs=I.periodic_bcs(), n=n, N=30, obj="MASS",
                   kmax=3.0, motion="heave")
    cfg["objective"] = I.objective("MASS", 1, 30)
    nc = int(np.prod(n))
    rng = np.random.default_rng(1)
    cfg["rho_init"] = 1 + 0.01 * rng.normal(size=nc)
    u0 = 0.03 * rng.normal(size=(3, nc))
    if dim == 2:
        u0[2] = 0
    cfg["u_init"] = u0
    g = I.gamma_field(cfg["nd"], dim, 2)
    r = O.solve(cfg, g, grad=False)
    m0 = cfg["rho_init"].sum()
    assert np.allclose(r["jn"][1:], m0, rtol=0, atol=1e-11 * m0)
    # momentum moves (the body pushes the fluid), so the test is not vacuous
    assert np.abs(r["u"].sum(axis=1) - u0.sum(axis=1)).max() > 1e-6


@pytest.mark.parametrize("dim,lattice", [(2, "D2Q9"), (3, "D3Q15"), (3, "D3Q19")])
def test_P3_momentum_conserved_without_body(dim, lattice):
    n = (12, 10) if dim == 2 else (8, 9, 7)
    cfg = tiny_cfg(dim=dim, lattice=lattice, bcs=I.periodic_bcs(), n=n, N=20, kmax=0.0)
    cfg["objective"] = I.objective("NONE", 1, 0)
    nc = int(np.prod(n))
    rng = np.random.default_rng(9)
    cfg["rho_init"] = 1 + 0.01 * rng.normal(size=nc)
    u0 = 0.03 * rng.normal(size=(3, nc))
    if dim == 2:
        u0[2] = 0
    cfg["u_init"] = u0
    r = O.solve(cfg, I.gamma_field(cfg["nd"], dim, 2), grad=False)
    assert np.abs(r["u"].sum(axis=1) - u0.sum(axis=1)).max() < 1e-12
    assert abs(r["rho"].sum() - cfg["rho_init"].sum()) < 1e-10


@pytest.mark.parametrize("dim,lattice", [(2, "D2Q9"), (3, "D3Q15"), (3, "D3Q19")])
def test_P7_uniform_flow_invariant(dim, lattice):
    n = (10, 9) if dim == 2 else (7, 6, 5)
    cfg = tiny_cfg(dim=dim, lattice=lattice, bcs=I.periodic_bcs(), n=n, N=15, kmax=0.0)
    cfg["objective"] = I.objective("NONE", 1, 0)
    U = (0.05, -0.03, 0.02 if dim == 3 else 0.0)
    cfg["u0"] = U
    cfg["rho0"] = 1.02
    r = O.solve(cfg, I.gamma_field(cfg["nd"], dim, 2), grad=False)
    assert np.abs(r["rho"] - 1.02).max() < 1e-14
    for a in range(3):
        assert np.abs(r["u"][a] - U[a]).max() < 1e-15


def test_P10_zero_sensitivity_design_independent_objective():
    """Total mass on a periodic box does not depend on gamma: the reverse sweep returns 0."""
    cfg = tiny_cfg(bcs=I.periodic_bcs(), n=(14, 12), N=20, kmax=2.0)
    cfg["objective"] = I.objective("MASS", 5, 20)
    rng = np.random.default_rng(4)
    cfg["u_init"] = np.vstack([0.02 * rng.normal(size=(2, 168)), np.zeros((1, 168))])
    g = I.gamma_field(cfg["nd"], 2, 3)
    r = O.solve(cfg, g)
    assert np.abs(r["grad"]).max() < 1e-13
    # the same setting with a design-dependent objective has a clearly non-zero sensitivity
    cfg["objective"] = I.objective("DRAG", 5, 20)
    assert np.abs(O.solve(cfg, g)["grad"]).max() > 1e-4


def test_P11_mirror_symmetry():
    """Symmetric channel, gamma symmetric about the centreline, no rotation, drag along x: the
    state is mirror symmetric (u_y odd) and so is the sensitivity."""
    n, nd, N = (16, 13), (5, 5), 30
    centre = ((n[0] - 1) / 2, (n[1] - 1) / 2, 0.0)
    cfg = I.make_config(dim=2, lattice="D2Q9", n=n, nd=nd, nu=0.05, nsteps=N,
                        motion=I.motion_static(N, centre), bcs=I.channel_bcs(2, 0.03),
                        obj=I.objective("DRAG", 1, N), u0=(0.03, 0, 0), kappa_max=1.0)
    g = I.gamma_field(nd, 2, 8).reshape(nd[1], nd[0])
    g = 0.5 * (g + g[::-1, :])
    r = O.solve(cfg, g.reshape(-1))
    gr = r["grad"].reshape(nd[1], nd[0])
    assert np.abs(gr - gr[::-1, :]).max() < 1e-12 * np.abs(gr).max()
    uy = r["u"][1].reshape(n[1], n[0])
    assert np.abs(uy + uy[::-1, :]).max() < 1e-14
    assert np.abs(gr).max() > 1e-4


# ------------------------------------------------------------------------------------------
# P4, P5, P6: closed forms of the scheme
# ------------------------------------------------------------------------------------------
def shear_gain(k, A):
    """Exact per-step gain of a shear wave (derived from the pull of the equilibrium)."""
    return 1.0 - (1.0 - math.cos(k)) / 3.0 + (A / 9.0) * (1.0 - math.cos(2 * k))


@pytest.mark.parametrize("dim,lattice,axes", [
    (2, "D2Q9", (0, 1)), (2, "D2Q9", (1, 0)),
    (3, "D3Q15", (0, 1)), (3, "D3Q15", (2, 0)), (3, "D3Q19", (0, 1)), (3, "D3Q19", (1, 2))])
@pytest.mark.parametrize("nu", [0.02, 0.1, 0.3])
def test_P4_shear_wave_exact_decay(dim, lattice, axes, nu):
    comp, var = axes
    L = 16
    n = (L, L) if dim == 2 else (L, 6, 5) if var == 0 else (6, L, 5) if var == 1 else (6, 5, L)
    if dim == 3 and var == 0:
        n = (L, 6, 5)
    N = 12
    cfg = tiny_cfg(dim=dim, lattice=lattice, bcs=I.periodic_bcs(), n=n, N=N, nu=nu, kmax=0.0)
    cfg["objective"] = I.objective("NONE", 1, 0)
    nc = int(np.prod(n))
    coords = np.array(np.unravel_index(np.arange(nc), n[::-1]))[::-1]  # (3, nc) x,y,z
    m = 2
    k = 2 * math.pi * m / n[var]
    U = 0.05
    u0 = np.zeros((3, nc))
    u0[comp] = U * np.sin(k * coords[var])
    cfg["u_init"] = u0
    r = O.solve(cfg, I.gamma_field(cfg["nd"], dim, 1), grad=False, traj=True)
    G = shear_gain(k, A_of(nu))
    for step in (1, 5, N):
        expect = u0[comp] * G ** step
        assert np.abs(r["u_traj"][step][comp] - expect).max() < 1e-14
        assert np.abs(r["rho_traj"][step] - 1.0).max() < 1e-14
    # small-k limit of the gain is 1 - nu k^2 (the paper's nu(A) relation)
    kk = 1e-3
    assert abs((1 - shear_gain(kk, A_of(nu))) / kk ** 2 - nu) < 1e-6


def test_P5_poiseuille_fixed_point_and_convergence():
    """Periodic x, no-slip walls at y=0 and y=H, body force g: u = g y (H - y) / (2 nu) exactly."""
    nx, ny = 6, 11
    H = ny - 1
    nu, g = 0.1, 1e-5
    bcs = [_bc("PERIODIC"), _bc("PERIODIC"), _bc("NOSLIP"), _bc("NOSLIP"), _bc("PERIODIC"), _bc("PERIODIC")]
    cfg = tiny_cfg(bcs=bcs, n=(nx, ny), N=60, nu=nu, kmax=0.0)
    cfg["objective"] = I.objective("NONE", 1, 0)
    cfg["body_force"] = (g, 0.0, 0.0)
    y = np.repeat(np.arange(ny), nx).astype(float)
    exact = g * y * (H - y) / (2 * nu)
    u0 = np.zeros((3, nx * ny))
    u0[0] = exact
    cfg["u_init"] = u0
    r = O.solve(cfg, I.gamma_field(cfg["nd"], 2, 1), grad=False)
    assert np.abs(r["u"][0] - exact).max() < 1e-16 + 1e-12 * exact.max()
    assert np.abs(r["u"][1]).max() < 1e-12 * exact.max()
    assert np.abs(r["rho"] - 1).max() < 1e-14
    # from rest it converges to the same profile
    cfg["u_init"] = None
    cfg["u0"] = (0, 0, 0)
    cfg["nsteps"] = 3000
    cfg["motion"] = I.motion_static(3000, (nx / 2, ny / 2, 0))
    cfg["nd"] = (1, 1, 1)
    r = O.solve(cfg, np.zeros(1), grad=False)
    assert np.abs(r["u"][0] - exact).max() < 1e-6 * exact.max()


def test_P6_couette_fixed_point():
    nx, ny, U = 5, 9, 0.04
    H = ny - 1
    bcs = [_bc("PERIODIC"), _bc("PERIODIC"), _bc("NOSLIP"), _bc("VELOCITY", 1.0, (U, 0, 0)),
           _bc("PERIODIC"), _bc("PERIODIC")]
    cfg = tiny_cfg(bcs=bcs, n=(nx, ny), N=40, nu=0.07, kmax=0.0)
    cfg["objective"] = I.objective("NONE", 1, 0)
    y = np.repeat(np.arange(ny), nx).astype(float)
    exact = U * y / H
    u0 = np.zeros((3, nx * ny))
    u0[0] = exact
    cfg["u_init"] = u0
    r = O.solve(cfg, I.gamma_field(cfg["nd"], 2, 1), grad=False)
    assert np.abs(r["u"][0] - exact).max() < 1e-15
    assert np.abs(r["u"][1]).max() < 1e-13 * U


# ------------------------------------------------------------------------------------------
# P8: transfer special cases and the rigid map
# ------------------------------------------------------------------------------------------
def one_frame_cfg(nd, n, rec, dim=2, weight="LIN", xi_G=None):
    mot = np.asarray(rec, dtype=float).reshape(1, 18)
    cfg = I.make_config(dim=dim, lattice="D2Q9" if dim == 2 else "D3Q19", n=n, nd=nd, nu=0.1,
                        nsteps=0, motion=mot, bcs=I.periodic_bcs(), obj=I.objective("NONE", 1, 0),
                        weight=weight, xi_G=xi_G)
    return cfg


def rec_of(R, Om=(0, 0, 0), xG=(0, 0, 0), uG=(0, 0, 0)):
    return list(np.asarray(R, float).reshape(-1)) + list(Om) + list(xG) + list(uG)


def test_P8_integer_shift_lin_is_exact_copy():
    nd, n = (5, 4), (16, 14)
    cfg = one_frame_cfg(nd, n, rec_of(np.eye(3), xG=(7, 6, 0)), xi_G=(2, 1, 0))
    kref = np.arange(1, 21, dtype=float)
    kap, uS = O.transfer(cfg, 0, kref)
    K = kap.reshape(n[1], n[0])
    expect = np.zeros_like(K)
    expect[5:9, 5:10] = kref.reshape(4, 5)  # xi=(i,j) -> x=(i+5, j+5)
    assert np.array_equal(K, expect)
    assert np.abs(uS).max() == 0.0


def test_P8_integer_shift_cos4_is_quarter_half_quarter_smoothing():
    nd, n = (3, 3), (14, 14)
    cfg = one_frame_cfg(nd, n, rec_of(np.eye(3), xG=(6, 6, 0)), weight="COS4", xi_G=(1, 1, 0))
    kref = np.zeros(9)
    kref[4] = 1.0  # single design point at x = (6, 6)
    kap, _ = O.transfer(cfg, 0, kref)
    K = kap.reshape(14, 14)
    k1 = np.array([0.25, 0.5, 0.25])
    expect = np.zeros((14, 14))
    expect[5:8, 5:8] = np.outer(k1, k1)
    # w(0) = 1/2 and w(+-1) = 1/4 (the printed "1 - cos" would give w(0) = 0)
    assert np.abs(K - expect).max() < 1e-15


def test_P8_quarter_turn_is_permutation():
    nd, n = (4, 3), (16, 16)
    R = [[0, -1, 0], [1, 0, 0], [0, 0, 1]]
    cfg = one_frame_cfg(nd, n, rec_of(R, xG=(8, 8, 0)), xi_G=(1, 1, 0))
    kref = np.arange(1, 13, dtype=float)
    kap, _ = O.transfer(cfg, 0, kref)
    K = kap.reshape(16, 16)
    for j in range(3):
        for i in range(4):
            # x = R (xi - xi_G) + x_G = (-(j-1), i-1) + (8, 8)
            assert K[8 + (i - 1), 8 - (j - 1)] == kref[i + 4 * j]
    assert np.count_nonzero(K) == 12


@pytest.mark.parametrize("weight", ["LIN", "COS4"])
def test_P8_partition_of_unity_axis_aligned(weight):
    """Uniform kappa_ref at theta = 0 and a fractional offset: interior kappa is exactly uniform."""
    nd, n = (12, 12), (24, 24)
    cfg = one_frame_cfg(nd, n, rec_of(np.eye(3), xG=(11.3, 11.7, 0)), weight=weight)
    kap, uS = O.transfer(cfg, 0, np.full(144, 0.7))
    K = kap.reshape(24, 24)
    assert np.abs(K[9:14, 9:14] - 0.7).max() < 1e-14


def test_P8_rigid_map_isometry_and_velocity():
    """Recover x_ref of each design point from the centroid of its LIN hat (exact for a hat), then
    check distances are preserved and u_S / sum(W) equals dx_ref/dt (central FD in time)."""
    n = (40, 40)
    N = 4
    centre = (19.2, 20.4, 0.0)
    w = 0.13
    mot = I.motion_heave(N, centre, 1.7, w, theta_amp=0.9)
    nd = (3, 2)
    cfg = I.make_config(dim=2, lattice="D2Q9", n=n, nd=nd, nu=0.1, nsteps=N, motion=mot,
                        bcs=I.periodic_bcs(), obj=I.objective("NONE", 1, 0), weight="LIN")
    xs = np.arange(n[0] * n[1]) % n[0]
    ys = np.arange(n[0] * n[1]) // n[0]

    def points(step):
        P = []
        for p in range(6):
            kr = np.zeros(6)
            kr[p] = 1.0
            kap, _ = O.transfer(cfg, step, kr)
            P.append((np.dot(kap, xs) / kap.sum(), np.dot(kap, ys) / kap.sum()))
        return np.array(P)

    P2 = points(2)
    xi = np.array([(i, j) for j in range(2) for i in range(3)], dtype=float)
    dP = np.linalg.norm(P2[:, None] - P2[None], axis=-1)
    dX = np.linalg.norm(xi[:, None] - xi[None], axis=-1)
    assert np.abs(dP - dX).max() < 1e-12
    # velocity: single-point design grid so u_S is that point's rigid velocity times W
    vel_fd = (points(3) - points(1)) / 2.0
    cfg1 = dict(cfg)
    for p in range(6):
        i, j = p % 3, p // 3
        cfg1 = I.make_config(dim=2, lattice="D2Q9", n=n, nd=(1, 1), nu=0.1, nsteps=N,
                             motion=mot, bcs=I.periodic_bcs(), obj=I.objective("NONE", 1, 0),
                             weight="LIN", xi_G=(1 - i, 0.5 - j, 0))
        kap, uS = O.transfer(cfg1, 2, np.ones(1))
        v = uS[:2].sum(axis=1) / kap.sum()
        assert np.abs(v - vel_fd[p]).max() < 5e-3 * max(1.0, np.abs(vel_fd[p]).max())


def test_P8_rigid_map_isometry_and_velocity_3d_tilted_axis():
    """The same recovery in 3D for a rotation about a tilted axis (trilinear hats): distances
    between design points are preserved, points on the axis stay put, and u_S / sum(W) equals
    dx_ref/dt (central FD in time)."""
    n = (20, 20, 20)
    N = 4
    centre = (9.3, 10.1, 9.6)
    axis = np.array([0.36, 0.48, 0.8])
    mot = I.motion_rotation_axis(N, centre, 0.21, axis)
    nd = (3, 3, 3)
    xi_G = (1.0, 1.0, 1.0)
    cfg = I.make_config(dim=3, lattice="D3Q19", n=n, nd=nd, nu=0.1, nsteps=N, motion=mot,
                        bcs=I.periodic_bcs(), obj=I.objective("NONE", 1, 0), weight="LIN", xi_G=xi_G)
    idx = np.arange(n[0] * n[1] * n[2])
    X = np.stack([idx % n[0], (idx // n[0]) % n[1], idx // (n[0] * n[1])], axis=1).astype(float)

    def points(step, c=cfg, npts=27):
        P = []
        for p in range(npts):
            kr = np.zeros(npts)
            kr[p] = 1.0
            kap, _ = O.transfer(c, step, kr)
            P.append(kap @ X / kap.sum())
        return np.array(P)

    P2 = points(2)
    xi = np.array([(i, j, k) for k in range(3) for j in range(3) for i in range(3)], dtype=float)
    dP = np.linalg.norm(P2[:, None] - P2[None], axis=-1)
    dX = np.linalg.norm(xi[:, None] - xi[None], axis=-1)
    assert np.abs(dP - dX).max() < 1e-12
    assert np.abs(P2[13] - np.asarray(centre)).max() < 1e-12        # xi_G sits on the axis
    vel_fd = (points(3) - points(1)) / 2.0
    assert np.abs(vel_fd[13]).max() < 1e-12
    for p in (0, 5, 22):
        i, j, k = p % 3, (p // 3) % 3, p // 9
        c1 = I.make_config(dim=3, lattice="D3Q19", n=n, nd=(1, 1, 1), nu=0.1, nsteps=N, motion=mot,
                           bcs=I.periodic_bcs(), obj=I.objective("NONE", 1, 0), weight="LIN",
                           xi_G=(xi_G[0] - i, xi_G[1] - j, xi_G[2] - k))
        kap, uS = O.transfer(c1, 2, np.ones(1))
        v = uS[:3].sum(axis=1) / kap.sum()
        assert np.abs(v - vel_fd[p]).max() < 5e-3 * max(1.0, np.abs(vel_fd[p]).max())
        # rigid velocity is perpendicular to the axis
        assert abs(np.dot(v, axis)) < 1e-12


def test_interp_forms():
    g = np.linspace(0, 1, 11)
    cfgp = tiny_cfg(interp="PAPER", kmax=7.0)
    cfgf = tiny_cfg(interp="FLUID_ONE", kmax=7.0)
    cfgp["nd"] = cfgf["nd"] = (11, 1, 1)
    kp, dp = O.interp(cfgp, g)
    kf, df = O.interp(cfgf, g)
    q = 0.1
    assert kp[0] == 0.0 and abs(kp[-1] - 7.0) < 1e-15          # gamma = 1 is solid (paper)
    assert kf[-1] == 0.0 and abs(kf[0] - 7.0) < 1e-15          # mirror form: gamma = 1 is fluid
    assert np.abs(kf - kp[::-1]).max() < 1e-14                 # I_fluid(g) = I_paper(1 - g)
    h = 1e-6
    kph, _ = O.interp(cfgp, g + h)
    kpm, _ = O.interp(cfgp, g - h)
    assert np.abs((kph - kpm) / (2 * h) - dp).max() < 1e-6 * np.abs(dp).max()
    assert abs(kp[5] - 7.0 * q * 0.5 / (0.5 + q)) < 1e-15


# ------------------------------------------------------------------------------------------
# P9: the paper's Appendix check (Taylor-Couette flow of a rotating disc in a static ring)
# ------------------------------------------------------------------------------------------
@pytest.mark.slow
def test_P9_taylor_couette_profile():
    """A disc of design points (gamma = 1) spins inside a static Brinkman ring.  The steady
    azimuthal velocity must follow the Appendix's closed form up to the smearing of the interface
    by the transfer kernel: it lies between the closed form for the nominal inner radius and the
    one for the radius grown by the LIN support (one cell), and within 8% of u_d of the nominal."""
    fx = json.load(open(os.path.join(GOLDEN, "taylor_couette.json")))
    scale = 0.4  # the paper's L=200, r1=45, r2=70 scaled down to keep the CPU test short
    L, r1, r2 = int(fx["L"] * scale), fx["r1"] * scale, fx["r2"] * scale
    ud, nu, N, kmax = 0.02, 0.1, 7000, 10.0
    w1 = ud / r1
    c = ((L - 1) / 2.0, (L - 1) / 2.0, 0.0)
    ndn = int(2 * r1 + 5)
    xg = np.arange(ndn) - (ndn - 1) / 2.0
    XX, YY = np.meshgrid(xg, xg)
    gamma = (np.hypot(XX, YY) <= r1).astype(float).reshape(-1)
    xs = np.arange(L * L) % L - c[0]
    ys = np.arange(L * L) // L - c[1]
    rr = np.hypot(xs, ys)
    ks = np.where(rr >= r2, kmax, 0.0)
    cfg = I.make_config(dim=2, lattice="D2Q9", n=(L, L), nd=(ndn, ndn), nu=nu, nsteps=N,
                        motion=I.motion_rotation(N, c, w1), bcs=I.periodic_bcs(),
                        obj=I.objective("NONE", 1, 0), interp="PAPER", kappa_max=kmax,
                        kappa_static=ks)
    r = O.solve(cfg, gamma, grad=False)
    ux, uy = r["u"][0], r["u"][1]
    ut = (-ys * ux + xs * uy) / np.maximum(rr, 1e-9)
    sel = (rr > r1 + 2.5) & (rr < r2 - 2.5)
    rs = rr[sel]

    def closed(a):  # inner radius a spinning at w1, outer radius r2 at rest
        return w1 * a * a / (r2 ** 2 - a ** 2) * (r2 ** 2 / rs - rs)

    lo, hi = closed(r1), closed(r1 + 1.0)
    assert np.all(ut[sel] >= lo - 0.01 * ud)
    assert np.all(ut[sel] <= hi + 0.01 * ud)
    assert np.abs(ut[sel] - lo).max() / ud < 0.08
