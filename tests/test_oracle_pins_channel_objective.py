"""Pins of the oracle's outflow rules and objective densities against closed forms.

Channel rules (Sec. 2.2, Eqs. bc_rho and bc_u, macroscopic values prescribed directly):
  * a pressure-driven channel (pressure held at both ends, no-slip walls) has the exact discrete
    fixed point rho linear in x, u_x = g y (H - y) / (2 nu) with g = -(1/3) d rho/dx (p = rho/3,
    Sec. 2.1): the pull is exact on a linear rho and the strain and its one-sided wall rows are
    exact on a quadratic u;
  * a velocity-inlet channel with the zero-gradient outflow develops to a steady state: the
    total mass stops changing, the downstream profile is a parabola and the volume flux is the
    same through every developed cross-section.  Reading "zero-gradient" as a copy of rho as
    well as u leaves the pressure level free and fails the first of these (mass grows every
    step).

Objective densities (Sec. 2.5 for J1 and J2; the body-force objectives use F_b = kappa (u - u_S),
the reaction of the Brinkman force on the fluid): values on constructed fields whose sums have
a closed form, through the single-step routine and through the whole solve (window, rectangle
rule, NORM_TIME and NORM_MASK).
"""
import math

import numpy as np
import pytest

import lks_inputs as I
from oracle import oracle as O


def setup_module(_m):
    O.build()


def _bc(kind, rho=1.0, u=(0.0, 0.0, 0.0)):
    return {"kind": kind, "rho": rho, "u": u}


def _channel_cfg(n, nu, bcs, nsteps=1, u0=(0.0, 0.0, 0.0)):
    centre = ((n[0] - 1) / 2.0, (n[1] - 1) / 2.0, 0.0)
    return I.make_config(dim=2, lattice="D2Q9", n=n, nd=(2, 2), nu=nu, nsteps=nsteps,
                         motion=I.motion_static(nsteps, centre), bcs=bcs,
                         obj=I.objective("NONE", 1, 0), u0=u0, kappa_max=0.0)


def _march(cfg, rho, u, steps):
    nc = rho.size
    kap, uS = np.zeros(nc), np.zeros((3, nc))
    for _ in range(steps):
        rho, u = O.step(cfg, kap, uS, rho, u)
    return rho, u


# ------------------------------------------------------------------------------------------
# pressure-driven channel: exact fixed point, for both pressure-held outflow kinds
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("outlet", ["PRESSURE", "ZERO_GRADIENT"])
def test_pressure_driven_channel_is_exact_fixed_point(outlet):
    nx, ny, nu = 14, 11, 0.08
    H = ny - 1
    r_in, r_out = 1.0024, 0.9991
    bcs = [_bc("PRESSURE", r_in), _bc(outlet, r_out), _bc("NOSLIP"), _bc("NOSLIP"),
           _bc("PERIODIC"), _bc("PERIODIC")]
    cfg = _channel_cfg((nx, ny), nu, bcs)
    x = np.tile(np.arange(nx), ny).astype(float)
    y = np.repeat(np.arange(ny), nx).astype(float)
    rho_ex = r_in + (r_out - r_in) * x / (nx - 1)
    g = (r_in - r_out) / (3.0 * (nx - 1))
    ux_ex = g * y * (H - y) / (2.0 * nu)
    u_ex = np.zeros((3, nx * ny))
    u_ex[0] = ux_ex
    rho, u = _march(cfg, rho_ex.copy(), u_ex.copy(), 200)
    assert np.abs(rho - rho_ex).max() < 1e-14
    assert np.abs(u[0] - ux_ex).max() < 1e-12 * ux_ex.max()
    assert np.abs(u[1]).max() < 1e-12 * ux_ex.max()


def test_pressure_driven_channel_converges_from_rest():
    """From rest the channel reaches the closed form: u_max = g H^2 / (8 nu), rho linear."""
    nx, ny, nu = 12, 9, 0.1
    H = ny - 1
    r_in, r_out = 1.003, 1.0
    bcs = [_bc("PRESSURE", r_in), _bc("ZERO_GRADIENT", r_out), _bc("NOSLIP"), _bc("NOSLIP"),
           _bc("PERIODIC"), _bc("PERIODIC")]
    cfg = _channel_cfg((nx, ny), nu, bcs)
    nc = nx * ny
    rho0, u0 = O.apply_bc(cfg, np.ones(nc), np.zeros((3, nc)))
    rho, u = _march(cfg, rho0, u0, 6000)
    x = np.tile(np.arange(nx), ny).astype(float)
    y = np.repeat(np.arange(ny), nx).astype(float)
    g = (r_in - r_out) / (3.0 * (nx - 1))
    ux_ex = g * y * (H - y) / (2.0 * nu)
    assert abs(u[0].max() - g * H * H / (8.0 * nu)) < 1e-6 * u[0].max()
    assert np.abs(u[0] - ux_ex).max() < 1e-6 * ux_ex.max()
    assert np.abs(rho - (r_in + (r_out - r_in) * x / (nx - 1))).max() < 1e-9


# ------------------------------------------------------------------------------------------
# velocity inlet + zero-gradient outflow (the benchmark channels): a steady state exists
# ------------------------------------------------------------------------------------------
def test_velocity_inlet_channel_reaches_steady_state():
    nx, ny, nu, U = 64, 17, 0.1, 0.02
    H = ny - 1
    cfg = _channel_cfg((nx, ny), nu, I.channel_bcs(2, U), u0=(U, 0, 0))
    nc = nx * ny
    rho, u = O.apply_bc(cfg, np.ones(nc), np.tile(np.array([[U], [0.0], [0.0]]), (1, nc)))
    rho, u = _march(cfg, rho, u, 9000)
    m_a = rho.sum()
    rho, u = _march(cfg, rho, u, 1000)
    m_b = rho.sum()
    rho2, _ = _march(cfg, rho, u, 1)
    # total mass: constant at the steady state (it grows by ~5e-5 per node and step when the
    # outflow copies rho instead of holding rho_bar)
    assert abs(m_b - m_a) < 1e-10 * m_b
    assert abs(rho2.sum() - m_b) < 1e-13 * m_b
    assert abs(rho.mean() - 1.0) < 2e-2
    ux = u[0].reshape(ny, nx)
    R = rho.reshape(ny, nx)
    # the outflow holds rho_bar = 1
    assert np.abs(R[1:-1, -1] - 1.0).max() == 0.0
    # developed region: a parabola through the wall nodes, the same on every column
    yy = np.arange(ny, dtype=float)
    shape = yy * (H - yy)
    for col in (nx // 2, 3 * nx // 4, nx - 2):
        prof = ux[:, col]
        fit = shape * (prof @ shape) / (shape @ shape)
        assert np.abs(prof - fit).max() < 1e-4 * prof.max(), col
    # the volume flux sum_y u_x is the same through every developed cross-section
    flux = ux.sum(axis=0)
    dev = flux[nx // 2:]
    assert np.abs(dev - dev.mean()).max() < 1e-5 * dev.mean()
    # and within 1 % of the inflow sum_y u_x = U (ny - 2) (the rest is the entrance diffusion
    # flux -(1/6) d rho/dx where the plug reshapes)
    assert abs(dev.mean() / (U * (ny - 2)) - 1.0) < 0.02
    # the centreline speed of a developed parabola carrying that flux: sum_y y(H-y) = H(H^2-1)/6
    assert abs(ux[H // 2, nx - 2] - dev.mean() * (H / 2) ** 2 / (H * (H * H - 1) / 6.0)) < 1e-3 * ux.max()


# ------------------------------------------------------------------------------------------
# objective densities on constructed fields
# ------------------------------------------------------------------------------------------
def _obj_cfg(kind, n=(9, 7), direction=(0.6, 0.8, 0.0), centre=(2.5, 1.5, 0.0), mask=None,
             norm=0, nsteps=1, n0=1, n1=1):
    c = ((n[0] - 1) / 2.0, (n[1] - 1) / 2.0, 0.0)
    return I.make_config(dim=2, lattice="D2Q9", n=n, nd=(2, 2), nu=0.1, nsteps=nsteps,
                         motion=I.motion_static(nsteps, c), bcs=I.periodic_bcs(),
                         obj=I.objective(kind, n0, n1, norm=norm, centre=centre,
                                         direction=direction, mask=mask))


def _rect_mask(n, x0, x1, y0, y1):
    m = np.zeros((n[1], n[0]), dtype=np.uint8)
    m[y0:y1 + 1, x0:x1 + 1] = 1
    return m.reshape(-1)


def test_objective_densities_on_uniform_fields():
    """Uniform kappa, u and u_S on a rectangle of M nodes: the body force is F = k (u - u_S)
    everywhere, so DRAG = M F.n, POWER = M F.u_S, and the torque about c is M (rbar - c) x F
    with rbar the rectangle's centroid."""
    n = (9, 7)
    nc = n[0] * n[1]
    x0, x1, y0, y1 = 2, 6, 1, 4
    mask = _rect_mask(n, x0, x1, y0, y1)
    M = (x1 - x0 + 1) * (y1 - y0 + 1)
    k, uv, us = 0.37, np.array([0.05, -0.02]), np.array([-0.01, 0.03])
    kap = np.full(nc, k)
    u = np.zeros((3, nc)); u[0], u[1] = uv
    uS = np.zeros((3, nc)); uS[0], uS[1] = us
    rho = np.full(nc, 1.013)
    F = k * (uv - us)                                   # (0.0222, -0.0185)
    nvec = np.array([0.6, 0.8])
    centre = np.array([2.5, 1.5])
    rbar = np.array([(x0 + x1) / 2.0, (y0 + y1) / 2.0])  # (4, 2.5)
    lever = rbar - centre                                # (1.5, 1.0)
    expect = {
        "DRAG": M * (F @ nvec),
        "POWER": M * (F @ us),
        "TORQUE": M * (lever[0] * F[1] - lever[1] * F[0]),
        "J1": -M * 1.013 / 3.0,
        "J2": -M * (nvec @ uv),
        "MASS": M * 1.013,
    }
    for kind, val in expect.items():
        cfg = _obj_cfg(kind, n=n, mask=mask, direction=(0.6, 0.8, 0.0) if kind != "TORQUE" else (0, 0, 1))
        got = O.objective_step(cfg, kap, uS, rho, u)
        assert abs(got - val) < 1e-14 * max(1.0, abs(val)), (kind, got, val)
    # the sign of the torque: a force along +x applied above the centre turns clockwise (-z)
    cfg = _obj_cfg("TORQUE", n=n, mask=_rect_mask(n, 3, 3, 5, 5), direction=(0, 0, 1), centre=(3, 2, 0))
    u1 = np.zeros((3, nc)); u1[0] = 0.1
    assert O.objective_step(cfg, np.ones(nc), np.zeros((3, nc)), rho, u1) == pytest.approx(-0.3, abs=1e-15)


def test_objective_partials_match_closed_form_derivatives():
    """On the same uniform fields, d/du of DRAG is k n, of POWER k u_S, of TORQUE k (e_z x r),
    d/dkappa of DRAG (u - u_S).n; J1 seeds rho with -1/3 and J2 seeds u with -n."""
    n = (6, 5)
    nc = n[0] * n[1]
    k, uv, us = 0.5, np.array([0.04, 0.01]), np.array([0.02, -0.03])
    kap = np.full(nc, k)
    u = np.zeros((3, nc)); u[0], u[1] = uv
    uS = np.zeros((3, nc)); uS[0], uS[1] = us
    rho = np.ones(nc)
    x = np.tile(np.arange(n[0]), n[1]).astype(float)
    y = np.repeat(np.arange(n[1]), n[0]).astype(float)
    cfg = _obj_cfg("DRAG", n=n, direction=(1.0, 0.0, 0.0))
    dP, dV, dK = O.objective_partials(cfg, kap, uS, rho, u)
    assert np.all(dP == 0) and np.allclose(dV[0], k) and np.allclose(dV[1], 0.0)
    assert np.allclose(dK, uv[0] - us[0])
    cfg = _obj_cfg("POWER", n=n)
    dP, dV, dK = O.objective_partials(cfg, kap, uS, rho, u)
    assert np.allclose(dV[0], k * us[0]) and np.allclose(dV[1], k * us[1])
    assert np.allclose(dK, (uv - us) @ us)
    cfg = _obj_cfg("TORQUE", n=n, direction=(0, 0, 1), centre=(2.0, 1.0, 0.0))
    dP, dV, dK = O.objective_partials(cfg, kap, uS, rho, u)
    # tau = r_x F_y - r_y F_x: d tau/d u_x = -k r_y, d tau/d u_y = k r_x
    assert np.allclose(dV[0], -k * (y - 1.0)) and np.allclose(dV[1], k * (x - 2.0))
    assert np.allclose(dK, (x - 2.0) * (uv[1] - us[1]) - (y - 1.0) * (uv[0] - us[0]))
    cfg = _obj_cfg("J1", n=n)
    dP, dV, dK = O.objective_partials(cfg, kap, uS, rho, u)
    assert np.allclose(dP, -1.0 / 3.0) and np.all(dV == 0) and np.all(dK == 0)
    cfg = _obj_cfg("J2", n=n, direction=(0.6, 0.8, 0.0))
    dP, dV, dK = O.objective_partials(cfg, kap, uS, rho, u)
    assert np.allclose(dV[0], -0.6) and np.allclose(dV[1], -0.8) and np.all(dK == 0)


def _translating_body_cfg(kind, norm, mask=None, direction=(0.6, 0.8, 0.0), centre=(0, 0, 0)):
    """Periodic box, uniform flow u0, a design grid translating at uG with its nodes on integer
    analysis nodes: with the hat transfer kappa = kappa_ref and u_S = uG exactly on the image."""
    n, nd, N = (16, 14), (4, 3), 1
    u0, uG = (0.03, -0.01, 0.0), (-0.02, 0.015, 0.0)
    rec = np.zeros((N + 1, 18))
    rec[:, 0:9] = np.eye(3).reshape(-1)
    rec[:, 12:15] = (7.0, 6.0, 0.0)
    rec[:, 15:18] = uG
    cfg = I.make_config(dim=2, lattice="D2Q9", n=n, nd=nd, nu=0.1, nsteps=N, motion=rec,
                        bcs=I.periodic_bcs(), xi_G=(1.0, 1.0, 0.0), u0=u0, rho0=1.02,
                        obj=I.objective(kind, 1, 1, norm=norm, centre=centre,
                                        direction=direction, mask=mask),
                        kappa_max=0.9, q=0.1, interp="FLUID_ONE", weight="LIN")
    return cfg, np.array(u0[:2]), np.array(uG[:2])


def test_solve_objective_translating_body_closed_form():
    """One step from a uniform state: the pull returns (rho0, u0), the Brinkman update gives
    u = (u0 + kappa uG) / (1 + kappa), so F_b = kappa (u0 - uG) / (1 + kappa) at each image
    node x = xi - xi_G + xG."""
    g = np.linspace(0.05, 0.9, 12)
    kref = 0.9 * 0.1 * (1 - g) / (0.1 + g)      # FLUID_ONE, kappa_max 0.9, q 0.1 (Sec. 2.3 form)
    w = kref / (1.0 + kref)
    xs = np.array([i - 1 + 7 for j in range(3) for i in range(4)], dtype=float)
    ys = np.array([j - 1 + 6 for j in range(3) for i in range(4)], dtype=float)
    nvec = np.array([0.6, 0.8])
    for kind in ("DRAG", "POWER", "TORQUE"):
        cfg, u0, uG = _translating_body_cfg(kind, 0, direction=(0.6, 0.8, 0.0) if kind == "DRAG" else (0, 0, 1),
                                            centre=(3.0, 2.0, 0.0))
        F = np.outer(w, u0 - uG)
        if kind == "DRAG":
            expect = (F @ nvec).sum()
        elif kind == "POWER":
            expect = (F @ uG).sum()
        else:
            expect = ((xs - 3.0) * F[:, 1] - (ys - 2.0) * F[:, 0]).sum()
        J = O.solve(cfg, g, grad=False)["J"]
        assert abs(J - expect) < 1e-14 * max(1e-3, abs(expect)), (kind, J, expect)
    # NORM_MASK divides by the mask count: a mask on 5 image nodes plus 7 empty ones
    mask = np.zeros(16 * 14, dtype=np.uint8)
    img = (ys * 16 + xs).astype(int)
    mask[img[:5]] = 1
    mask[[0, 1, 2, 3, 4, 5, 6]] = 1
    cfg, u0, uG = _translating_body_cfg("DRAG", 2, mask=mask)
    expect = (np.outer(w[:5], u0 - uG) @ nvec).sum() / 12.0
    assert abs(O.solve(cfg, g, grad=False)["J"] - expect) < 1e-15


@pytest.mark.parametrize("norm", [0, 1, 2, 3])
def test_solve_objective_window_and_normalisation(norm):
    """Uniform flow without a body stays uniform (no kappa), so over the window n0..n1 of T
    steps and a mask of M nodes: J1 = -T M rho0 / 3 and J2 = -T M n.u0, divided by T for
    NORM_TIME and by M for NORM_MASK."""
    n, N, n0, n1 = (8, 6), 7, 3, 6
    T = n1 - n0 + 1
    mask = _rect_mask(n, 1, 4, 2, 4)
    M = int(mask.sum())
    rho0, u0 = 0.97, (0.02, -0.05, 0.0)
    div = (T if norm & 1 else 1) * (M if norm & 2 else 1)
    for kind, per in (("J1", -rho0 / 3.0), ("J2", -(0.6 * u0[0] + 0.8 * u0[1]))):
        cfg = I.make_config(dim=2, lattice="D2Q9", n=n, nd=(2, 2), nu=0.1, nsteps=N,
                            motion=I.motion_static(N, (3.5, 2.5, 0.0)), bcs=I.periodic_bcs(),
                            obj=I.objective(kind, n0, n1, norm=norm, direction=(0.6, 0.8, 0.0),
                                            mask=mask),
                            u0=u0, rho0=rho0, kappa_max=0.0)
        r = O.solve(cfg, np.full(4, 0.5), grad=False)
        assert abs(r["J"] - T * M * per / div) < 1e-14, (kind, norm)
        # the per-step values: zero outside the window, equal inside it
        assert np.all(r["jn"][:n0] == 0) and np.all(r["jn"][n1 + 1:] == 0)
        assert np.allclose(r["jn"][n0:n1 + 1], M * per / div, rtol=0, atol=1e-14)


def test_j1_j2_on_the_pressure_driven_channel():
    """J1 on a column of the exact pressure-driven channel is -(1/3) of its linear rho; J2 along
    +x on the interior of a column is -(g / 2 nu) mean y (H - y)."""
    nx, ny, nu = 10, 9, 0.1
    H = ny - 1
    r_in, r_out = 1.003, 1.0
    x = np.tile(np.arange(nx), ny).astype(float)
    y = np.repeat(np.arange(ny), nx).astype(float)
    rho = r_in + (r_out - r_in) * x / (nx - 1)
    g = (r_in - r_out) / (3.0 * (nx - 1))
    u = np.zeros((3, nx * ny))
    u[0] = g * y * (H - y) / (2.0 * nu)
    col = 4
    mask = ((x == col) & (y >= 1) & (y <= H - 1)).astype(np.uint8)
    cfgJ1 = _obj_cfg("J1", n=(nx, ny), mask=mask)
    cfgJ2 = _obj_cfg("J2", n=(nx, ny), mask=mask, direction=(1.0, 0.0, 0.0))
    z = np.zeros(nx * ny)
    yy = np.arange(1, H)
    assert abs(O.objective_step(cfgJ1, z, np.zeros((3, nx * ny)), rho, u)
               + (H - 1) * (r_in + (r_out - r_in) * col / (nx - 1)) / 3.0) < 1e-14
    assert abs(O.objective_step(cfgJ2, z, np.zeros((3, nx * ny)), rho, u)
               + g / (2 * nu) * float((yy * (H - yy)).sum())) < 1e-16


# ------------------------------------------------------------------------------------------
# the paper's own adjoint form (Sec. 2.4): checked where it must coincide with the exact step, by
# the closed-form gain of an adjoint shear wave under a uniform kappa, and against central
# differences the way the paper verifies it (Sec. 2.6)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("nu,kap", [(0.05, 0.3), (0.12, 2.0), (0.3, 0.7)])
def test_paper_adjoint_shear_wave_gain_closed_form(axis, nu, kap):
    """Fluid at rest, uniform kappa, periodic box, an adjoint velocity W sin(k y) along x (or the
    same rotated).  Worked out by hand for D2Q9: the pull transpose gives 3 u~ = g1 W with
    g1 = 1 - (1 - cos k)/3 and no rho~; the strain transpose adds g2 W with g2 = (A/9)(1 - cos 2k).
    The exact transpose divides the whole adjoint velocity by (1 + kappa) first, so its gain is
    (g1 + g2)/(1 + kappa).  The paper's form (Eq. au_ex) divides only the carried 3 u~, so with
    W_n = U3_n/(1 + kappa) + (V_n - U3_n) it advances V = (g1 + g2) W, U3 = g1 W, and W gains
    g1/(1 + kappa) + g2 per step; its kappa seed is -(U3/(1 + kappa)).(u - u_S)."""
    L = 16
    n = (L, 5) if axis == 0 else (5, L)  # the wave varies along `axis`, the velocity is across it
    nc = n[0] * n[1]
    cfg = _obj_cfg("NONE", n=n)
    cfg["nu"] = nu
    comp = 1 - axis
    coord = np.array(np.unravel_index(np.arange(nc), n[::-1]))[::-1][axis]
    k = 2 * math.pi * 3 / L
    A = 4.5 * (1.0 / 6.0 - nu)
    g1 = 1 - (1 - math.cos(k)) / 3
    g2 = (A / 9) * (1 - math.cos(2 * k))
    shape = np.sin(k * coord)
    kappa = np.full(nc, kap)
    uS = np.zeros((3, nc)); uS[0], uS[1] = 0.02, -0.015
    zero = np.zeros((3, nc))
    alpha, beta = 1.0, 0.4  # V and U3 amplitudes of the level being left
    V = np.zeros((3, nc)); V[comp] = alpha * shape
    U3 = np.zeros((3, nc)); U3[comp] = beta * shape
    P = np.zeros(nc)
    Pe, Ve, _ = O.step_T(cfg, kappa, uS, zero, zero, P, V)
    assert np.abs(Pe).max() < 1e-15 and np.abs(Ve[axis]).max() < 1e-15
    assert np.abs(Ve[comp] - (g1 + g2) / (1 + kap) * alpha * shape).max() < 1e-14
    W = beta / (1 + kap) + alpha - beta
    for _ in range(4):
        Pp, Vp, U3p, kb = O.step_T_paper(cfg, kappa, uS, zero, zero, P, V, U3)
        expect_kb = (beta / (1 + kap)) * uS[comp, 0] * shape
        assert np.abs(kb - expect_kb).max() < 1e-15
        assert np.abs(Pp).max() < 1e-15 and np.abs(Vp[axis]).max() < 1e-15
        assert np.abs(Vp[comp] - (g1 + g2) * W * shape).max() < 1e-14
        assert np.abs(U3p[comp] - g1 * W * shape).max() < 1e-14
        alpha, beta = (g1 + g2) * W, g1 * W
        W_next = beta / (1 + kap) + alpha - beta
        assert abs(W_next - (g1 / (1 + kap) + g2) * W) < 1e-15
        W, P, V, U3 = W_next, Pp, Vp, U3p


def test_paper_adjoint_step_reduces_to_exact_without_flow_and_viscous_term():
    """With u = 0 before the step and A = 0 (nu = 1/6) the adjoint velocity is the pulled moment
    alone (V = 3 u~), so dividing only 3 u~ by (1 + kappa) and forming the kappa seed from it is
    the exact transpose; on a periodic box (no boundary seeds) the two steps agree to round-off."""
    n = (9, 8)
    nc = n[0] * n[1]
    cfg = _obj_cfg("DRAG", n=n)
    cfg["nu"] = 1.0 / 6.0
    rng = np.random.default_rng(4)
    kap = rng.random(nc) * 0.7
    uS = np.zeros((3, nc)); uS[:2] = rng.normal(size=(2, nc)) * 0.01
    u_cur = np.zeros((3, nc)); u_cur[:2] = rng.normal(size=(2, nc)) * 0.02
    P = rng.normal(size=nc)
    V = np.zeros((3, nc)); V[:2] = rng.normal(size=(2, nc))
    zero = np.zeros((3, nc))
    Pe, Ve, kbe = O.step_T(cfg, kap, uS, zero, u_cur, P, V)
    Pp, Vp, U3p, kbp = O.step_T_paper(cfg, kap, uS, zero, u_cur, P, V, V)
    assert np.abs(Pp - Pe).max() < 1e-14 and np.abs(Vp - Ve).max() < 1e-14
    assert np.abs(kbp - kbe).max() < 1e-14
    # and the new level's 3 u~ is the whole new adjoint velocity
    assert np.abs(U3p[:2] - Vp[:2]).max() < 1e-14
    # with flow the two differ (the paper form is not the transpose of the discrete step)
    u_prev = np.zeros((3, nc)); u_prev[:2] = rng.normal(size=(2, nc)) * 0.05
    _, Ve2, _ = O.step_T(cfg, kap, uS, u_prev, u_cur, P, V)
    _, Vp2, _, _ = O.step_T_paper(cfg, kap, uS, u_prev, u_cur, P, V, V)
    assert np.abs(Vp2 - Ve2).max() < 1e-14  # one step from U3 = V: still the exact division
    _, Vp3, _, kb3 = O.step_T_paper(cfg, kap, uS, u_prev, u_cur, P, V, 0.5 * V)
    assert np.abs(Vp3 - Ve2).max() > 1e-3 and np.abs(kb3 - kbe).max() > 1e-3


def test_paper_adjoint_gradient_approximates_central_differences():
    """A rotating ellipse (gamma 0.9 in 0.1, the paper's interpolation, cosine transfer) in a walled
    box, J1 on a line: the exact reverse sweep matches central differences of J to 1e-5, the
    paper's form to a few per cent (the O(kappa) and O(|u| s~) terms it drops)."""
    n, nd, N = (36, 36), (22, 22), 150
    c = ((n[0] - 1) / 2.0, (n[1] - 1) / 2.0, 0.0)
    mask = np.zeros((n[1], n[0]), np.uint8)
    mask[8:28, 31] = 1
    walls = [_bc("NOSLIP")] * 4 + [_bc("PERIODIC")] * 2
    cfg = I.make_config(dim=2, lattice="D2Q9", n=n, nd=nd, nu=0.1, nsteps=N,
                        motion=I.motion_rotation(N, c, 2 * math.pi / 300), bcs=walls,
                        obj=I.objective("J1", 1, N, norm=3, mask=mask.reshape(-1)),
                        interp="PAPER", kappa_max=1.0, q=0.1, weight="COS4")
    X, Y = np.meshgrid(np.arange(nd[0]), np.arange(nd[1]))
    g = np.where(((X - 10.5) / 9.0) ** 2 + ((Y - 10.5) / 4.0) ** 2 <= 1.0, 0.9, 0.1).reshape(-1)
    ex = O.solve(cfg, g)["grad"]
    pa = O.solve(dict(cfg, adjoint="PAPER"), g)["grad"]
    idx = [10 * nd[0] + i for i in range(1, nd[0], 3)]
    h = 1e-6
    fd = []
    for i in idx:
        gp, gm = g.copy(), g.copy()
        gp[i] += h
        gm[i] -= h
        fd.append((O.solve(cfg, gp, grad=False)["J"] - O.solve(cfg, gm, grad=False)["J"]) / (2 * h))
    fd = np.array(fd)
    e_ex = np.abs(ex[idx] - fd).max() / np.abs(fd).max()
    e_pa = np.abs(pa[idx] - fd).max() / np.abs(fd).max()
    assert e_ex < 1e-5, e_ex
    assert 1e-4 < e_pa < 0.2, e_pa
