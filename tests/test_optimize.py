"""The optimisation loop (Sec. 2.7): the method of moving asymptotes against a closed-form optimum,
the filter and projection against their definitions and transposes, the chained design gradient
against central differences, and a short run of the whole loop with the oracle's gradient."""
import math

import numpy as np
import pytest

import lks_inputs as I
from oracle import oracle as O
from paper_2506_23895_amd.optimize import MMA, ConeFilter, optimize, project, project_grad


def setup_module(_m):
    O.build()


def test_mma_reaches_closed_form_optimum():
    """min sum c_j / x_j  s.t.  sum x_j <= V: x_j = V sqrt(c_j) / sum sqrt(c) (Lagrange)."""
    rng = np.random.default_rng(0)
    n, V = 40, 12.0
    c = rng.uniform(0.5, 2.0, n)
    x = np.full(n, 0.5)
    m = MMA(n, xmin=0.01, xmax=1.0)
    for _ in range(80):
        f0, df0 = float(np.sum(c / x)), -c / x ** 2
        f1, df1 = float(np.sum(x) - V), np.ones(n)
        x = m.step(x, f0, df0, f1, df1)
    exact = V * np.sqrt(c) / np.sum(np.sqrt(c))
    assert np.abs(x - exact).max() < 1e-4
    assert np.sum(x) <= V + 1e-6


def test_mma_linear_objective_with_loose_constraint_goes_to_the_bounds():
    """min sum c_j x_j with a constraint that never binds: x_j -> 0 where c_j > 0, 1 where c_j < 0."""
    rng = np.random.default_rng(1)
    n = 25
    c = rng.uniform(-1.0, 1.0, n)
    x = np.full(n, 0.5)
    m = MMA(n)
    for _ in range(60):
        x = m.step(x, float(c @ x), c, float(np.sum(x) - 1e3), np.ones(n))
    assert np.abs(x - (c < 0)).max() < 1e-9


def test_mma_binding_constraint_with_linear_objective():
    """min -sum w_j x_j s.t. sum x_j <= V (a knapsack relaxation): the V largest w_j go to 1."""
    rng = np.random.default_rng(5)
    n, V = 30, 9
    w = rng.permutation(np.linspace(0.1, 1.0, n))
    x = np.full(n, 0.2)
    m = MMA(n)
    for _ in range(150):
        x = m.step(x, float(-w @ x), -w, float(np.sum(x) - V), np.ones(n))
    top = np.argsort(-w)[:V]
    want = np.zeros(n)
    want[top] = 1.0
    assert np.abs(x - want).max() < 1e-3 and np.sum(x) <= V + 1e-6


def test_filter_definition_and_transpose():
    f = ConeFilter((7, 9), 2.4)
    # constant fields are preserved, the weights are the cone max(0, R - |d|) normalised
    assert np.allclose(f.apply(np.ones(63)), 1.0)
    psi = np.zeros((7, 9))
    psi[3, 4] = 1.0
    out = f.apply(psi.reshape(-1)).reshape(7, 9)
    w = lambda d: max(0.0, 2.4 - d)  # noqa: E731
    norm_34 = sum(w(math.hypot(i - 3, j - 4)) for i in range(7) for j in range(9))
    assert out[3, 4] == pytest.approx(2.4 / norm_34, rel=1e-12)
    norm_35 = sum(w(math.hypot(i - 3, j - 5)) for i in range(7) for j in range(9))
    assert out[3, 5] == pytest.approx(1.4 / norm_35, rel=1e-12)
    rng = np.random.default_rng(2)
    a, b = rng.random(63), rng.random(63)
    assert np.dot(f.apply(a), b) == pytest.approx(np.dot(a, f.transpose(b)), rel=1e-12)


def test_projection_values_and_gradient():
    x = np.linspace(0, 1, 11)
    for beta in (1.0, 4.0, 16.0):
        p = project(x, beta)
        assert p[0] == pytest.approx(0.0, abs=1e-15) and p[-1] == pytest.approx(1.0, abs=1e-15)
        assert project(np.array([0.5]), beta)[0] == pytest.approx(0.5)
        h = 1e-6
        fd = (project(x + h, beta) - project(x - h, beta)) / (2 * h)
        assert np.abs(fd - project_grad(x, beta)).max() < 1e-6 * max(1.0, beta)


def _tiny_cfg(N=25):
    n, nd = (16, 14), (6, 6)
    centre = ((n[0] - 1) / 2.0, (n[1] - 1) / 2.0, 0.0)
    return I.make_config(dim=2, lattice="D2Q9", n=n, nd=nd, nu=0.05, nsteps=N,
                         motion=I.motion_rotation(N, centre, 2 * math.pi / 80), bcs=I.channel_bcs(2, 0.03),
                         obj=I.objective("DRAG", 3, N, norm=1), u0=(0.03, 0, 0), kappa_max=0.8)


def test_chained_design_gradient_matches_central_differences():
    """d/dpsi of J(H_beta(F psi)) through the oracle's exact gradient and the chain rule."""
    cfg = _tiny_cfg()
    f = ConeFilter((6, 6), 2.4)
    beta = 4.0
    psi = np.random.default_rng(3).random(36)

    def J_of(p):
        return O.solve(cfg, project(f.apply(p), beta), grad=False)["J"]

    gt = f.apply(psi)
    g = O.solve(cfg, project(gt, beta))["grad"]
    chained = f.transpose(g * project_grad(gt, beta))
    h = 1e-6
    for i in (0, 7, 14, 21, 35):
        pp, pm = psi.copy(), psi.copy()
        pp[i] += h
        pm[i] -= h
        fd = (J_of(pp) - J_of(pm)) / (2 * h)
        assert abs(fd - chained[i]) <= 1e-6 * np.abs(chained).max(), (i, fd, chained[i])


def test_loop_reduces_objective_and_meets_the_volume_limit():
    cfg = _tiny_cfg()

    def evaluate(gamma):
        r = O.solve(cfg, gamma)
        return r["J"], r["grad"]

    hist = []
    res = optimize(evaluate, (6, 6), np.full(36, 0.5), vmax=0.4, max_iter=40, beta_every=15,
                   beta_max=4.0, callback=hist.append)
    J0 = hist[0].J
    assert res.history[-1].J < J0
    assert res.history[-1].G <= 1e-3
    assert [r.beta for r in res.history][-1] > 1.0  # the continuation ran
