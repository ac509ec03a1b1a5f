"""The optimisation loop around the sensitivity (Sec. 2.7, Steps 1-7; Sec. 3.1-3.3 settings).

Design variable psi in [0, 1] on the design grid.  Each iteration:
  1. physical density gamma = H_beta(F psi): a linear cone filter of radius R (density filter),
     then the smoothed Heaviside projection of Wang, Lazarov and Sigmund (2011) with threshold eta;
  2-5. J(gamma) and dJ/dgamma from the LKS forward / reverse sweeps (on the GPU through the C ABI,
     or any callable with the same signature), the volume constraint
     G = sum(gamma) / (V_max |D|) - 1 <= 0 (the paper's constraint equation) and dG/dgamma;
     both chained back to psi through the projection and the filter;
  6. psi updated by the method of moving asymptotes (Svanberg 1987): separable convex
     approximations with moving asymptotes L < psi < U, the subproblem solved through its
     one-dimensional dual (one constraint);
  7. stop when |J^k - J^(k-1)| / |J^(k-1)| <= 1e-6 with G <= 0, or after max_iter.
Continuation: beta doubles every `beta_every` iterations or when the criterion of step 7 is met
below beta_max (Sec. 3.1); V_max may start higher and drop to its target at a given iteration
(Sec. 3.3).  The forward state can be warm-started from the previous iteration's final state
(Sec. 3.2, for flows that are periodic in time); the reverse sweep always starts from zero, so
every gradient is the exact one of the objective it belongs to.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np


# ---------------------------------------------------------------------------------------------
# filter and projection
# ---------------------------------------------------------------------------------------------
class ConeFilter:
    """gamma~_i = sum_j w_ij psi_j / sum_j w_ij with w_ij = max(0, R - |x_i - x_j|) on the design
    grid (unit spacing, no wrap), applied as a convolution; the transpose for the chain rule."""

    def __init__(self, shape: Sequence[int], radius: float):
        self.shape = tuple(int(v) for v in shape)
        self.radius = float(radius)
        r = int(math.ceil(radius)) - (1 if float(math.ceil(radius)) == radius else 0)
        axes = [np.arange(-r, r + 1)] * len(self.shape)
        grids = np.meshgrid(*axes, indexing="ij")
        dist = np.sqrt(sum(g.astype(float) ** 2 for g in grids))
        self.kernel = np.maximum(0.0, self.radius - dist)
        self.norm = self._conv(np.ones(self.shape))

    def _conv(self, a: np.ndarray) -> np.ndarray:
        from scipy.ndimage import convolve
        return convolve(a, self.kernel, mode="constant", cval=0.0)

    def apply(self, psi: np.ndarray) -> np.ndarray:
        return (self._conv(psi.reshape(self.shape)) / self.norm).reshape(-1)

    def transpose(self, g: np.ndarray) -> np.ndarray:
        # the kernel is symmetric, so W^T v = conv(v / norm)
        return self._conv(g.reshape(self.shape) / self.norm).reshape(-1)


def project(x: np.ndarray, beta: float, eta: float = 0.5) -> np.ndarray:
    """Smoothed Heaviside: (tanh(beta eta) + tanh(beta (x - eta))) / (tanh(beta eta) + tanh(beta (1 - eta)))."""
    d = math.tanh(beta * eta) + math.tanh(beta * (1.0 - eta))
    return (math.tanh(beta * eta) + np.tanh(beta * (x - eta))) / d


def project_grad(x: np.ndarray, beta: float, eta: float = 0.5) -> np.ndarray:
    d = math.tanh(beta * eta) + math.tanh(beta * (1.0 - eta))
    return beta * (1.0 - np.tanh(beta * (x - eta)) ** 2) / d


# ---------------------------------------------------------------------------------------------
# method of moving asymptotes (one inequality constraint)
# ---------------------------------------------------------------------------------------------
class MMA:
    """Svanberg's method of moving asymptotes for min f0(x) s.t. f1(x) <= 0, xmin <= x <= xmax.

    At x^k each function is replaced by the convex separable approximation
        f~_i(x) = r_i + sum_j p_ij / (U_j - x_j) + q_ij / (x_j - L_j),
    with p_ij = (U_j - x_j)^2 ((1 + rho) d+ + rho d- + e), q_ij = (x_j - L_j)^2 (rho d+ + (1 + rho) d- + e),
    d+/- the positive / negative part of df_i/dx_j: the 1987 choice (p from the positive part, q from
    the negative part) plus a small curvature in both directions (rho = 1e-3 of |df|, e = 1e-5 per
    unit range), as in Svanberg's later formulation, which keeps the approximation strictly convex
    and stops it from jumping to a bound where the gradient is small; r_i makes f~_i(x^k) = f_i(x^k).
    The asymptotes start at x -/+ s0 (xmax - xmin) and then widen (x 1.2) where the last two steps
    moved the same way, narrow (x 0.7) where they oscillated.  The subproblem min f~_0 subject to
    f~_1 <= 0 within the move limits is solved through its dual: for a multiplier lam >= 0 each
    x_j minimises (p_0j + lam p_1j)/(U_j - x_j) + (q_0j + lam q_1j)/(x_j - L_j) in closed form,
    and lam is the root of the dual derivative f~_1(x(lam)) (bisection; lam = 0 if f~_1 <= 0 there).
    """

    def __init__(self, n: int, xmin: float = 0.0, xmax: float = 1.0, s0: float = 0.5,
                 s_grow: float = 1.2, s_shrink: float = 0.7, move: float = 0.2, eps: float = 1e-5,
                 rho: float = 1e-3):
        self.n = n
        self.xmin = np.full(n, float(xmin))
        self.xmax = np.full(n, float(xmax))
        self.s0, self.s_grow, self.s_shrink, self.move = s0, s_grow, s_shrink, move
        self.eps, self.rho = eps, rho
        self.hist: List[np.ndarray] = []
        self.L = self.U = None

    def _asymptotes(self, x: np.ndarray):
        span = self.xmax - self.xmin
        if len(self.hist) < 2:
            self.L = x - self.s0 * span
            self.U = x + self.s0 * span
        else:
            x1, x2 = self.hist[-1], self.hist[-2]
            sgn = (x - x1) * (x1 - x2)
            fac = np.where(sgn > 0, self.s_grow, np.where(sgn < 0, self.s_shrink, 1.0))
            self.L = x - fac * (x1 - self.L)
            self.U = x + fac * (self.U - x1)
            self.L = np.clip(self.L, x - 10.0 * span, x - 0.01 * span)
            self.U = np.clip(self.U, x + 0.01 * span, x + 10.0 * span)

    def step(self, x: np.ndarray, f0: float, df0: np.ndarray, f1: float, df1: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        self._asymptotes(x)
        L, U = self.L, self.U
        span = self.xmax - self.xmin
        lo = np.maximum.reduce([self.xmin, L + 0.1 * (x - L), x - self.move * span])
        hi = np.minimum.reduce([self.xmax, U - 0.1 * (U - x), x + self.move * span])
        ux, xl = U - x, x - L
        e = self.eps / span

        def pq(df):
            pos, neg = np.maximum(df, 0.0), np.maximum(-df, 0.0)
            return (ux ** 2 * ((1.0 + self.rho) * pos + self.rho * neg + e),
                    xl ** 2 * (self.rho * pos + (1.0 + self.rho) * neg + e))

        p0, q0 = pq(df0)
        p1, q1 = pq(df1)
        r1 = f1 - np.sum(p1 / ux + q1 / xl)

        def x_of(lam: float) -> np.ndarray:
            P = p0 + lam * p1
            Q = q0 + lam * q1
            sp, sq = np.sqrt(P), np.sqrt(Q)
            return np.clip((sp * L + sq * U) / (sp + sq), lo, hi)

        def g1(lam: float) -> float:  # the approximated constraint at x(lam)
            xx = x_of(lam)
            return r1 + float(np.sum(p1 / (U - xx) + q1 / (xx - L)))

        if g1(0.0) <= 0.0:
            lam = 0.0
        else:
            a, b = 0.0, 1.0
            while g1(b) > 0.0 and b < 1e30:
                a, b = b, 2.0 * b
            for _ in range(200):  # g1 decreases in lam (the dual is concave)
                m = 0.5 * (a + b)
                if g1(m) > 0.0:
                    a = m
                else:
                    b = m
                if b - a <= 1e-14 * max(1.0, b):
                    break
            lam = b
        xn = x_of(lam)
        self.hist.append(x.copy())
        if len(self.hist) > 2:
            self.hist.pop(0)
        return xn


# ---------------------------------------------------------------------------------------------
# the loop
# ---------------------------------------------------------------------------------------------
Evaluate = Callable[[np.ndarray], Tuple[float, np.ndarray]]


@dataclass
class Record:
    it: int
    J: float
    G: float
    beta: float
    vmax: float
    change: float


@dataclass
class Result:
    psi: np.ndarray
    gamma: np.ndarray
    history: List[Record] = field(default_factory=list)
    converged: bool = False


def optimize(evaluate: Evaluate, nd: Sequence[int], psi0: np.ndarray, *, vmax: float,
             radius: float = 2.4, beta0: float = 1.0, beta_max: float = 16.0, beta_every: int = 80,
             eta: float = 0.5, tol: float = 1e-6, max_iter: int = 200, vmax_start: Optional[float] = None,
             vmax_switch: int = 0, move: float = 0.2, callback=None) -> Result:
    """Steps 1-7 of Sec. 2.7.  evaluate(gamma) -> (J, dJ/dgamma) on the design grid (minimised).
    vmax_start / vmax_switch: run with V_max = vmax_start until iteration vmax_switch (Sec. 3.3)."""
    n = int(np.prod(nd))
    filt = ConeFilter([int(v) for v in nd][::-1], radius)  # arrays are (.., y, x), x fastest
    psi = np.clip(np.asarray(psi0, dtype=np.float64).reshape(-1), 0.0, 1.0)
    mma = MMA(n, move=move)
    beta = beta0
    res = Result(psi=psi, gamma=np.empty(0))
    J_prev = None
    since_beta = 0
    for it in range(1, max_iter + 1):
        vm = vmax_start if (vmax_start is not None and it <= vmax_switch) else vmax
        gt = filt.apply(psi)
        gamma = project(gt, beta, eta)
        J, dJ = evaluate(gamma)
        G = float(np.sum(gamma) / (vm * n) - 1.0)
        dG = np.full(n, 1.0 / (vm * n))
        dgt = project_grad(gt, beta, eta)
        dJ_psi = filt.transpose(dJ * dgt)
        dG_psi = filt.transpose(dG * dgt)
        change = abs(J - J_prev) / abs(J_prev) if J_prev not in (None, 0.0) else float("inf")
        res.history.append(Record(it, float(J), G, beta, vm, change))
        if callback:
            callback(res.history[-1])
        since_beta += 1
        converged = change <= tol and G <= 1e-9
        if converged and beta >= beta_max:
            res.converged = True
            res.gamma = gamma
            res.psi = psi
            return res
        if (converged or since_beta >= beta_every) and beta < beta_max:
            beta = min(2.0 * beta, beta_max)
            since_beta = 0
            J_prev = None  # the objective jumps with beta: restart the criterion
        else:
            J_prev = J
        psi = mma.step(psi, J, dJ_psi, G, dG_psi)
    res.psi = psi
    res.gamma = project(filt.apply(psi), beta, eta)
    return res


def gpu_evaluator(cfg: dict, warm_start: bool = False) -> Evaluate:
    """evaluate(gamma) through the C ABI on the current GPU: forward, reverse sweep, dJ/dgamma.
    warm_start: each forward starts from the previous one's final state (a new context each
    call; periodic flows, Sec. 3.2)."""
    from . import lks
    state = {"init": None}
    solver = None if warm_start else lks.Solver(cfg)

    def evaluate(gamma: np.ndarray):
        nonlocal solver
        g = np.asarray(gamma, dtype=np.float64 if cfg["precision"] == "F64" else np.float32)
        if warm_start:
            c = dict(cfg)
            if state["init"] is not None:
                r, u = state["init"]
                c["rho_init"] = 1.0 + r.astype(np.float64)
                u3 = np.zeros((3, r.size))
                u3[:cfg["dim"]] = u
                c["u_init"] = u3
            with lks.Solver(c) as s:
                J = s.forward(g)
                state["init"] = s.read_state(lks.STATE_FINAL)
                s.adjoint()
                grad = s.sensitivity()
        else:
            J = solver.forward(g)
            solver.adjoint()
            grad = solver.sensitivity()
        return J, np.asarray(grad, dtype=np.float64)

    return evaluate
