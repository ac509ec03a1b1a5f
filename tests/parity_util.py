"""Helpers for the GPU parity tests: run the HIP path through the C ABI and the oracle on the same
seeded inputs and compare.  (Not collected by pytest: no test_ prefix.)"""
from __future__ import annotations

import sys

import numpy as np

import lks_inputs as I
from oracle import oracle as O


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_max(a, b) -> float:
    """max |a - b| / max |b|: catches an error confined to a few nodes (a face, the edge of the
    footprint) that the L2 norm of a large grid would dilute."""
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    mb = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0)) if a.size else 0.0


# the per-node bound is this multiple of the L2 tolerance, relative to the field's largest value
MAX_FACTOR = 10.0


def announce(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def run_gpu(cfg: dict, gamma: np.ndarray, states=(), grad: bool = True) -> dict:
    from paper_2506_23895_amd import lks
    out = {}
    with lks.Solver(cfg) as s:
        out["J"] = s.forward(gamma)
        out["jn"] = s.objective_steps()
        out["final"] = s.read_state(lks.STATE_FINAL)
        out["ckpt"] = {k: s.read_state(k) for k in states}
        if grad:
            s.adjoint()
            out["grad"] = s.sensitivity().astype(np.float64)
            out["final_after_adj"] = s.read_state(lks.STATE_FINAL)
    return out


def run_oracle(cfg: dict, gamma: np.ndarray, grad: bool = True, traj: bool = False) -> dict:
    c64 = dict(cfg)
    c64["precision"] = "F64"
    return O.solve(c64, np.asarray(gamma, dtype=np.float64), grad=grad, traj=traj)


def compare(cfg: dict, gamma: np.ndarray, tol_field: float, tol_grad: float, tol_J: float,
            check_ckpt: bool = False) -> dict:
    """GPU vs oracle: final rho-1 and u, per-step j, J, dJ/dgamma, and optionally checkpoints."""
    N, K = cfg["nsteps"], cfg["checkpoint_every"]
    want_grad = cfg["objective"]["kind"] != "NONE"
    ks = []
    if check_ckpt and K > 0:
        ks = list(range(0, (N + K - 1) // K))
    g = run_gpu(cfg, gamma.astype(np.float64 if cfg["precision"] == "F64" else np.float32),
                states=ks, grad=want_grad)
    o = run_oracle(cfg, gamma, grad=want_grad, traj=bool(ks))
    dim = cfg["dim"]
    res = {}
    res["rho"] = rel_l2(g["final"][0], o["rho"] - 1.0)
    res["u"] = rel_l2(g["final"][1], o["u"][:dim])
    res["rho_max"] = rel_max(g["final"][0], o["rho"] - 1.0)
    res["u_max"] = rel_max(g["final"][1], o["u"][:dim])
    assert res["rho"] <= tol_field, res
    assert res["u"] <= tol_field, res
    assert res["rho_max"] <= MAX_FACTOR * tol_field, res
    assert res["u_max"] <= MAX_FACTOR * tol_field, res
    if want_grad:
        res["J"] = abs(g["J"] - o["J"]) / max(abs(o["J"]), 1e-300)
        res["jn"] = rel_l2(g["jn"], o["jn"])
        res["grad"] = rel_l2(g["grad"], o["grad"])
        res["grad_max"] = rel_max(g["grad"], o["grad"])
        assert res["J"] <= tol_J, res
        assert res["jn"] <= tol_J, res
        assert res["grad"] <= tol_grad, res
        assert res["grad_max"] <= MAX_FACTOR * tol_grad, res
        # the reverse sweep must not disturb the stored final state
        assert np.array_equal(g["final"][1], g["final_after_adj"][1])
    for k in ks:
        step = k * K
        r = rel_l2(g["ckpt"][k][0], o["rho_traj"][step] - 1.0)
        u = rel_l2(g["ckpt"][k][1], o["u_traj"][step][:dim])
        rm = rel_max(g["ckpt"][k][0], o["rho_traj"][step] - 1.0)
        um = rel_max(g["ckpt"][k][1], o["u_traj"][step][:dim])
        # the initial state is exact; later ones within the field tolerance
        assert r <= max(tol_field, 1e-15) and u <= max(tol_field, 1e-15), (k, r, u)
        assert rm <= MAX_FACTOR * max(tol_field, 1e-15) and um <= MAX_FACTOR * max(tol_field, 1e-15), (k, rm, um)
    return res
