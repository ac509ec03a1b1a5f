"""The autograd wrapper: gradient equals the oracle's on a small copy, matches FP64 central
differences of J on the full 1024x1024 workload, and survives an interleaved forward."""
import math

import numpy as np
import pytest

import lks_inputs as I
from oracle import oracle as O
from parity_util import announce, rel_l2

pytestmark = pytest.mark.gpu


def test_autograd_matches_oracle_copy96():
    import torch
    from paper_2506_23895_amd.autograd import Evaluator
    cfg = I.config_c3(n_side=96, nd_side=24, precision="F32", nsteps=2000)
    announce("autograd vs oracle, 96^2 copy")
    g0 = I.gamma_field(cfg["nd"], 2, 2)
    ev = Evaluator(cfg)
    gamma = torch.tensor(g0, dtype=torch.float32, device="cuda", requires_grad=True)
    J = ev(gamma)
    (2.0 * J).backward()
    ref = O.solve(dict(cfg, precision="F64"), g0)
    assert abs(J.item() - ref["J"]) <= 1e-4 * abs(ref["J"])
    assert rel_l2(gamma.grad.cpu().numpy(), 2.0 * ref["grad"]) <= 1e-3
    ev.close()


def test_backward_after_interleaved_forward():
    import torch
    from paper_2506_23895_amd.autograd import Evaluator
    cfg = I.config_c3(n_side=96, nd_side=24, precision="F32", nsteps=300, checkpoint_every=40)
    announce("autograd interleaved")
    ev = Evaluator(cfg)
    g1 = torch.tensor(I.gamma_field(cfg["nd"], 2, 1), dtype=torch.float32, device="cuda", requires_grad=True)
    g2 = torch.tensor(I.gamma_field(cfg["nd"], 2, 9), dtype=torch.float32, device="cuda", requires_grad=True)
    J1 = ev(g1)
    J2 = ev(g2)   # overwrites the context's trajectory
    J1.backward()
    J2.backward()
    ref1 = O.solve(dict(cfg, precision="F64"), g1.detach().cpu().numpy().astype(np.float64))
    ref2 = O.solve(dict(cfg, precision="F64"), g2.detach().cpu().numpy().astype(np.float64))
    assert rel_l2(g1.grad.cpu().numpy(), ref1["grad"]) <= 1e-3
    assert rel_l2(g2.grad.cpu().numpy(), ref2["grad"]) <= 1e-3
    ev.close()


def test_full_size_gradient_vs_fp64_central_differences():
    """1024x1024 grid, 256x256 design, 10000 steps, checkpoint every 100, time-averaged drag
    (the motion period is the finite-run one the benchmark uses).  The FP32 autograd gradient is
    compared with FP64 central differences (h = 1e-6) of J on 32 seeded design cells chosen among
    those with |g| >= 0.1 max|g|.  FD round-off at this horizon is ~1e-4..1e-3 relative, so the
    bound is 1e-2 per cell; every cell's error is printed and, when LKS_RECORD_DIR is set, written
    to fd_check_c3.txt there."""
    import os
    import torch
    from paper_2506_23895_amd import lks
    from paper_2506_23895_amd.autograd import Evaluator
    cfg = I.config_c3(precision="F32", period=5000.0)
    announce("full-size FD check")
    g0 = I.gamma_field(cfg["nd"], 2, 2)
    ev = Evaluator(cfg)
    gamma = torch.tensor(g0, dtype=torch.float32, device="cuda", requires_grad=True)
    ev(gamma).backward()
    grad = gamma.grad.cpu().numpy().astype(np.float64)
    ev.close()
    rng = np.random.default_rng(19)
    cand = np.flatnonzero(np.abs(grad) >= 0.1 * np.abs(grad).max())
    cells = rng.choice(cand, size=min(32, cand.size), replace=False)
    c64 = dict(cfg, precision="F64", objective=dict(cfg["objective"]))
    h = 1e-6
    errs, rows = [], []
    with lks.Solver(c64) as s:
        for i in cells:
            gp = g0.copy()
            gm = g0.copy()
            gp[i] += h
            gm[i] -= h
            fd = (s.forward(gp) - s.forward(gm)) / (2 * h)
            errs.append(abs(grad[i] - fd) / abs(fd))
            rows.append(f"{int(i) % 256:5d} {int(i) // 256:5d} {grad[i]: .9e} {fd: .9e} {errs[-1]:.3e}")
    summary = ("# C3 full size (1024^2 grid, 256^2 design, 10000 steps, K = 100, period 5000): FP32 "
               "autograd gradient vs FP64 central differences of J (h = 1e-6) on 32 seeded cells\n"
               "#   i     j   dJ/dgamma (FP32 path)  central difference (FP64)  relative error\n"
               + "\n".join(rows) + "\n" +
               f"max {max(errs):.3e}  median {float(np.median(errs)):.3e}\n")
    print(summary)
    if os.environ.get("LKS_RECORD_DIR"):
        with open(os.path.join(os.environ["LKS_RECORD_DIR"], "fd_check_c3.txt"), "w") as f:
            f.write(summary)
    assert max(errs) < 1e-2
