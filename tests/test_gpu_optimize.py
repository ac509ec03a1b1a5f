"""The optimisation loop of Sec. 2.7 driving the GPU sensitivity: the 2D rotor of Sec. 3.1 at the
paper's size (a 100 x 100 design grid rotating about (75, 75) with its centre (50, 50) on it, period
3000 steps; J1; V_max = 25 %; Heaviside projection with R = 2.4 and beta doubling from 1).  The
figure-only details are chosen stand-ins: a 150 x 150 box with walls, J1 the mean pressure on the
right wall over one period, nu = 0.05, the paper's interpolation with kappa_max = 1 and q = 0.1, the
cosine transfer, FP32, beta doubled every 20 iterations (the paper: 80) to show the continuation
within a short run.  The paper's shapes and histories are figure-only, so the run is checked only
for what any run must do: J falls, the volume limit holds, every gradient is finite."""
import math
import os

import numpy as np
import pytest

import lks_inputs as I
from parity_util import announce

pytestmark = pytest.mark.gpu


def rotor_config():
    n, nd, N = (150, 150), (100, 100), 3000
    mask = np.zeros((n[1], n[0]), np.uint8)
    mask[1:-1, n[0] - 1] = 1
    walls = [{"kind": "NOSLIP", "rho": 1.0, "u": (0.0, 0.0, 0.0)}] * 4 + \
            [{"kind": "PERIODIC", "rho": 1.0, "u": (0.0, 0.0, 0.0)}] * 2
    return I.make_config(dim=2, lattice="D2Q9", n=n, nd=nd, nu=0.05, nsteps=N,
                         motion=I.motion_rotation(N, (75.0, 75.0, 0.0), 2 * math.pi / 3000), bcs=walls,
                         obj=I.objective("J1", 1, N, norm=3, mask=mask.reshape(-1)),
                         interp="PAPER", kappa_max=1.0, q=0.1, weight="COS4", precision="F32",
                         checkpoint_every=60, name="rotor2d")


def test_rotor2d_optimisation():
    from paper_2506_23895_amd.optimize import gpu_evaluator, optimize
    announce("2d rotor optimisation, 150^2 / 100^2, 3000 steps per evaluation")
    cfg = rotor_config()
    evaluate = gpu_evaluator(cfg)
    grads = []

    def checked(gamma):
        J, g = evaluate(gamma)
        grads.append(bool(np.isfinite(g).all()))
        return J, g

    hist = []
    res = optimize(checked, (100, 100), np.full(100 * 100, 0.25), vmax=0.25, radius=2.4, beta0=1.0,
                   beta_max=8.0, beta_every=20, max_iter=60, callback=hist.append)
    lines = [f"{r.it:4d} {r.J: .9e} {r.G: .3e} {r.beta:5.1f} {r.change:.2e}" for r in res.history]
    summary = ("# 2D rotor (Sec. 3.1 stand-in): 150^2 box with walls, 100^2 design rotating about (75, 75),\n"
               "# period 3000 steps per evaluation, J1 = -mean p on the right wall, V_max 0.25, R 2.4, FP32 GPU\n"
               "# iteration  J  G  beta  |dJ/J|\n" + "\n".join(lines) + "\n"
               + f"final volume fraction {float(np.mean(res.gamma)):.4f}; gray fraction (0.1 < gamma < 0.9) "
               + f"{float(np.mean((res.gamma > 0.1) & (res.gamma < 0.9))):.4f}\n")
    print(summary)
    if os.environ.get("LKS_RECORD_DIR"):
        with open(os.path.join(os.environ["LKS_RECORD_DIR"], "optimization_rotor2d.txt"), "w") as f:
            f.write(summary)
    assert all(grads)
    assert res.history[-1].J < res.history[0].J
    assert res.history[-1].G <= 1e-2
