"""lks_forward_noalloc (the forward sweep with every kernel buffer in the library's static device
scratch) against the allocating entry points lks_create + lks_forward + lks_read_state: two calls
in a row through the C ABI, the second on a smaller workload, each bitwise equal to the
allocating path and within the FP64 parity bound of the oracle; and a workload too large for the
scratch is refused with a message before any device work."""
import math

import numpy as np
import pytest

import lks_inputs as I
from parity_util import announce, rel_l2, run_oracle

pytestmark = pytest.mark.gpu


def _cfg(n, nd, N, prec, K=7):
    c = ((n[0] - 1) / 2.0 + 0.3, (n[1] - 1) / 2.0 - 0.2, 0.0)
    return I.make_config(dim=2, lattice="D2Q9", n=n, nd=nd, nu=0.04, nsteps=N,
                         motion=I.motion_rotation(N, c, 2 * math.pi / 600), bcs=I.channel_bcs(2, 0.03),
                         obj=I.objective("DRAG", 2, N, norm=1, direction=(0.8, 0.6, 0.0)),
                         u0=(0.03, 0, 0), kappa_max=0.5, precision=prec, checkpoint_every=K)


def _cfg3(n, nd, N):
    centre = tuple((v - 1) / 2.0 for v in n)
    bcs = [{"kind": "VELOCITY", "rho": 1.0, "u": (0.03, 0, 0)}, {"kind": "ZERO_GRADIENT", "rho": 1.0, "u": (0, 0, 0)}]
    bcs += [{"kind": "PERIODIC", "rho": 1.0, "u": (0, 0, 0)}] * 4
    return I.make_config(dim=3, lattice="D3Q19", n=n, nd=nd, nu=0.05, nsteps=N,
                         motion=I.motion_rotation(N, centre, 2 * math.pi / 80), bcs=bcs,
                         obj=I.objective("TORQUE", 1, N, centre=centre, direction=(0, 0, 1)),
                         u0=(0.03, 0, 0), kappa_max=0.6, precision="F32", checkpoint_every=9)


def _both(cfg, seed):
    import torch
    from paper_2506_23895_amd import lks
    dt = torch.float64 if cfg["precision"] == "F64" else torch.float32
    nc, D = int(np.prod(cfg["n"])), cfg["dim"]
    g = torch.as_tensor(I.gamma_field(cfg["nd"], D, seed), dtype=dt).cuda()
    drho = torch.full((nc,), float("nan"), dtype=dt, device="cuda")
    u = torch.full((D, nc), float("nan"), dtype=dt, device="cuda")
    J0 = lks.forward_noalloc(cfg, g, drho, u, stream=torch.cuda.current_stream().cuda_stream)
    with lks.Solver(cfg) as s:
        J1 = s.forward(g.cpu().numpy())
        r1, u1 = s.read_state(lks.STATE_FINAL)
    return J0, drho.cpu().numpy(), u.cpu().numpy(), J1, r1, u1, g.cpu().numpy()


def test_noalloc_forward_equals_allocating_path_twice():
    import torch
    torch.cuda.set_device(0)
    cases = [("2d 181x97 fp64", _cfg((181, 97), (30, 28), 150, "F64"), 3),
             ("2d 70x37 fp32 (smaller)", _cfg((70, 37), (14, 12), 60, "F32"), 4)]
    for name, cfg, seed in cases:
        announce(f"no-alloc forward {name}")
        J0, r0, u0, J1, r1, u1, g = _both(cfg, seed)
        assert J0 == J1, (name, J0, J1)
        assert np.array_equal(r0, r1) and np.array_equal(u0, u1), name
        o = run_oracle(cfg, g.astype(np.float64), grad=False)
        tol = 1e-11 if cfg["precision"] == "F64" else 1e-4
        assert rel_l2(r0, o["rho"] - 1.0) <= tol and rel_l2(u0, o["u"][:2]) <= tol, name
        assert abs(J0 - o["J"]) <= tol * abs(o["J"]), name


def test_noalloc_forward_3d_then_2d():
    import torch
    torch.cuda.set_device(0)
    for name, cfg, seed in (("3d 40x36x34 fp32", _cfg3((40, 36, 34), (10, 9, 8), 30), 5),
                            ("2d 48x40 fp64 (smaller)", _cfg((48, 40), (10, 10), 25, "F64"), 6)):
        announce(f"no-alloc forward {name}")
        J0, r0, u0, J1, r1, u1, _ = _both(cfg, seed)
        assert J0 == J1 and np.array_equal(r0, r1) and np.array_equal(u0, u1), name


def test_noalloc_refuses_oversize():
    from paper_2506_23895_amd import lks
    big = I.config_c3(n_side=4096, nd_side=256, nsteps=10)
    with pytest.raises(lks.LksError) as ei:
        lks.forward_noalloc(big, np.zeros(256 * 256, np.float32))
    assert ei.value.code == lks.LKS_EINVAL and "scratch" in str(ei.value)
