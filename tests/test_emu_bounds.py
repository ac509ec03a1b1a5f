"""The library's own kernels and host runtime, built for the CPU against a host stand-in for the HIP
runtime (tests/emu) and run under AddressSanitizer: every global-memory and LDS access of every
launch is checked against the exact extent of its allocation (guard regions around each device
buffer and around each launch's dynamic LDS), a block barrier or wave exchange that not every
thread reaches is reported, and the results are compared with the FP64 oracle.

This is how a kernel's indexing is cleared on the host before it runs on a GPU.  The default set
is sized for the CPU suite; LKS_EMU_FULL=1 runs every GPU parity configuration at full length.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import lks_inputs as I
from parity_util import rel_l2, rel_max, run_oracle

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")

CASES = {
    # the 3D walls-on-every-face configuration with heave (z faces ZERO_GRADIENT / NOSLIP,
    # PRESSURE outlet with a tangential z value): general z layout of every 3D kernel
    "d3q19_walls_everywhere_power": {"module": "test_gpu_parity_3d", "builder": "box3",
                                     "case": "d3q19_walls_everywhere_power", "kwargs": {"N": 6, "K": 4},
                                     "seed": 7, "ckpt": True},
    # periodic z (the three-plane ring variants), D3Q15, FP32
    "d3q15_channel_fp32": {"module": "test_gpu_parity_3d", "builder": "box3",
                           "kwargs": {"N": 5, "K": 3, "lattice": "D3Q15", "prec": "F32"}, "seed": 8},
    # 2D: wave strips with x faces, footprint marches, fused gather
    "d2q9_small": {"module": "test_gpu_parity_2d", "builder": "small", "kwargs": {"N": 10, "K": 4},
                   "seed": 3, "ckpt": True},
    # the paper's adjoint form (its three plain launches), pressure outlet
    "d2q9_paper_adjoint": {"module": "test_gpu_parity_2d", "builder": "small", "case": "pressure_outlet",
                           "kwargs": {"N": 12, "K": 5}, "seed": 3, "override": {"adjoint": "PAPER"}},
}

FULL = os.environ.get("LKS_EMU_FULL") == "1"


def _full_cases():
    sys.path.insert(0, HERE)
    import test_gpu_parity_2d as P2
    import test_gpu_parity_3d as P3
    out = {}
    for name in P3.CASES:
        out[f"3d_{name}"] = {"module": "test_gpu_parity_3d", "builder": "box3", "case": name, "seed": 7,
                             "ckpt": True}
    for name in P2.CASES:
        out[f"2d_{name}"] = {"module": "test_gpu_parity_2d", "builder": "small", "case": name, "seed": 6}
    return out


ALL = _full_cases() if FULL else CASES


@pytest.fixture(scope="module")
def emu_lib():
    sys.path.insert(0, EMU)
    import build_emu
    build_emu.build()
    return build_emu


@pytest.mark.parametrize("name", sorted(ALL))
def test_emulated_kernels_in_bounds_and_match_oracle(emu_lib, name, tmp_path):
    spec = ALL[name]
    sp = tmp_path / "spec.json"
    out = tmp_path / "out.npz"
    sp.write_text(json.dumps(spec))
    p = subprocess.run([sys.executable, os.path.join(EMU, "run_case.py"), str(sp), str(out)],
                       env=emu_lib.asan_env(), capture_output=True, text=True, timeout=1800)
    assert p.returncode == 0, p.stdout[-3000:] + p.stderr[-6000:]
    assert "AddressSanitizer" not in p.stderr, p.stderr[-6000:]
    r = np.load(out)
    sys.path.insert(0, os.path.join(EMU))
    from run_case import build_cfg
    cfg = build_cfg(spec)
    cfg.update(spec.get("override", {}))
    g = I.gamma_field(cfg["nd"], cfg["dim"], spec["seed"])
    want_grad = cfg["objective"]["kind"] != "NONE"
    o = run_oracle(cfg, g, grad=want_grad, traj=bool(spec.get("ckpt")))
    D = cfg["dim"]
    tol = 1e-11 if cfg["precision"] == "F64" else 1e-4
    assert rel_l2(r["rho"], o["rho"] - 1.0) <= tol and rel_max(r["rho"], o["rho"] - 1.0) <= 10 * tol
    assert rel_l2(r["u"], o["u"][:D]) <= tol and rel_max(r["u"], o["u"][:D]) <= 10 * tol
    if want_grad:
        gt = 1e-10 if cfg["precision"] == "F64" else 1e-3
        assert abs(float(r["J"]) - o["J"]) <= tol * abs(o["J"])
        assert rel_l2(r["grad"], o["grad"]) <= gt
    K = cfg["checkpoint_every"]
    if spec.get("ckpt") and K > 0:
        for k in range((cfg["nsteps"] + K - 1) // K):
            assert rel_l2(r[f"ck{k}_u"], o["u_traj"][k * K][:D]) <= max(tol, 1e-15)
