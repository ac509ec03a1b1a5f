"""Run one workload through the host-emulated library (liblks_emu.so, AddressSanitizer) and store its
results.  TEST INFRASTRUCTURE ONLY: started as a child process with the ASan runtime preloaded.

    python run_case.py <spec.json> <out.npz>

spec: {"module": "test_gpu_parity_3d", "builder": "box3", "kwargs": {...}, "seed": 7,
       "ckpt": true}  builds the configuration with that test module's own builder.
"""
import importlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TESTS = os.path.dirname(HERE)
ROOT = os.path.dirname(TESTS)
for p in (ROOT, TESTS):
    if p not in sys.path:
        sys.path.insert(0, p)
sys.modules["torch"] = None  # the emulated library needs no HIP runtime

import lks_inputs as I  # noqa: E402
from paper_2506_23895_amd import lks  # noqa: E402


def build_cfg(spec):
    if spec.get("config"):
        return getattr(I, spec["config"])(**spec.get("kwargs", {}))
    mod = importlib.import_module(spec["module"])
    kwargs = dict(spec.get("kwargs", {}))
    if "case" in spec:
        kwargs.update(getattr(mod, spec.get("cases", "CASES"))[spec["case"]])
    return getattr(mod, spec["builder"])(**kwargs)


def main():
    spec = json.load(open(sys.argv[1]))
    out = sys.argv[2]
    lks.LIB_PATH = os.path.join(HERE, "_build", "liblks_emu.so")
    cfg = build_cfg(spec)
    for k, v in spec.get("override", {}).items():
        cfg[k] = v
    g = I.gamma_field(cfg["nd"], cfg["dim"], spec.get("seed", 7))
    g = g.astype(np.float64 if cfg["precision"] == "F64" else np.float32)
    res = {}
    N, K = cfg["nsteps"], cfg["checkpoint_every"]
    with lks.Solver(cfg) as s:
        print(f"[emu] forward {spec}", flush=True)
        res["J"] = np.array(s.forward(g))
        res["jn"] = s.objective_steps()
        r, u = s.read_state(lks.STATE_FINAL)
        res["rho"], res["u"] = r, u
        if spec.get("ckpt") and K > 0:
            for k in range((N + K - 1) // K):
                rk, uk = s.read_state(k)
                res[f"ck{k}_rho"], res[f"ck{k}_u"] = rk, uk
        if cfg["objective"]["kind"] != "NONE":
            print("[emu] adjoint", flush=True)
            s.adjoint()
            res["grad"] = s.sensitivity().astype(np.float64)
    np.savez(out, **res)
    print("[emu] done", flush=True)


if __name__ == "__main__":
    main()
