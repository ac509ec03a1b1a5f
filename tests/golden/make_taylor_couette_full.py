"""Writes taylor_couette_full_oracle.json: the FP64 oracle's final state of the full-size
Taylor-Couette case (L = 200, r1 = 45, r2 = 70, 8000 steps; the case is defined in
tests/test_gpu_verification.py) at seeded sample nodes, so that the GPU path can be compared with
the oracle at full size without rerunning the oracle (about a minute on one core).

Calls only the oracle.  Run from the repository root:  python tests/golden/make_taylor_couette_full.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as O  # noqa: E402
from test_gpu_verification import L, R1, R2, NSTEPS, _case  # noqa: E402


def main():
    cfg, gamma, xs, ys, rr, w1 = _case("F64")
    r = O.solve(cfg, gamma, grad=False)
    rng = np.random.default_rng(20250630)
    gap = np.flatnonzero((rr > R1 + 1.0) & (rr < R2 - 1.0))
    disc = np.flatnonzero(rr <= R1 + 1.0)
    ring = np.flatnonzero(rr >= R2 - 1.0)
    nodes = np.sort(np.concatenate([rng.choice(gap, 96, replace=False),
                                    rng.choice(disc, 32, replace=False),
                                    rng.choice(ring, 32, replace=False)]))
    out = {
        "note": "FP64 oracle, final state after %d steps at the listed flat node indices "
                "(x + L*y); written by make_taylor_couette_full.py" % NSTEPS,
        "L": L, "r1": R1, "r2": R2, "nsteps": NSTEPS,
        "nodes": nodes.tolist(),
        "drho": [float(v) - 1.0 for v in r["rho"][nodes]],
        "ux": [float(v) for v in r["u"][0][nodes]],
        "uy": [float(v) for v in r["u"][1][nodes]],
    }
    with open(os.path.join(HERE, "taylor_couette_full_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
