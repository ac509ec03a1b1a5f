"""Host-side checks of the C ABI that need no GPU: the library loads, exports every symbol that
include/lks.h declares, and validates descriptors (and sizes the HBM ledger) before any HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import lks_inputs as I
from paper_2506_23895_amd import lks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "lks.h")).read()
    return sorted(set(re.findall(r"\b(lks_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = lks.lib()
    names = declared()
    assert set(names) == set(lks.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_no_cpu_fallback_in_binding():
    src = open(os.path.join(ROOT, "paper_2506_23895_amd", "lks.py")).read()
    assert "oracle" not in src.replace("oracle/", "")


@pytest.mark.parametrize("mutate,code", [
    (lambda c: c.update(nu=-0.1), lks.LKS_EINVAL),
    (lambda c: c.update(nu=float("nan")), lks.LKS_EINVAL),
    (lambda c: c.update(dim=4), lks.LKS_EINVAL),
    (lambda c: c.update(lattice="D3Q19"), lks.LKS_EINVAL),
    (lambda c: c["bc"].__setitem__(0, {"kind": "PERIODIC", "rho": 1.0, "u": (0, 0, 0)}), lks.LKS_EINVAL),
    (lambda c: c.update(n=(3, 64, 1)), lks.LKS_EINVAL),
    (lambda c: c["objective"].update(n0=0), lks.LKS_EINVAL),
    (lambda c: c["objective"].update(n1=10 ** 6), lks.LKS_EINVAL),
    (lambda c: c.update(checkpoint_every=-2), lks.LKS_EINVAL),
    (lambda c: c["motion"].__setitem__((5, 0), 2.0), lks.LKS_EINVAL),           # R not orthogonal
    (lambda c: c["motion"].__setitem__((7, 12), 5.0), lks.LKS_EINVAL),          # footprint leaves
    (lambda c: c.update(zchunk=4), lks.LKS_EINVAL),                              # z chunk below 8
    (lambda c: c.update(zchunk=64), lks.LKS_EINVAL),                             # ... above 32
])
def test_descriptor_validation(mutate, code):
    cfg = I.config_c1()
    cfg["motion"] = cfg["motion"].copy()
    cfg["bc"] = [dict(b) for b in cfg["bc"]]
    cfg["objective"] = dict(cfg["objective"])
    mutate(cfg)
    with pytest.raises(lks.LksError) as e:
        lks.query_bytes(cfg)
    assert e.value.code == code


def test_ledger_sizes_and_budget():
    c3 = I.config_c3()
    b = lks.query_bytes(c3)
    # checkpoints (100 x 3 fields) + two trajectory banks (2 x 101 x 2 fields: one segment is
    # recomputed while the adjoint reads the other) dominate, padded 1024 rows
    F = 1024 * 1024 * 4
    assert 100 * 3 * F + 2 * 101 * 2 * F < b < 100 * 3 * F + 2 * 101 * 2 * F + 0.5e9
    c3b = I.config_c3(checkpoint_every=0, nsteps=1000)  # whole trajectory kept
    assert lks.query_bytes(c3b) > 1000 * 2 * F
    # over the budget: create refuses before touching the device; query still reports the size
    assert lks.query_bytes(c3, hbm_budget=1 << 20) == b


def test_grids_of_2_pow_31_nodes_rejected():
    # the kernels decompose node indices with 32-bit arithmetic: create refuses larger grids
    # (checked before any allocation, so this runs without a GPU)
    cfg = I.config_c4(n_side=16, nd_side=6, nsteps=2)
    cfg["n"] = (2048, 1024, 1024)  # 2^31 nodes
    with pytest.raises(lks.LksError) as e:
        lks.query_bytes(cfg)
    assert e.value.code == lks.LKS_EINVAL
    assert "2^31" in str(e.value)


def test_create_rejects_over_budget_without_gpu():
    with pytest.raises(lks.LksError) as e:
        lks.Solver(I.config_c3(), hbm_budget=1 << 20)
    assert e.value.code == lks.LKS_ENOMEM


def test_error_strings():
    L = lks.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.lks_strerror(code)
