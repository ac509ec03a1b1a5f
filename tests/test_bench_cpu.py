"""Host logic of bench.py (CPU only): the one-GPU refusal, the kernel-source hash that keys the
committed HBM-traffic summaries, the counter calibration of those summaries, and the rule that a
summary taken at other kernel sources is not reported."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _sources():
    csrc = os.path.join(ROOT, "paper_2506_23895_amd", "csrc")
    return {f: open(os.path.join(csrc, f)).read() for f in os.listdir(csrc)
            if f.endswith((".hip", ".hpp"))}


def test_kernel_source_hash_ignores_comments_and_whitespace_but_not_code():
    src = _sources()

    def reader(s):
        return lambda f: list(s) if f is None else s[f]

    h0 = bench.kernel_source_hash(reader(src))
    dev = next(f for f in sorted(src) if f != "lks_api.hip" and f.endswith(".hip"))
    commented = dict(src)
    commented[dev] = "// a note\n/* a block\n comment */\n" + src[dev].replace("\n", "\n\n", 3)
    assert bench.kernel_source_hash(reader(commented)) == h0
    host = dict(src)
    host["lks_api.hip"] = src["lks_api.hip"] + "\nint unrelated_host_change;\n"
    assert bench.kernel_source_hash(reader(host)) == h0  # the host runtime is not device code
    changed = dict(src)
    changed[dev] = src[dev] + "\n__device__ int one_more_symbol;\n"
    assert bench.kernel_source_hash(reader(changed)) != h0


def _counter_csv(path, counter, rows):
    cols = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    with open(path, "w") as f:
        f.write(",".join(cols) + "\n")
        for i, (name, grid, val) in enumerate(rows):
            f.write(f'{i},"{name}",{grid},{counter},{val}\n')


def test_traffic_summary_scales_each_counter_by_the_copy_calibration(tmp_path, monkeypatch):
    """FETCH_SIZE reading half of a 1 GiB copy and WRITE_SIZE all of it give factors 2 and 1; the
    per-launch bytes of the most frequent grid of each kernel are then scaled by them."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_HASH_OVERRIDE", "feedfacecafebeef")
    (tmp_path / "profiles").mkdir()
    gib_kib = 1024.0 * 1024.0
    fwd, adj = "void lks::k_fwd2d_batch<float>(args)", "void lks::k_adj2d_batch<float>(args)"
    fetch = [("__amd_rocclr_copyBuffer", 1, gib_kib / 2)] + [(fwd, 427264, 9000.0)] * 5 + \
            [(fwd, 131072, 1.0)] + [(adj, 221184, 19000.0)] * 4
    write = [("__amd_rocclr_copyBuffer", 1, gib_kib)] + [(fwd, 427264, 12000.0)] * 5 + \
            [(fwd, 131072, 1.0)] + [(adj, 221184, 13000.0)] * 4
    _counter_csv(tmp_path / "f_counter_collection.csv", "FETCH_SIZE", fetch)
    _counter_csv(tmp_path / "w_counter_collection.csv", "WRITE_SIZE", write)
    bench.pmc_summary(str(tmp_path / "f_counter_collection.csv"), str(tmp_path / "w_counter_collection.csv"),
                      "c3", 300)
    kv = {}
    for line in open(tmp_path / "profiles" / "traffic_fwd_step_c3.txt"):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    assert float(kv["fetch_factor"]) == pytest.approx(2.0)
    assert float(kv["write_factor"]) == pytest.approx(1.0)
    assert float(kv["hbm_bytes_per_launch"]) == pytest.approx((9000.0 * 2 + 12000.0) * 1024, rel=1e-9)
    cells = 1024 * 1024
    assert float(kv["ratio_to_algorithmic"]) == pytest.approx((9000.0 * 2 + 12000.0) * 1024 / (24 * cells), abs=1e-3)
    assert kv["kernel_source_hash"] == "feedfacecafebeef"
    # the summary is reported while the sources match, and not once they change
    assert bench.read_traffic("fwd_step", "c3", 24 * cells) == pytest.approx(float(kv["hbm_bytes_per_launch"]))
    monkeypatch.setattr(bench, "_HASH_OVERRIDE", "0123456789abcdef")
    assert bench.read_traffic("fwd_step", "c3", 24 * cells) is None


def test_algorithmic_bytes_per_lattice_update():
    """The per-update bytes the roofline counts (fields read and written once per step)."""
    cfg3, _ = bench.workload("c3", 10)
    cfg4, _ = bench.workload("c4", 10)
    assert bench.bytes_per_lup(cfg3) == {"fwd_step": 24, "adj_step": 32}
    assert bench.bytes_per_lup(cfg4) == {"fwd_step": 32, "adj_step": 44}
