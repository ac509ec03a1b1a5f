#!/usr/bin/env python3
"""Benchmark: throughput of the full sensitivity evaluation on one MI355X.

One benchmark "step" is one pass of the whole hot path over the workload: the forward sweep
(transfer + LKS step for every time step, checkpoints every K steps), the reverse sweep (restore
each checkpoint, recompute its segment, adjoint step + sensitivity gather for every time step)
and the sensitivity dJ/dgamma on the design grid.  All inputs are seeded synthetic fields already
resident in HBM when the timed region starts (gamma lives in device memory).

Default workload: D2Q9 channel, 1024x1024 analysis grid, 256x256 design grid rotating (period
5000 steps: the stated 1000 drives the forward non-finite), 10000 steps, checkpoint every 100
with recomputation, time-averaged drag, FP32, LIN transfer.
Other workloads: --workload c2 (2048x1024 forward only, 20000 steps), c1 (64x64 FP64, 400 steps),
c4 (256^3 D3Q19, 3000 steps, checkpoint every 50), c5 (served sensitivity requests only).
Variant runs of a workload: --lattice D3Q15 (c4) and --transfer COS4 (the paper's cosine kernel).

Served leg (in the default line as "served", or alone with --workload c5): seeded requests from
the served mix (2D 128^2..1024^2 or 3D 64^3..160^3, 500..5000 steps) arrive as a Poisson stream
at --rate requests/s; the continuous-batching server runs them, then the same list runs back to
back through the single-job entry points.  Reports evals/s and p50/p99 latency of both.

Prints ONE JSON line.  value = MLUPS = cells * time steps / seconds (forward + reverse, or
forward only for c2).  The roofline object reports the dominant kernel's algorithmic bytes per
launch over its mean launch duration, measured with HIP events on the library's stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import lks_inputs as I  # noqa: E402

METRIC = "MLUPS fwd+adjoint (D2Q9/D3Q19, % HBM peak); sens-evals/s + p50/p99 latency"
HBM_PEAK_GBS = 8000.0
KINDS = {0: "fwd_step", 1: "adj_step", 2: "sens_gather"}


# Rotation / heave periods the benchmark uses.  With the stated ones (c3: 1000 steps, corner speed
# 1.14; c2: 2000 steps, heave plus a pitch whose corner speed is 0.57) the forward goes non-finite
# within 128 steps, in FP64 exactly as in FP32; these are the fastest periods of the tested sweeps
# (c3: 1000 .. 5000, c2: 2000 .. 40000) that stay finite over the whole horizon.
STABLE_PERIOD = {"c2": 10000.0, "c3": 5000.0}


def workload(name: str, nsteps: int, period: float = 0.0):
    if name == "c1":
        cfg = I.config_c1("F64")
    elif name == "c2":
        cfg = I.config_c2("F32", nsteps=nsteps or 20000, period=period or STABLE_PERIOD["c2"])
    elif name == "c3":
        cfg = I.config_c3(precision="F32", nsteps=nsteps or 10000,
                          period=period or STABLE_PERIOD["c3"])
    elif name == "c4":
        cfg = I.config_c4(precision="F32", nsteps=nsteps or 3000)
    else:
        raise SystemExit(f"unknown workload {name}")
    seed = {"c1": 0, "c2": 1, "c3": 2, "c4": 3}[name]
    gamma = I.gamma_field(cfg["nd"], cfg["dim"], seed)
    return cfg, gamma


def bytes_per_lup(cfg: dict) -> dict:
    """Algorithmic HBM bytes per lattice update of each stencil kernel (what it must move)."""
    e = 8 if cfg["precision"] == "F64" else 4
    D = cfg["dim"]
    # adjoint: read lambda and u^{n-1}, write lambda.  The 3D adjoint runs as two launches (a
    # pointwise kernel writes (P*, V*), the marching kernel reads them back); that intermediate is
    # this implementation's cost, not the method's, so it is not counted.  The footprint box
    # (kappa, u_S, kappa_bar) and the design grid are not counted either (under 2 B per update).
    adj = (2 * (1 + D) + D) * e
    return {
        "fwd_step": (2 * (1 + D)) * e,          # read rho, u; write rho, u
        "adj_step": adj,
    }


_HASH_OVERRIDE = None


def kernel_source_hash(read=None) -> str:
    """Hash of the device-code sources (the host runtime lks_api.hip is not part of it), with
    comments and whitespace removed, so that documentation edits keep measured profiles valid.
    read(name) -> text reads another revision of the sources (default: the working tree)."""
    import re
    if _HASH_OVERRIDE and read is None:
        return _HASH_OVERRIDE
    csrc = os.path.join(ROOT, "paper_2506_23895_amd", "csrc")
    if read is None:
        names = os.listdir(csrc)
        read = lambda f: open(os.path.join(csrc, f)).read()  # noqa: E731
    else:
        names = read(None)
    h = hashlib.sha256()
    for f in sorted(names):
        if f.endswith((".hip", ".hpp")) and f != "lks_api.hip":
            text = read(f)
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            h.update(f.encode() + b"\0" + " ".join(text.split()).encode())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, wl: str, per_launch_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it matches the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{wl}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_SINGLE = r"""
import sys, time, json
sys.path.insert(0, {root!r})
import numpy as np
import lks_inputs as I
from oracle import oracle as O
sys.path.insert(0, {root!r})
import bench
cfg, gamma = bench.workload({wl!r}, 0)
c = bench.sample_cfg(cfg, {steps})
t0 = time.perf_counter()
O.solve(c, gamma, grad=c["objective"]["kind"] != "NONE")
print(json.dumps({{"seconds": time.perf_counter() - t0, "threads": O.num_threads()}}))
"""


def sample_cfg(cfg: dict, sample_steps: int) -> dict:
    c = dict(cfg)
    c["nsteps"] = sample_steps
    c["motion"] = cfg["motion"][: sample_steps + 1]
    ob = dict(cfg["objective"])
    if ob["kind"] != "NONE":
        ob["n1"] = min(ob["n1"], sample_steps)
    c["objective"] = ob
    return c


def single_thread_rate(wl: str, cfg: dict, steps: int) -> dict:
    """The same oracle in a child process restricted to one OpenMP thread (a shorter sample)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", _SINGLE.format(root=ROOT, wl=wl, steps=steps)], env=env,
                         capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        return {"error": out.stderr[-300:]}
    r = json.loads(out.stdout.strip().splitlines()[-1])
    cells = int(np.prod(cfg["n"]))
    return {"value": round(cells * steps / r["seconds"] / 1e6, 4), "unit": "MLUPS", "cores": r["threads"],
            "sample": f"first {steps} steps, {r['seconds']:.1f} s"}


def cpu_baseline(wl: str, cfg: dict, gamma: np.ndarray) -> dict:
    """The FP64 oracle as it stands, on a bounded sample of the same workload."""
    from oracle import oracle as O
    sample_steps = {"c1": 400, "c2": 40, "c3": 100, "c4": 3}[wl]
    c = dict(cfg)
    c["nsteps"] = sample_steps
    c["motion"] = cfg["motion"][: sample_steps + 1]
    ob = dict(cfg["objective"])
    if ob["kind"] != "NONE":
        ob["n1"] = min(ob["n1"], sample_steps)
    c["objective"] = ob
    grad = ob["kind"] != "NONE"
    t0 = time.perf_counter()
    O.solve(c, gamma, grad=grad)
    dt = time.perf_counter() - t0
    cells = int(np.prod(c["n"]))
    single_steps = {"c1": 100, "c2": 6, "c3": 12, "c4": 1}[wl]
    return {"value": round(cells * sample_steps / dt / 1e6, 4), "unit": "MLUPS",
            "cores": O.num_threads(), "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{'x'.join(str(v) for v in c['n'][:c['dim']])} grid, first {sample_steps} steps "
                      f"{'forward + reverse' if grad else 'forward'}, FP64 C oracle, {dt:.1f} s",
            "single_thread": single_thread_rate(wl, cfg, single_steps)}


# z planes per block the server gives batched 3D jobs: a lone job's chunk is chosen to fill the
# GPU by itself (8 planes on the served grids); in a batch the other jobs fill it, and longer
# chunks re-evaluate fewer halo planes per block
SERVED_ZCHUNK = 16


def copy_reference(torch, dev, mib: int = 1024, reps: int = 10) -> dict:
    """A plain device-to-device copy of `mib` MiB timed with events: the achievable HBM rate of a
    streaming kernel on this GPU, reported beside the roofline fractions as a secondary reference."""
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    del a, b
    return {"achieved": round(gbs, 1), "unit": "GB/s", "bytes_moved_per_copy": 2 * n * 4,
            "ms_per_copy": round(ms, 4), "frac": round(gbs / 8000.0, 4)}


def served_leg(n_req: int, rate: float, seed: int = 5, fill_cells: float = 0.0, zchunk: int = 0,
               srpt_jobs: int = 4, max_active: int = 128) -> dict:
    """Continuous batching vs back-to-back plain solves on one seeded Poisson request list.  zchunk:
    z planes per block that the server gives 3D jobs (0: each job's own choice, as the plain solves
    make it)."""
    from paper_2506_23895_amd.server import Request, Server, serve_plain, summarize
    rng = np.random.default_rng(seed)
    t, reqs = 0.0, []
    for k in range(n_req):
        t += float(rng.exponential(1.0 / rate))
        cfg = I.served_job(rng)
        reqs.append(Request(k, t, cfg, I.gamma_field(cfg["nd"], cfg["dim"], 100 + k)))
    srv = Server(fill_cells=fill_cells, zchunk=zchunk, srpt_jobs=srpt_jobs, max_active=max_active)
    served = summarize(srv.serve(reqs))
    rounds = srv.rounds
    srv.close()
    plain = summarize(serve_plain(reqs))
    out = {"requests": n_req, "rate_req_per_s": rate, "served": served, "plain": plain,
           "rounds": rounds, "served_zchunk": zchunk, "srpt_jobs": srpt_jobs, "max_active": max_active,
           "mix": f"{sum(r.cfg['dim'] == 2 for r in reqs)} 2D / {sum(r.cfg['dim'] == 3 for r in reqs)} 3D, "
                  f"{sum(r.cfg['nsteps'] for r in reqs)} steps in total"}
    if served.get("evals_per_s") and plain.get("evals_per_s"):
        out["speedup_vs_plain"] = round(served["evals_per_s"] / plain["evals_per_s"], 3)
    return out


# ---- rocprofv3 summaries (run on the CPU after a profiled run; they write profiles/) ----------
# rocprofv3 kernel names of each timed kind, per dimension (3D adjoint: two launches per step)
PROFILED = {("fwd_step", 2): ["k_fwd2d_batch"], ("fwd_step", 3): ["k_fwd3d_batch"],
            ("adj_step", 2): ["k_adj2d_batch"],
            ("adj_step", 3): ["k_adj3d_prep_batch", "k_adj3d_main_batch"]}


def _csv(path):
    import csv
    return list(csv.DictReader(open(path)))


def _json_line(path):
    lines = [ln for ln in open(path) if ln.startswith("{")]
    return json.loads(lines[-1]) if lines else {}


def pmc_summary(fetch_csv: str, write_csv: str, wl: str, nsteps: int) -> None:
    """HBM bytes per launch of fwd_step and adj_step from one FETCH_SIZE and one WRITE_SIZE pass
    (each of a `--calibrate-copy` run), scaled by what the counters read for the 1 GiB copy."""
    import collections
    cfg, _ = workload(wl, nsteps)
    cells = int(np.prod(cfg["n"]))
    per = {}
    for path, cn in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        agg = collections.defaultdict(list)
        for r in _csv(path):
            if r["Counter_Name"] == cn:
                agg[(r["Kernel_Name"], r["Grid_Size"])].append(float(r["Counter_Value"]))
        per[cn] = agg
    gib_kib = 1024.0 * 1024.0
    factor = {}
    for cn, agg in per.items():
        big = max((max(v) for (k, _), v in agg.items() if "copyBuffer" in k), default=0.0)
        factor[cn] = gib_kib / big if big > 0 else float("nan")
    bpl = bytes_per_lup(cfg)
    for kind in ("fwd_step", "adj_step"):
        names = PROFILED[(kind, cfg["dim"])]
        kib = {}
        desc = []
        for cn, agg in per.items():
            tot = 0.0
            for nm in names:
                # the launches of this kernel with the most common grid (the per-step launches)
                cand = [(len(v), g, v) for (k, g), v in agg.items() if nm in k]
                if not cand:
                    break
                n_l, grid, v = max(cand)
                tot += sum(v) / len(v)
                if cn == "FETCH_SIZE":
                    desc.append(f"{nm}: {n_l} launches of grid {grid}")
            else:
                kib[cn] = tot
        if len(kib) != 2:
            continue
        hbm = (kib["FETCH_SIZE"] * factor["FETCH_SIZE"] + kib["WRITE_SIZE"] * factor["WRITE_SIZE"]) * 1024
        alg = bpl[kind] * cells
        cmd = ("rocprofv3 --pmc {c} -d {d} -o {o} --output-format csv -- python3 bench.py "
               f"--no-cpu-baseline --no-served --no-extra --steps 1 --warmup 0 --workload {wl} "
               f"--nsteps {nsteps} --calibrate-copy")
        out = [f"# HBM traffic per launch of {kind} ({', '.join(names)}) for the {cfg['name']} workload",
               "# commands (two passes, one counter each):"]
        for path, cn in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
            d = os.path.dirname(path)
            o = os.path.basename(path).split("_counter_collection")[0]
            out.append("#   " + cmd.format(c=cn, d=d, o=o))
        out += ["# calibration: --calibrate-copy runs one 1 GiB device-to-device copy first; the counters "
                "of that copy give",
                f"#   fetch_factor = {factor['FETCH_SIZE']:.4f}, write_factor = {factor['WRITE_SIZE']:.4f} "
                "(bytes moved / (counter KiB x 1024))",
                "# launches averaged: " + "; ".join(desc),
                f"# algorithmic bytes per launch: {bpl[kind]} B x {cells} cells = {alg}",
                f"kernel = {kind}", f"workload = {wl}",
                f"kernel_source_hash = {kernel_source_hash()}",
                f"fetch_kib_per_launch = {kib['FETCH_SIZE']:.1f}",
                f"write_kib_per_launch = {kib['WRITE_SIZE']:.1f}",
                f"fetch_factor = {factor['FETCH_SIZE']:.4f}",
                f"write_factor = {factor['WRITE_SIZE']:.4f}",
                f"hbm_bytes_per_launch = {hbm:.0f}",
                f"ratio_to_algorithmic = {hbm / alg:.3f}"]
        path = os.path.join(ROOT, "profiles", f"traffic_{kind}_{wl}.txt")
        open(path, "w").write("\n".join(out) + "\n")
        print("\n".join(out))


def trace_summary(prefix: str, log: str, plain_log: str, wl: str, cmd: str) -> None:
    """Per-kernel durations of a `rocprofv3 --kernel-trace --stats` run, the per-step kernels split by
    queue and grid, next to the bench lines of the profiled and of an unprofiled run."""
    import collections
    cfg, _ = workload(wl, 0)
    stats = _csv(prefix + "_kernel_stats.csv")
    out = [f"# rocprofv3 kernel trace: {cfg['name']} workload, {cfg['lattice']} "
           f"{'x'.join(str(v) for v in cfg['n'][:cfg['dim']])}, {cfg['precision']}, "
           f"{cfg['nsteps']} steps, checkpoint every {cfg['checkpoint_every']}",
           f"# command: {cmd}",
           f"# kernel sources: {kernel_source_hash()}   GPU: MI355X (gfx950), one device", "",
           f"{'kernel':58s} {'calls':>7s} {'avg us':>8s} {'min us':>8s} {'max us':>8s} {'share %':>8s}"]
    for r in stats[:12]:
        name = r["Name"].replace('"', "").split("(")[0][:58]
        out.append(f"{name:58s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:8.2f} "
                   f"{float(r['MinNs']) / 1e3:8.2f} {float(r['MaxNs']) / 1e3:8.2f} "
                   f"{float(r['Percentage']):8.2f}")
    agg = collections.defaultdict(list)
    for r in _csv(prefix + "_kernel_trace.csv"):
        k = r["Kernel_Name"]
        if any(nm in k for v in PROFILED.values() for nm in v):
            agg[(k.split("(")[0].replace("void ", ""), r["Queue_Id"], r["Grid_Size_X"])].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out += ["", "per-step kernels by queue and grid (the lowest queue id carries the forward sweep and "
                "the adjoint; the other one the segment recompute):"]
    for (k, q, gsz), v in sorted(agg.items()):
        if len(v) >= 4:
            out.append(f"  {k:34s} queue {q:>2s} grid {gsz:>8s}: {len(v):6d} launches, "
                       f"mean {sum(v) / len(v):8.2f} us")
    keys = ("value", "ms_per_step", "kernels", "roofline")
    prof, plain = _json_line(log), _json_line(plain_log) if plain_log else {}
    out += ["", "bench.py line of the profiled run (live HIP-event timing on the library stream):",
            "  " + json.dumps({k: prof.get(k) for k in keys})]
    if plain:
        out += ["bench.py line of the same workload without the profiler:",
                "  " + json.dumps({k: plain.get(k) for k in keys})]
    path = os.path.join(ROOT, "profiles", f"kernels_{cfg['lattice'].lower()}_{wl}.txt")
    open(path, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def measure(cfg: dict, gamma: np.ndarray, wl: str, steps: int, warmup: int, timing_every: int,
            variant: bool) -> dict:
    """Warm up, then time `steps` whole evaluations (forward, and reverse + sensitivity when the
    workload has an objective) with every input already in device memory."""
    import torch
    from paper_2506_23895_amd import lks
    dev = torch.device("cuda:0")
    tdtype = torch.float64 if cfg["precision"] == "F64" else torch.float32
    g_dev = torch.from_numpy(gamma).to(dev, dtype=tdtype)
    out = torch.empty_like(g_dev)
    has_adj = cfg["objective"]["kind"] != "NONE"
    cells = int(np.prod(cfg["n"]))
    N = cfg["nsteps"]
    print(f"[bench] workload {cfg['name']} cells={cells} steps={N} K={cfg['checkpoint_every']}",
          flush=True)
    solver = lks.Solver(cfg, io_on_device=True)

    def one():
        J = solver.forward(g_dev)
        if has_adj:
            solver.adjoint()
            solver.sensitivity(out)
        return J

    for w in range(warmup):
        J = one()
        print(f"[bench] warmup {w} J={J:.6e}", flush=True)
    solver.set_timing(timing_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tf = 0.0
    for k in range(steps):
        a0 = time.perf_counter()
        J = solver.forward(g_dev)
        tf += time.perf_counter() - a0
        if has_adj:
            solver.adjoint()
            solver.sensitivity(out)
        print(f"[bench] step {k} J={J:.6e}", flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = cells * N * steps / dt / 1e6
    finite = bool(torch.isfinite(out).all().item()) if has_adj else True

    # live means: forward-sweep launches for fwd_step; reverse-sweep launches of the one segment
    # that runs with no recompute beside it for adj_step and sens_gather
    timing = {}
    for kind, name in KINDS.items():
        cnt, mean = solver.kernel_timing(kind)
        timing[name] = {"samples": cnt, "mean_ms": mean}
    solver.close()
    K = cfg["checkpoint_every"] or N
    S = (N + K - 1) // K
    # forward-step launches: N in the forward sweep plus the recomputed segments (all but the last)
    # (2D: the gather of each adjoint step rides in the next adjoint launch; only the last one
    # is a launch of its own)
    launches = {"fwd_step": N + ((S - 1) * K if has_adj else 0),
                "adj_step": N if has_adj else 0,
                "sens_gather": (N if cfg["dim"] == 3 else 1) if has_adj else 0}
    tot = {k: launches[k] * timing[k]["mean_ms"] for k in launches}
    dom = max(tot, key=tot.get)
    bpl = bytes_per_lup(cfg)
    alg = bpl.get(dom, 0) * cells
    mean_s = timing[dom]["mean_ms"] / 1e3
    achieved = alg / mean_s / 1e9 if mean_s > 0 else 0.0
    # the committed counter summaries cover the workloads as stated, not their variants
    traffic = None if variant else read_traffic(dom, wl, alg)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": dom, "alg_bytes_per_launch": alg, "mean_launch_ms": timing[dom]["mean_ms"]}
    # whole evaluation at the algorithmic bytes of every launch it makes
    eval_bytes = sum(launches[k] * bpl.get(k, 0) * cells for k in ("fwd_step", "adj_step"))
    return {
        "value": round(value, 1), "unit": "MLUPS", "ms_per_eval": round(dt / steps * 1e3, 3),
        "config": {"workload": cfg["name"], "grid": list(cfg["n"][:cfg["dim"]]),
                   "design": list(cfg["nd"][:cfg["dim"]]), "lattice": cfg["lattice"],
                   "transfer": cfg["weight"], "precision": cfg["precision"],
                   "time_steps": N, "checkpoint_every": cfg["checkpoint_every"],
                   "objective": cfg["objective"]["kind"], "parallelism": "single GPU",
                   "motion_period": STABLE_PERIOD.get(wl)},
        "J": J, "sens_finite": finite, "fwd_ms_per_step": round(tf / steps * 1e3, 3),
        "evals_per_s": round(steps / dt, 4) if has_adj else None,
        "whole_eval_hbm_frac": round(eval_bytes * steps / dt / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": timing,
        "roofline": roof,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--requests", type=int, default=40, help="served leg: number of requests")
    ap.add_argument("--rate", type=float, default=50.0, help="served leg: arrivals per second")
    ap.add_argument("--rates", default="", help="c5: comma-separated arrival rates to sweep")
    ap.add_argument("--no-served", action="store_true", help="skip the served leg")
    ap.add_argument("--no-extra", action="store_true", help="skip the c4 and c2 legs of the default line")
    ap.add_argument("--fill-cells", type=float, default=0.0,
                    help="served leg: cells per round, shortest remaining work first (0: every job)")
    ap.add_argument("--zchunk", type=int, default=SERVED_ZCHUNK,
                    help="served leg: z planes per block of batched 3D jobs (0: each job's own choice)")
    ap.add_argument("--max-active", type=int, default=128, help="served leg: jobs admitted at once")
    ap.add_argument("--srpt-jobs", type=int, default=4,
                    help="served leg: with at most this many jobs running, one job per round, the one "
                         "with the least remaining work")
    ap.add_argument("--nsteps", type=int, default=0, help="override the time horizon (profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-every", type=int, default=8)
    ap.add_argument("--period", type=float, default=0.0, help="override the motion period")
    ap.add_argument("--lattice", choices=["D3Q19", "D3Q15"], default=None,
                    help="velocity set of a 3D workload (variant run; the default is D3Q19)")
    ap.add_argument("--transfer", choices=["LIN", "COS4"], default=None,
                    help="transfer kernel w (variant run; the workloads use LIN)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_*.txt from two rocprofv3 counter passes (CPU only)")
    ap.add_argument("--trace-summary", nargs=3, metavar=("PREFIX", "LOG", "PLAIN_LOG"),
                    help="write profiles/kernels_*.txt from a rocprofv3 kernel trace (CPU only)")
    ap.add_argument("--trace-command", default="", help="the profiled command, for the summary")
    ap.add_argument("--source-rev", default="",
                    help="summaries: git revision whose device sources were profiled (default: the "
                         "hash in the profiled run's log, else the working tree)")
    args = ap.parse_args()
    global _HASH_OVERRIDE
    if args.source_rev:
        import subprocess

        def read(f, rev=args.source_rev):
            path = "paper_2506_23895_amd/csrc"
            if f is None:
                out = subprocess.check_output(["git", "ls-tree", "--name-only", f"{rev}:{path}"], cwd=ROOT)
                return out.decode().split()
            return subprocess.check_output(["git", "show", f"{rev}:{path}/{f}"], cwd=ROOT).decode()
        _HASH_OVERRIDE = kernel_source_hash(read)
    elif args.trace_summary:
        _HASH_OVERRIDE = _json_line(args.trace_summary[1]).get("kernel_source_hash") or None
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, args.workload, args.nsteps)
        return 0
    if args.trace_summary:
        trace_summary(*args.trace_summary, args.workload, args.trace_command)
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (the multi-GPU "
                                   "halo-exchange design is documented, not built)"}))
        return 2

    import torch
    from paper_2506_23895_amd import lks
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {a.numel() * 4} bytes done", flush=True)
        del a, b

    if args.workload == "c5" and args.rates:
        # rate sweep: the same seeded request list shape at each rate, served then plain
        rows, sweep = [], []
        for rate in [float(v) for v in args.rates.split(",")]:
            print(f"[bench] served sweep: {args.requests} requests at {rate}/s", flush=True)
            sv = served_leg(args.requests, rate, fill_cells=args.fill_cells, zchunk=args.zchunk,
                            srpt_jobs=args.srpt_jobs, max_active=args.max_active)
            sweep.append(sv)
            a, b = sv["served"], sv["plain"]
            rows.append(f"{rate:6.1f} {a.get('evals_per_s', 0):8.3f} {a.get('p50_latency_s', 0):7.2f} "
                        f"{a.get('p99_latency_s', 0):7.2f} {b.get('evals_per_s', 0):8.3f} "
                        f"{b.get('p50_latency_s', 0):7.2f} {b.get('p99_latency_s', 0):7.2f} "
                        f"{sv.get('speedup_vs_plain', 0):6.3f}")
        print("# rate  served: evals/s  p50 s  p99 s | plain: evals/s  p50 s  p99 s | served/plain")
        print("\n".join(rows), flush=True)
        best = max(sweep, key=lambda v: v["served"].get("evals_per_s", 0))
        print(json.dumps({
            "metric": "sens-evals/s served (continuous batching) + p50/p99 latency",
            "value": best["served"].get("evals_per_s"), "unit": "evals/s", "n_gpus": 1, "steps": 1,
            "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "c5_served_mix", "requests": args.requests, "rates": args.rates,
                       "fill_cells": args.fill_cells, "parallelism": "single GPU"},
            "sweep": sweep}), flush=True)
        return 0
    if args.workload == "c5":
        t0 = time.perf_counter()
        sv = served_leg(args.requests, args.rate, fill_cells=args.fill_cells, zchunk=args.zchunk,
                        srpt_jobs=args.srpt_jobs, max_active=args.max_active)
        dt = time.perf_counter() - t0
        print(json.dumps({
            "metric": "sens-evals/s served (continuous batching) + p50/p99 latency",
            "value": sv["served"].get("evals_per_s"), "unit": "evals/s", "n_gpus": 1, "steps": 1,
            "warmup": 0, "ms_per_step": round(dt * 1e3, 1), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "c5_served_mix", "requests": args.requests,
                       "rate_req_per_s": args.rate, "parallelism": "single GPU"},
            "served": sv}), flush=True)
        return 0

    cfg, gamma = workload(args.workload, args.nsteps, args.period)
    variant = []
    if args.lattice and args.lattice != cfg["lattice"]:
        if cfg["dim"] != 3:
            raise SystemExit("--lattice applies to the 3D workload (c4)")
        cfg["lattice"] = args.lattice
        variant.append(args.lattice.lower())
    if args.transfer and args.transfer != cfg["weight"]:
        cfg["weight"] = args.transfer
        variant.append(args.transfer.lower())
    if variant:
        cfg["name"] += "_" + "_".join(variant)
    m = measure(cfg, gamma, args.workload, args.steps, args.warmup, args.timing_every, bool(variant))
    has_adj = cfg["objective"]["kind"] != "NONE"
    line = {
        "metric": METRIC if has_adj else "MLUPS fwd (D2Q9)",
        "value": m["value"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_per_eval"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if cfg["precision"] == "F64" else "f32", "data": "synthetic",
        "config": dict(m["config"], motion_period=args.period or STABLE_PERIOD.get(args.workload)),
    }
    line.update({k: v for k, v in m.items() if k not in ("value", "ms_per_eval", "config")})
    line["kernel_source_hash"] = kernel_source_hash()
    if args.workload == "c3" and not args.nsteps and not variant and not args.no_extra:
        # the D2Q9 headline is C3; the D3Q19 half of the metric (C4) and the forward-only C2 ride
        # in the same line, each with its own roofline, traffic and CPU baseline
        for wl, steps in (("c4", 2), ("c2", 2)):
            c2cfg, c2g = workload(wl, 0)
            print(f"[bench] {wl} leg", flush=True)
            sub = measure(c2cfg, c2g, wl, steps, 1, args.timing_every, False)
            sub["steps"], sub["warmup"] = steps, 1
            if not args.no_cpu_baseline:
                sub["cpu_baseline"] = cpu_baseline(wl, c2cfg, c2g)
            line[wl] = sub
        line["copy_reference"] = copy_reference(torch, dev)
    if has_adj and not args.no_served:
        print(f"[bench] served leg: {args.requests} requests at {args.rate}/s", flush=True)
        line["served"] = served_leg(args.requests, args.rate, fill_cells=args.fill_cells, zchunk=args.zchunk,
                        srpt_jobs=args.srpt_jobs, max_active=args.max_active)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, cfg, gamma)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
