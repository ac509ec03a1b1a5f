"""Continuous-batching sensitivity server.

Requests (a workload dictionary and a design field gamma) arrive over time.  The server admits a
request as soon as the HBM ledger (lks_query_bytes: state, checkpoints, trajectory store and
footprint stores of that job) fits under the budget and a slot is free, creates its context (so
its checkpoints stay resident on the device), and starts its evaluation with lks_begin.  Every
loop iteration is one lks_batch_round over all admitted jobs: each job advances by one
micro-step (forward step, recomputed step, or adjoint step plus sensitivity gather) and the
kernels of all jobs share one launch per kernel kind, so requests that arrive while others run
overlap with them on the device.  Finished jobs are detected with lks_poll (non-blocking), their
memory is released and queued requests are admitted.

serve_plain() runs the same request list back to back through lks_forward / lks_adjoint /
lks_sensitivity, one job at a time: the baseline the batched path is compared with.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import lks


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of serve()
    cfg: dict
    gamma: np.ndarray


@dataclass
class Result:
    rid: int
    J: float
    grad: np.ndarray
    arrival: float
    admitted: float
    finished: float
    status: str = "ok"
    cells_steps: float = 0.0
    alg_bytes: float = 0.0  # algorithmic HBM bytes of the evaluation (see alg_bytes)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def served_checkpoint(nsteps: int) -> int:
    """Checkpoint spacing for served jobs: sqrt(N) segments of sqrt(N) steps."""
    return max(1, int(math.ceil(math.sqrt(nsteps))))


@dataclass
class _Active:
    req: Request
    solver: lks.Solver
    gamma: torch.Tensor
    out: torch.Tensor
    nbytes: int
    admitted: float
    done: bool = False
    rounds: int = 0         # micro-steps taken (a job needs about 2 N: forward, then reverse)

    @property
    def cells(self) -> int:
        n = self.req.cfg["n"]
        return int(n[0] * n[1] * n[2])

    @property
    def remaining(self) -> float:
        return self.cells * max(1, 2 * self.req.cfg["nsteps"] - self.rounds)


class Server:
    """fill_cells > 0: each round advances only the admitted jobs with the least remaining work
    (cells x micro-steps left), as many as it takes to reach fill_cells cells in the round, so
    that short jobs finish first instead of sharing every round with long ones; 0 advances every
    admitted job every round."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 32, fill_cells: float = 0.0):
        free, total = torch.cuda.mem_get_info()
        self.budget = int(hbm_budget) if hbm_budget else int(0.8 * free)
        self.max_active = max_active
        self.fill_cells = float(fill_cells)
        self.stream = torch.cuda.current_stream().cuda_stream
        self.batch = lks.Batch(self.stream)
        self.rounds = 0
        self.admission_waits = 0
        self.peak_used = 0

    def serve(self, requests: List[Request]) -> List[Result]:
        pending = sorted(requests, key=lambda r: r.arrival)
        active: List[_Active] = []
        used = 0
        results: List[Result] = []
        t0 = time.perf_counter()
        dev = torch.device("cuda")
        while pending or active:
            now = time.perf_counter() - t0
            # admission: FIFO, by HBM ledger and slot count
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                rq = pending[0]
                need = lks.query_bytes(rq.cfg)
                if need > self.budget:
                    pending.pop(0)
                    results.append(Result(rq.rid, float("nan"), np.empty(0), rq.arrival, now, now,
                                          "rejected: over the HBM budget"))
                    continue
                if used + need > self.budget:
                    self.admission_waits += 1
                    break
                pending.pop(0)
                dt = torch.float64 if rq.cfg["precision"] == "F64" else torch.float32
                s = lks.Solver(rq.cfg, io_on_device=True, stream=self.stream)
                g = torch.as_tensor(rq.gamma, dtype=dt).to(dev)
                out = torch.empty_like(g)
                s.begin(g, out)
                used += need
                self.peak_used = max(self.peak_used, used)
                active.append(_Active(rq, s, g, out, need, time.perf_counter() - t0))
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (time.perf_counter() - t0))))
                continue
            running = [a for a in active if not a.done]
            if running and self.fill_cells > 0:
                running.sort(key=lambda a: a.remaining)
                acc, k = 0, 0
                while k < len(running) and (k == 0 or acc < self.fill_cells):
                    acc += running[k].cells
                    k += 1
                running = running[:k]
            if running:
                flags = self.batch.round([a.solver for a in running])
                self.rounds += 1
                for a, f in zip(running, flags):
                    a.done = bool(f)
                    a.rounds += 1
            # retire completed jobs without waiting on the stream
            for a in list(active):
                if a.done and a.solver.poll():
                    try:
                        J = a.solver.finish()
                        status = "ok"
                    except lks.LksError as e:
                        J, status = float("nan"), f"failed: {e}"
                    fin = time.perf_counter() - t0
                    cfg = a.req.cfg
                    results.append(Result(a.req.rid, J, a.out.cpu().numpy(), a.req.arrival,
                                          a.admitted, fin, status,
                                          float(np.prod(cfg["n"])) * cfg["nsteps"], alg_bytes(cfg)))
                    a.solver.close()
                    used -= a.nbytes
                    active.remove(a)
            if active and all(a.done for a in active):
                time.sleep(0.0005)  # everything enqueued: wait for the device
        return sorted(results, key=lambda r: r.rid)

    def close(self):
        self.batch.close()


def serve_plain(requests: List[Request]) -> List[Result]:
    """Baseline: the same requests one after another through the single-job entry points."""
    results = []
    t0 = time.perf_counter()
    stream = torch.cuda.current_stream().cuda_stream
    for rq in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if rq.arrival > now:
            time.sleep(rq.arrival - now)
        start = time.perf_counter() - t0
        dt = torch.float64 if rq.cfg["precision"] == "F64" else torch.float32
        with lks.Solver(rq.cfg, io_on_device=True, stream=stream) as s:
            g = torch.as_tensor(rq.gamma, dtype=dt).cuda()
            out = torch.empty_like(g)
            try:
                J = s.forward(g)
                s.adjoint()
                s.sensitivity(out)
                status = "ok"
            except lks.LksError as e:
                J, status = float("nan"), f"failed: {e}"
            torch.cuda.synchronize()
        fin = time.perf_counter() - t0
        results.append(Result(rq.rid, J, out.cpu().numpy(), rq.arrival, start, fin, status,
                              float(np.prod(rq.cfg["n"])) * rq.cfg["nsteps"], alg_bytes(rq.cfg)))
    return sorted(results, key=lambda r: r.rid)


HBM_PEAK_GBS = 8000.0


def alg_bytes(cfg: dict) -> float:
    """Algorithmic HBM bytes of one sensitivity evaluation: every forward step (sweep and segment
    recompute) reads and writes rho and u, every adjoint step reads lambda and u^{n-1} and writes
    lambda.  The footprint box and the design grid are not counted (under 2 B per update)."""
    e = 8 if cfg["precision"] == "F64" else 4
    D, N = cfg["dim"], cfg["nsteps"]
    cells = float(np.prod(cfg["n"]))
    K = cfg.get("checkpoint_every") or 0
    recomputed = 0 if K <= 0 else N - (N - ((N - 1) // K) * K)  # every segment but the last
    fwd, adj = 2 * (1 + D) * e, (2 * (1 + D) + D) * e
    return cells * ((N + recomputed) * fwd + N * adj)


def summarize(results: List[Result]) -> dict:
    ok = [r for r in results if r.status == "ok"]
    if not ok:
        return {"completed": 0}
    lat = np.array([r.latency for r in ok])
    span = max(r.finished for r in ok) - min(r.arrival for r in ok)
    return {"completed": len(ok), "failed": len(results) - len(ok),
            "evals_per_s": len(ok) / span if span > 0 else float("nan"),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mlups": sum(r.cells_steps for r in ok) / span / 1e6 if span > 0 else float("nan"),
            "achieved_gbs": sum(r.alg_bytes for r in ok) / span / 1e9 if span > 0 else float("nan"),
            "hbm_frac": sum(r.alg_bytes for r in ok) / span / 1e9 / HBM_PEAK_GBS if span > 0 else float("nan")}
