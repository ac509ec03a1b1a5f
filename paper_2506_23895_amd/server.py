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

Two ways in: serve(requests) replays a list of requests with arrival times (the benchmark);
submit(cfg, gamma) hands one request to a serving thread and returns a concurrent.futures.Future
that resolves to (J, dJ/dgamma, latency in s), or raises if the job failed (non-finite state, over
the HBM budget).

serve_plain() runs the same request list back to back through lks_forward / lks_adjoint /
lks_sensitivity, one job at a time: the baseline the batched path is compared with.
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

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
    waited: int = 0         # rounds since this job last took a micro-step
    future: Optional[cf.Future] = None

    @property
    def cells(self) -> int:
        n = self.req.cfg["n"]
        return int(n[0] * n[1] * n[2])

    @property
    def remaining(self) -> float:
        return self.cells * max(1, 2 * self.req.cfg["nsteps"] - self.rounds)


def select_round(jobs: Sequence, fill_cells: float, max_wait: int) -> list:
    """The jobs that take a micro-step this round.  fill_cells <= 0: every job.  Otherwise first
    every job that has waited max_wait rounds or more (so no job is passed over for ever, however
    long it is), then the jobs with the least remaining work (cells x micro-steps left), until the
    round holds fill_cells cells: short jobs finish first."""
    if fill_cells <= 0 or not jobs:
        return list(jobs)
    due = [a for a in jobs if a.waited >= max_wait]
    rest = sorted((a for a in jobs if a.waited < max_wait), key=lambda a: a.remaining)
    order = sorted(due, key=lambda a: -a.waited) + rest
    acc, k = 0, 0
    while k < len(order) and (k == 0 or acc < fill_cells or order[k].waited >= max_wait):
        acc += order[k].cells
        k += 1
    return order[:k]


def round_fill(n_running: int, fill_cells: float, srpt_jobs: int) -> float:
    """fill_cells of the next round: with at most srpt_jobs jobs running, a round holds only the job
    with the least remaining work (shortest remaining processing time first), else fill_cells."""
    return 1.0 if n_running <= srpt_jobs else fill_cells


def admitted_cfg(cfg: dict, n_active: int, zchunk: int, zchunk_jobs: int) -> dict:
    """The configuration a request is admitted with.  A 3D request that sets no z chunk of its own
    takes zchunk planes when, with it, at least zchunk_jobs jobs share the GPU: alone, its own
    choice fills the GPU and the longer chunk would leave part of it idle.  The caller's dict is
    left as it is."""
    if zchunk and cfg["dim"] == 3 and "zchunk" not in cfg and n_active + 1 >= zchunk_jobs:
        return dict(cfg, zchunk=zchunk)
    return cfg


class Server:
    """fill_cells > 0: each round advances only the admitted jobs with the least remaining work
    (cells x micro-steps left), as many as it takes to reach fill_cells cells in the round, so that
    short jobs finish first instead of sharing every round with long ones, and every job at least
    once every max_wait rounds; 0 advances every admitted job every round.

    srpt_jobs > 0 (default 4): while at most that many jobs are running, each round advances only
    the one with the least remaining work (its other rounds are the ones above).  At low load a job
    then runs with the GPU to itself instead of sharing every round, which keeps the median latency
    below the back-to-back plain solves at every arrival rate (mixed 2D/3D requests at 2 per
    second: p50 0.23 s against 0.29 s plain and 0.36 s with every job every round), at the cost of
    the tail at low rates: long jobs wait for the short ones (p99 3.9 s against 1.9 s plain and
    2.5 s).  0 keeps every round full (the tail setting).

    zchunk > 0: 3D jobs that do not set their own and are admitted while at least three others
    are active take z chunks of that many planes (8..32; the lks_desc field of that name).  A lone
    job's chunk is chosen to fill the GPU by itself; in a loaded batch the other jobs fill it, and
    longer chunks re-evaluate fewer halo planes per block.  Such
    a job's dJ/dgamma is bitwise the one of a Solver given the same zchunk, and its J differs from
    the default only in the FP64 rounding of the per-block partial sums."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 128, fill_cells: float = 0.0,
                 max_wait: int = 64, zchunk: int = 0, srpt_jobs: int = 4):
        free, total = torch.cuda.mem_get_info()
        self.budget = int(hbm_budget) if hbm_budget else int(0.8 * free)
        self.max_active = max_active
        self.fill_cells = float(fill_cells)
        self.max_wait = int(max_wait)
        self.zchunk = int(zchunk)
        self.zchunk_jobs = 4  # jobs sharing the GPU (this one included) from which zchunk applies
        self.srpt_jobs = int(srpt_jobs)
        self.device = torch.cuda.current_device()
        self.stream = torch.cuda.current_stream().cuda_stream
        self.batch = lks.Batch(self.stream)
        self.rounds = 0
        self.admission_waits = 0
        self.peak_used = 0
        self._inbox: "queue.Queue" = queue.Queue()
        self._thread: Optional[threading.Thread] = None
        self._stop = threading.Event()
        self._t0 = time.perf_counter()
        self._next_id = 0
        self._lock = threading.Lock()

    # -- request interface: a serving thread and futures ----------------------------------------
    def submit(self, cfg: dict, gamma) -> cf.Future:
        """Queue one sensitivity evaluation; the Future resolves to (J, dJ/dgamma, latency s)."""
        fut: cf.Future = cf.Future()
        with self._lock:
            rid = self._next_id
            self._next_id += 1
            if self._thread is None:
                self._thread = threading.Thread(target=self._run, name="lks-server", daemon=True)
                self._thread.start()
        req = Request(rid, time.perf_counter() - self._t0, cfg, np.asarray(gamma))
        self._inbox.put((req, fut))
        return fut

    def _run(self):
        torch.cuda.set_device(self.device)
        with torch.cuda.stream(torch.cuda.ExternalStream(self.stream)):
            self._loop(live=True)

    def shutdown(self, wait: bool = True):
        """Stop the serving thread once every submitted request is done (wait) or now."""
        if self._thread is not None:
            self._stop.set()
            if wait:
                self._thread.join()
            self._thread = None

    def serve(self, requests: List[Request]) -> List[Result]:
        """Replay requests at their arrival times (seconds after the call); results by request id."""
        self._t0 = time.perf_counter()
        for rq in sorted(requests, key=lambda r: r.arrival):
            self._inbox.put((rq, None))
        return sorted(self._loop(live=False, expected=len(requests)), key=lambda r: r.rid)

    def _loop(self, live: bool, expected: int = 0) -> List[Result]:
        pending: List[tuple] = []
        active: List[_Active] = []
        used = 0
        results: List[Result] = []
        t0 = self._t0
        dev = torch.device("cuda")

        def finish(res: Result, fut: Optional[cf.Future], grad=None):
            results.append(res)
            if fut is not None:
                if res.status == "ok":
                    fut.set_result((res.J, grad if grad is not None else res.grad, res.latency))
                else:
                    code = (lks.LKS_ENONFINITE if "non-finite" in res.status else
                            lks.LKS_ENOMEM if "budget" in res.status else lks.LKS_EINVAL)
                    fut.set_exception(lks.LksError(code, res.status))

        while True:
            while True:  # take what has been handed in
                try:
                    pending.append(self._inbox.get_nowait())
                except queue.Empty:
                    break
            pending.sort(key=lambda p: p[0].arrival)
            if not live and not pending and not active and len(results) >= expected:
                break
            if live and not pending and not active:
                if self._stop.is_set() and self._inbox.empty():
                    break
                try:
                    pending.append(self._inbox.get(timeout=0.005))
                except queue.Empty:
                    pass
                continue
            now = time.perf_counter() - t0
            # admission: FIFO, by HBM ledger and slot count
            while pending and pending[0][0].arrival <= now and len(active) < self.max_active:
                rq, fut = pending[0]
                try:
                    cfg = admitted_cfg(rq.cfg, len(active), self.zchunk, self.zchunk_jobs)
                    need = lks.query_bytes(cfg)
                except lks.LksError as e:
                    pending.pop(0)
                    finish(Result(rq.rid, float("nan"), np.empty(0), rq.arrival, now, now,
                                  f"failed: {e}"), fut)
                    continue
                if need > self.budget:
                    pending.pop(0)
                    finish(Result(rq.rid, float("nan"), np.empty(0), rq.arrival, now, now,
                                  "rejected: over the HBM budget"), fut)
                    continue
                if used + need > self.budget:
                    self.admission_waits += 1
                    break
                pending.pop(0)
                dt = torch.float64 if rq.cfg["precision"] == "F64" else torch.float32
                try:
                    s = lks.Solver(cfg, io_on_device=True, stream=self.stream)
                    g = torch.as_tensor(rq.gamma, dtype=dt).to(dev)
                    out = torch.empty_like(g)
                    s.begin(g, out)
                except lks.LksError as e:
                    finish(Result(rq.rid, float("nan"), np.empty(0), rq.arrival, now, now,
                                  f"failed: {e}"), fut)
                    continue
                used += need
                self.peak_used = max(self.peak_used, used)
                active.append(_Active(rq, s, g, out, need, time.perf_counter() - t0, future=fut))
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0][0].arrival - (time.perf_counter() - t0))))
                continue
            running = [a for a in active if not a.done]
            chosen = select_round(running, round_fill(len(running), self.fill_cells, self.srpt_jobs),
                                  self.max_wait)
            if chosen:
                flags = self.batch.round([a.solver for a in chosen])
                self.rounds += 1
                picked = set(id(a) for a in chosen)
                for a in running:
                    a.waited = 0 if id(a) in picked else a.waited + 1
                for a, f in zip(chosen, flags):
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
                    grad = a.out.cpu().numpy()
                    finish(Result(a.req.rid, J, grad, a.req.arrival, a.admitted, fin, status,
                                  float(np.prod(cfg["n"])) * cfg["nsteps"], alg_bytes(cfg)), a.future)
                    a.solver.close()
                    used -= a.nbytes
                    active.remove(a)
            if active and all(a.done for a in active):
                time.sleep(0.0005)  # everything enqueued: wait for the device
        return results

    def close(self):
        self.shutdown(wait=True)
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
