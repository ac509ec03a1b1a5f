"""Host logic of the served path, without a GPU: which jobs take a micro-step in a round (shortest
remaining work first, aged by waiting), and which admitted 3D jobs take the server's z chunk."""
from dataclasses import dataclass

from paper_2506_23895_amd.server import admitted_cfg, round_fill, select_round


@dataclass
class Job:
    cells: int
    left: int          # micro-steps left
    waited: int = 0

    @property
    def remaining(self):
        return self.cells * self.left


def simulate(max_wait, rounds=400):
    """One long job among short ones that keep arriving; returns the rounds the long job waited
    at most between two of its micro-steps."""
    long_job = Job(cells=1_000_000, left=10_000)
    shorts = [Job(cells=100_000, left=50) for _ in range(4)]
    worst = 0
    for r in range(rounds):
        jobs = [long_job] + shorts
        chosen = select_round(jobs, fill_cells=300_000, max_wait=max_wait)
        ids = set(id(j) for j in chosen)
        for j in jobs:
            if id(j) in ids:
                j.waited = 0
                j.left -= 1
            else:
                j.waited += 1
        worst = max(worst, long_job.waited)
        shorts = [j for j in shorts if j.left > 0]
        while len(shorts) < 4:  # sustained arrivals of short jobs
            shorts.append(Job(cells=100_000, left=50))
    return worst


def test_every_job_each_round_without_fill():
    jobs = [Job(10, 5), Job(20, 1)]
    assert select_round(jobs, 0.0, 64) == jobs


def test_shortest_work_first_fills_the_round():
    a, b, c = Job(100, 10), Job(100, 2), Job(300, 1)
    # keys (cells x steps left) b 200, c 300, a 1000: b alone holds 100 cells < 150, so c joins
    assert select_round([a, b, c], 150, 64) == [b, c]
    a.waited = 64  # a job that has waited max_wait rounds goes first, whatever its key
    assert select_round([a, b, c], 150, 64)[0] is a


def test_long_job_is_not_starved():
    assert simulate(max_wait=10**9) >= 399     # shortest-first alone: never picked
    assert simulate(max_wait=64) == 64         # picked again after at most max_wait rounds


def test_z_chunk_only_for_3d_jobs_admitted_into_a_loaded_gpu():
    c3, c2 = {"dim": 3, "nsteps": 10}, {"dim": 2, "nsteps": 10}
    assert admitted_cfg(c3, 2, 16, 4) is c3               # with it, three jobs share the GPU
    got = admitted_cfg(c3, 3, 16, 4)                       # four: the chunk applies
    assert got == {"dim": 3, "nsteps": 10, "zchunk": 16} and "zchunk" not in c3
    assert admitted_cfg(c2, 10, 16, 4) is c2               # 2D jobs have no z chunk
    own = {"dim": 3, "zchunk": 8}
    assert admitted_cfg(own, 10, 16, 4) is own             # a request's own choice stands
    assert admitted_cfg(c3, 10, 0, 4) is c3                # zchunk 0: off
    assert admitted_cfg(c3, 0, 16, 1)["zchunk"] == 16      # zchunk_jobs 1: every 3D job


def test_single_shortest_job_rounds_at_low_load():
    assert round_fill(3, 0.0, 4) == 1.0 and round_fill(4, 0.0, 4) == 1.0   # one job per round
    assert round_fill(5, 0.0, 4) == 0.0 and round_fill(5, 4e6, 4) == 4e6   # the usual rounds
    assert round_fill(1, 0.0, 0) == 0.0                                     # srpt_jobs 0: off
    a, b = Job(100, 10), Job(50, 3)
    assert select_round([a, b], round_fill(2, 0.0, 4), 64) == [b]          # the least work left
