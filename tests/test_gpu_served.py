"""The served path: batched rounds give each job exactly the result it gets alone (bitwise) and
through the single-job entry points, the HBM ledger gates admission, and a served job matches
the oracle."""
import math

import numpy as np
import pytest

import lks_inputs as I
from parity_util import announce, rel_l2

pytestmark = pytest.mark.gpu


def jobs():
    a = I.config_c3(n_side=96, nd_side=24, precision="F32", nsteps=120, checkpoint_every=25)
    b = I.make_config(dim=2, lattice="D2Q9", n=(130, 70), nd=(20, 16), nu=0.05, nsteps=90,
                      motion=I.motion_heave(90, (64.5, 34.5, 0.0), 3.0, 2 * math.pi / 60, theta_amp=0.3),
                      bcs=I.channel_bcs(2, 0.02), obj=I.objective("POWER", 1, 90),
                      u0=(0.02, 0, 0), precision="F32", checkpoint_every=11)
    c = I.config_c4(n_side=40, nd_side=14, precision="F32", nsteps=70, checkpoint_every=16)
    d = I.config_c4(n_side=36, nd_side=12, precision="F32", nsteps=50, checkpoint_every=0,
                    lattice="D3Q15")
    return [a, b, c, d]


def run_batched(cfgs, gammas, starts):
    """Start job i at round starts[i]; return (J, grad) per job."""
    import torch
    from paper_2506_23895_amd import lks
    stream = torch.cuda.current_stream().cuda_stream
    B = lks.Batch(stream)
    S = [lks.Solver(c, io_on_device=True, stream=stream) for c in cfgs]
    G = [torch.tensor(g, dtype=torch.float32, device="cuda") for g in gammas]
    O = [torch.empty_like(g) for g in G]
    active, done, r = [], [False] * len(cfgs), 0
    while not all(done):
        for i, st in enumerate(starts):
            if st == r:
                S[i].begin(G[i], O[i])
                active.append(i)
        run = [i for i in active if not done[i]]
        if run:
            flags = B.round([S[i] for i in run])
            for i, f in zip(run, flags):
                done[i] = bool(f)
        r += 1
    out = []
    for i in range(len(cfgs)):
        J = S[i].finish()
        out.append((J, O[i].cpu().numpy()))
        S[i].close()
    B.close()
    return out


def test_batched_equals_alone_and_plain_bitwise():
    from paper_2506_23895_amd import lks
    cfgs = jobs()
    gammas = [I.gamma_field(c["nd"], c["dim"], 10 + k).astype(np.float32) for k, c in enumerate(cfgs)]
    announce("served: mixed vs alone vs plain")
    mixed = run_batched(cfgs, gammas, starts=[0, 7, 3, 40])
    for k, c in enumerate(cfgs):
        alone = run_batched([c], [gammas[k]], starts=[0])[0]
        with lks.Solver(c) as s:
            Jp = s.forward(gammas[k])
            s.adjoint()
            gp = s.sensitivity()
        assert mixed[k][0] == alone[0] == Jp, (k, mixed[k][0], alone[0], Jp)
        assert np.array_equal(mixed[k][1], alone[1]), k
        assert np.array_equal(mixed[k][1], gp), k


def test_served_job_matches_oracle():
    from oracle import oracle as O
    c = jobs()[1]
    g = I.gamma_field(c["nd"], 2, 3)
    announce("served job vs oracle")
    J, grad = run_batched([c], [g.astype(np.float32)], starts=[0])[0]
    ref = O.solve(dict(c, precision="F64"), g)
    assert abs(J - ref["J"]) <= 1e-4 * abs(ref["J"])
    assert rel_l2(grad, ref["grad"]) <= 1e-3


def test_server_admission_by_budget():
    """With a budget that fits the largest job alone, requests wait for memory, the ledger never
    exceeds the budget, and every request completes."""
    from paper_2506_23895_amd import lks
    from paper_2506_23895_amd.server import Request, Server
    cfgs = jobs()[:3]
    need = max(lks.query_bytes(c) for c in cfgs)
    reqs = [Request(k, 0.0, c, I.gamma_field(c["nd"], c["dim"], 20 + k)) for k, c in enumerate(cfgs)]
    announce("server admission")
    srv = Server(hbm_budget=need + 1)
    res = srv.serve(reqs)
    srv.close()
    assert [r.status for r in res] == ["ok"] * 3
    assert srv.admission_waits > 0
    assert srv.peak_used <= need + 1


def test_server_shortest_work_first_bitwise():
    """With fill_cells set, jobs skip rounds while shorter ones advance; every result is still
    bitwise the one the job gets through the single-job entry points."""
    from paper_2506_23895_amd.server import Request, Server, serve_plain
    cfgs = jobs()[:3]
    reqs = [Request(k, 0.0, c, I.gamma_field(c["nd"], c["dim"], 40 + k)) for k, c in enumerate(cfgs)]
    announce("server shortest work first")
    srv = Server(fill_cells=1.0)  # one job per round
    res = srv.serve(reqs)
    srv.close()
    ref = serve_plain(reqs)
    for a, b in zip(res, ref):
        assert a.status == b.status == "ok"
        assert a.J == b.J, (a.rid, a.J, b.J)
        assert np.array_equal(a.grad, b.grad), a.rid


def test_server_single_shortest_job_rounds_bitwise():
    """With srpt_jobs set, rounds with few jobs running advance only the shortest one and fuller
    rounds advance every job; every result is still bitwise the single-job entry points' one."""
    from paper_2506_23895_amd.server import Request, Server, serve_plain
    cfgs = jobs()[:3]
    reqs = [Request(k, 0.0, c, I.gamma_field(c["nd"], c["dim"], 50 + k)) for k, c in enumerate(cfgs)]
    announce("server single shortest job rounds")
    srv = Server(srpt_jobs=2)  # three jobs: full rounds until one finishes, then one job per round
    res = srv.serve(reqs)
    srv.close()
    ref = serve_plain(reqs)
    for a, b in zip(res, ref):
        assert a.status == b.status == "ok"
        assert a.J == b.J, (a.rid, a.J, b.J)
        assert np.array_equal(a.grad, b.grad), a.rid


def test_submit_returns_futures_with_the_plain_results():
    """Server.submit: requests handed in while others run resolve to (J, dJ/dgamma, latency),
    bitwise those of the single-job entry points; a job whose state goes non-finite raises."""
    import torch
    from paper_2506_23895_amd import lks
    from paper_2506_23895_amd.server import Server
    torch.cuda.set_device(0)
    cfgs = jobs()[:3]
    gammas = [I.gamma_field(c["nd"], c["dim"], 30 + k).astype(np.float32) for k, c in enumerate(cfgs)]
    bad = dict(cfgs[1], nu=0.6)  # unstable viscosity: the forward goes non-finite
    announce("served: submit and futures")
    srv = Server()
    futs = []
    for k, (c, g) in enumerate(zip(cfgs, gammas)):
        futs.append(srv.submit(c, g))
        if k == 0:
            fbad = srv.submit(bad, gammas[1])
    results = [f.result(timeout=300) for f in futs]
    with pytest.raises(lks.LksError) as ei:
        fbad.result(timeout=300)
    assert ei.value.code == lks.LKS_ENONFINITE
    srv.close()
    for k, c in enumerate(cfgs):
        with lks.Solver(c) as s:
            Jp = s.forward(gammas[k])
            s.adjoint()
            gp = s.sensitivity()
        J, grad, lat = results[k]
        assert J == Jp and np.array_equal(grad, gp) and lat > 0, k


def test_server_zchunk_keeps_the_gradient_and_matches_a_solver_with_the_same_chunk():
    """Server(zchunk=16) gives 3D jobs 16-plane z chunks: each result is bitwise that of a Solver
    given the same chunk; dJ/dgamma is bitwise that of the default chunk, and J differs only in the
    FP64 rounding of the per-block partial sums."""
    import torch
    from paper_2506_23895_amd import lks
    from paper_2506_23895_amd.server import Server
    torch.cuda.set_device(0)
    cfgs = [c for c in jobs() if c["dim"] == 3]
    gammas = [I.gamma_field(c["nd"], c["dim"], 50 + k).astype(np.float32) for k, c in enumerate(cfgs)]
    announce("served: zchunk 16")
    srv = Server(zchunk=16)
    srv.zchunk_jobs = 1  # every 3D job takes the chunk, however few share the GPU
    futs = [srv.submit(c, g) for c, g in zip(cfgs, gammas)]
    results = [f.result(timeout=300) for f in futs]
    srv.close()
    for k, c in enumerate(cfgs):
        assert "zchunk" not in c  # the caller's configuration is left as it is
        with lks.Solver(dict(c, zchunk=16)) as s:
            J16 = s.forward(gammas[k])
            s.adjoint()
            g16 = s.sensitivity()
        with lks.Solver(c) as s:
            J0 = s.forward(gammas[k])
            s.adjoint()
            g0 = s.sensitivity()
        J, grad, _ = results[k]
        assert J == J16 and np.array_equal(grad, g16), k
        assert np.array_equal(g16, g0), k
        assert abs(J16 - J0) <= 1e-12 * abs(J0), (k, J16, J0)
