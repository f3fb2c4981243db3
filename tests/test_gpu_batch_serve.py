"""GPU tests of batched (uneven multi-system) execution and of the serving
loop: results do not depend on batching, streams, residency or chunking."""
import sys

import numpy as np
import pytest

from paper_1405_0194_amd import lattice

pytestmark = pytest.mark.gpu
BETA = lattice.BETA_300K


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _alone(torch, system, mu, P, nsets=2):
    from paper_1405_0194_amd import binding as B
    a = B.Analysis.from_system(system)
    H = torch.from_numpy(system.hval).to("cuda")
    S = torch.from_numpy(system.sval).to("cuda")
    out, tr, info, _, _ = B.density_matrix(a, H, S, BETA, 1.0 + abs(mu), mu, P, nsets=nsets)
    torch.cuda.synchronize()
    return out.cpu().numpy(), tr


def _small_mix(seed=1):
    return [
        (lattice.make_system("cubic", (5, 5, 5), 4, 2.0, seed + 1), 24, 0.01),
        (lattice.make_system("chain", 90, 4, 2.0, seed + 2), 40, -0.02),
        (lattice.make_system("honeycomb", (6, 6), 13, 3.0, seed + 3), 30, 0.0),
        (lattice.make_system("cubic", (4, 4, 5), 13, 2.0, seed + 4), 20, 0.03),
        (lattice.make_system("chain", 170, 13, 2.0, seed + 5), 36, 0.0),
    ]


def test_batch_runner_equals_individual_runs(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd.batch import BatchRunner, Job
    mix = _small_mix()
    jobs = [Job(system=s, poles=P, mu=mu) for s, P, mu in mix]
    say("case: batch of", len(jobs), "systems on 3 streams")
    br = BatchRunner(jobs, budget_bytes=8 * 2**30, nstreams=3, keep_outputs=True)
    br.run()
    for j in jobs:
        out, tr = _alone(torch, j.system, j.mu, j.poles)
        assert np.array_equal(j.out.cpu().numpy(), out), j.system.kind
        assert np.array_equal(j.traces, tr)
        assert np.all(j.info == 0)


def test_server_results_alone_equal_results_in_mix(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd.serve import Request, Server, poisson_arrivals
    mix = _small_mix(seed=7)
    rng = np.random.default_rng(3)
    reqs = []
    for s, P, mu in mix:
        eps = np.sort(rng.uniform(mu - 0.1, mu + 0.1, 6))
        reqs.append(Request(system=s, mu=mu, poles=P, eps=eps))
    # SCF-style repeats: same pattern, perturbed H, other mu
    for k in (0, 2, 2):
        s, P, mu = mix[k]
        hv = s.hval * (1.0 + 1e-3 * rng.standard_normal(s.nnz_lower))
        import dataclasses
        reqs.append(Request(system=dataclasses.replace(s, hval=hv), mu=mu + 0.005, poles=P))
    arr = poisson_arrivals(len(reqs), rate=200.0, seed=5)
    for q, t in zip(reqs, arr):
        q.arrival = float(t)
    say("case: serving mix of", len(reqs), "requests, 3 streams, small budget")
    srv = Server(budget_bytes=3 * 2**30, nstreams=3, keep_outputs=True)
    summary = srv.run(reqs, realtime=True)
    say(summary)
    assert summary["symbolic_hits"] >= 3
    assert summary["plan_hits"] >= 1
    for q in reqs:
        out, tr = _alone(torch, q.system, q.mu, q.poles)
        assert np.array_equal(q.out.cpu().numpy(), out), q.rid
        assert np.array_equal(q.traces, tr), q.rid
        if q.eps is not None:
            from paper_1405_0194_amd import binding as B
            a = B.Analysis.from_system(q.system)
            neg, _ = B.inertia(a, torch.from_numpy(q.system.hval).to("cuda"),
                               torch.from_numpy(q.system.sval).to("cuda"), q.eps)
            assert np.array_equal(q.neg_counts, neg)


def test_server_chunks_a_request_larger_than_the_budget(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd.serve import Request, Server, resident_bytes
    s = lattice.make_system("cubic", (5, 5, 6), 13, 2.0, 21)
    P = 40
    a = B.Analysis.from_system(s)
    budget = resident_bytes(a, 12, 2) + 1024      # fits 12 of the 40 shifts
    srv = Server(budget_bytes=budget, nstreams=2, keep_outputs=True)
    req = Request(system=s, mu=0.0, poles=P)
    say("case: chunked request, budget", budget)
    srv.run([req], realtime=False)
    assert req.chunks > 1
    out, tr = _alone(torch, s, 0.0, P)
    got = req.out.cpu().numpy()
    assert np.max(np.abs(got - out)) <= 1e-12 * np.max(np.abs(out))
    assert np.allclose(req.traces, tr, rtol=1e-12, atol=1e-12)


def _alone_hermitian(torch, system, mu, P, analysis=None, nsets=2):
    from paper_1405_0194_amd import binding as B
    a = analysis if analysis is not None else B.Analysis.from_system(system)
    H = torch.from_numpy(system.hval).to("cuda")
    S = torch.from_numpy(system.sval).to("cuda")
    sh, wt = B.poles(BETA, 1.0 + abs(mu), mu, P, nsets)
    f = B.HermitianFactorization(a, H, S, sh)
    f.selinv()
    out, tr = f.pole_sum(wt)
    torch.cuda.synchronize()
    return out.cpu().numpy(), tr


def test_hermitian_plan_replays_match_eager(torch_cuda):
    """The captured L D U + two-sided SelInv + pole sums, replayed with new
    pole tables and new H values (eager library work in between), equal the
    eager Hermitian runs bit for bit every time."""
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    s = lattice.make_hermitian_system("honeycomb", (6, 5), 13, 3.0, 91)
    a = B.Analysis.from_system(s)
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    P = 20
    say("case: hermitian graph plan replays")
    plan = B.Plan(a, H, S, P, nsets=2)
    rng = np.random.default_rng(3)
    for rep in range(4):
        mu = float(rng.uniform(-0.1, 0.1))
        if rep == 2:
            H.copy_(torch.from_numpy(s.hval * (1.0 + 1e-3 * rng.standard_normal(s.nnz_lower))).cuda())
        sh, wt = B.poles(BETA, 1.0 + abs(mu), mu, P, 2)
        out_g, tr_g, info = plan.run(sh, wt)
        out_g = out_g.cpu().numpy().copy()
        f = B.HermitianFactorization(a, H, S, sh)
        f.selinv()
        out_e, tr_e = f.pole_sum(wt)
        torch.cuda.synchronize()
        assert np.array_equal(out_g, out_e.cpu().numpy()), rep
        assert np.array_equal(tr_g, tr_e), rep
        assert np.all(info == 0)


def test_batch_with_kpoints_equals_individual_runs(torch_cuda):
    """Real systems and four Hermitian 'k-points' (one pattern, one shared
    analysis, different values) in one batch on 3 streams: every result
    equals its run alone."""
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd.batch import BatchRunner, Job
    kp = [lattice.make_hermitian_system("honeycomb", (5, 5), 13, 3.0, 200 + k) for k in range(4)]
    assert all(np.array_equal(k.rowind, kp[0].rowind) for k in kp)
    shared = B.Analysis.from_system(kp[0])
    jobs = [Job(system=k, poles=24, mu=0.01 * i, analysis=shared) for i, k in enumerate(kp)]
    real = _small_mix(seed=7)[:3]
    jobs += [Job(system=s, poles=P, mu=mu) for s, P, mu in real]
    say("case: batch with", len(kp), "k-points and", len(real), "real systems on 3 streams")
    br = BatchRunner(jobs, budget_bytes=16 * 2**30, nstreams=3, keep_outputs=True)
    br.run()
    for j in jobs:
        if np.iscomplexobj(j.system.hval):
            out, tr = _alone_hermitian(torch, j.system, j.mu, j.poles, analysis=shared)
        else:
            out, tr = _alone(torch, j.system, j.mu, j.poles)
        assert np.array_equal(j.out.cpu().numpy(), out), j.system.kind
        assert np.array_equal(j.traces, tr)
        assert np.all(j.info == 0)
