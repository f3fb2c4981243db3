"""GPU tests of batched (uneven multi-system) execution, graph plans and the
serving loop: every result equals the oracle's density matrix entry by entry
(the bar of the eager parity tests: |x - y| / max(|y|, 1e-3 max|y|) <= 1e-10,
traces within 1e-10 relative, inertia counts exact), and results do not
depend on batching, streams, residency or chunking (bit for bit where the
same kernels run in the same order)."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import dense as odense
from oracle import hermitian as oherm
from oracle import poles as opoles
from paper_1405_0194_amd import lattice

pytestmark = pytest.mark.gpu
BETA = lattice.BETA_300K
TOL = 1e-10
SETNAMES = ("rho", "E", "F", "d")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


_EIG = {}


def _eig(system):
    """Generalised eigenpairs of the pencil, cached per value arrays; the
    cache holds the arrays themselves, so their ids cannot be reused by
    other arrays while an entry exists."""
    k = (id(system.hval), id(system.sval))
    hit = _EIG.get(k)
    if hit is None or hit[0] is not system.hval or hit[1] is not system.sval:
        Hd, Sd = system.dense()
        eig = oherm.gen_eigh(Hd, Sd) if system.hermitian else odense.gen_eigh(Hd, Sd)
        hit = (system.hval, system.sval, Hd, Sd, eig)
        _EIG[k] = hit
    return hit[2:]


def assert_oracle(system, mu, P, dE, out, traces, nsets=2, what=""):
    """out (nsets, nnz) and traces (nsets, 2) of the HIP path against the
    oracle's eigenbasis route with its own pole table.

    Per-entry error |x - y| / max(|y|, 1e-3 scale).  For Gamma^rho the scale
    is max|Gamma^rho|.  The energy set's weights are omega^E_l = (z_l + mu)
    omega^rho_l-like, |z_l + mu| <= Delta E, so the terms it sums are up to
    Delta E times those of Gamma^rho and its rounding error scales with
    Delta E max|Gamma^rho|: that is its scale when it exceeds max|Gamma^E|
    (a spectrum much narrower than Delta E makes Gamma^E itself small)."""
    Hd, Sd, eig = _eig(system)
    names = SETNAMES[:nsets]
    ow, oom = opoles.pole_table(BETA, dE, mu, P, sets=names)
    if system.hermitian:
        G = oherm.gamma_route_b(Hd, Sd, ow, oom, eig=eig)
        trf = oherm.traces
    else:
        G = odense.gamma_route_b(Hd, Sd, ow, oom, eig=eig)
        trf = odense.traces
    cols = system.entry_cols()
    out = np.asarray(out)
    rho_max = float(np.max(np.abs(G["rho"][system.rowind, cols])))
    for g, name in enumerate(names):
        y = G[name][system.rowind, cols]
        scale = float(np.max(np.abs(y)))
        if name == "E":
            scale = max(scale, dE * rho_max)
        e = float(np.max(np.abs(out[g] - y) / np.maximum(np.abs(y), 1e-3 * scale)))
        tS, tH = trf(G[name], Hd, Sd)
        say(f"  oracle {what} {system.kind} N={system.n} P={P} {name}: worst entry error {e:.2e}")
        assert e <= TOL, (what, name, e)
        assert abs(traces[g][0] - tS) <= TOL * max(1.0, abs(tS)), (what, name, traces[g][0], tS)
        assert abs(traces[g][1] - tH) <= TOL * max(1.0, abs(tH)), (what, name, traces[g][1], tH)


def assert_counts(system, eps, neg):
    _, _, eig = _eig(system)
    ev = np.sort(eig[0])
    want = np.array([odense.inertia_count(ev, e) for e in eps])
    assert np.array_equal(np.asarray(neg), want), (neg, want)


def _alone(torch, system, mu, P, dE, nsets=2):
    from paper_1405_0194_amd import binding as B
    a = B.Analysis.from_system(system)
    H = torch.from_numpy(system.hval).to("cuda")
    S = torch.from_numpy(system.sval).to("cuda")
    out, tr, info, _, _ = B.density_matrix(a, H, S, BETA, dE, mu, P, nsets=nsets)
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


def test_batch_runner_equals_individual_runs_and_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd.batch import BatchRunner, Job
    mix = _small_mix()
    jobs = [Job(system=s, poles=P, mu=mu) for s, P, mu in mix]
    say("case: batch of", len(jobs), "systems on 3 streams")
    br = BatchRunner(jobs, budget_bytes=8 * 2**30, nstreams=3, keep_outputs=True)
    br.run()
    for j in jobs:
        got = j.out.cpu().numpy()
        assert np.all(j.info == 0)
        assert_oracle(j.system, j.mu, j.poles, j.dE, got, j.traces, what="batch")
        out, tr = _alone(torch, j.system, j.mu, j.poles, j.dE)
        assert np.array_equal(got, out), j.system.kind
        assert np.array_equal(j.traces, tr)


def test_uneven_batch_sample_against_oracle(torch_cuda):
    """Six systems of the 64-system uneven batch (two of each kind, N up to
    1,950, 40-70 poles), run together through the batch runner with the
    tuned analyses the benchmark uses; every result against the oracle."""
    from paper_1405_0194_amd import tune
    from paper_1405_0194_amd.batch import BatchRunner, Job
    pick = {6, 7, 9, 26, 28, 41}
    items = lattice.batch_systems(only=pick)
    jobs = [Job(system=s, poles=P, mu=0.0) for s, P in items]
    say("case: uneven batch sample", [(j.system.kind, j.system.n, j.poles) for j in jobs])
    br = BatchRunner(jobs, budget_bytes=32 * 2**30, nstreams=4, keep_outputs=True,
                     tuned=tune.load_cache() or None)
    br.run()
    for j in jobs:
        assert np.all(j.info == 0)
        assert_oracle(j.system, j.mu, j.poles, j.dE, j.out.cpu().numpy(), j.traces, what="uneven batch")


def test_server_results_alone_equal_results_in_mix_and_oracle(torch_cuda):
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
        got = q.out.cpu().numpy()
        assert np.all(q.info == 0)
        assert_oracle(q.system, q.mu, q.poles, q.dE, got, q.traces, what=f"served request {q.rid}")
        out, tr = _alone(torch, q.system, q.mu, q.poles, q.dE)
        if q.chunks == 1:
            # the same kernels in the same order: the same bits
            assert np.array_equal(got, out), q.rid
            assert np.array_equal(q.traces, tr), q.rid
        else:
            # pole chunks add their sums in another order
            assert np.max(np.abs(got - out)) <= 1e-12 * np.max(np.abs(out)), q.rid
            assert np.allclose(q.traces, tr, rtol=1e-12, atol=1e-12), q.rid
        if q.eps is not None:
            assert_counts(q.system, q.eps, q.neg_counts)


def test_server_chunks_a_request_larger_than_the_budget(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd.serve import Request, Server, resident_bytes
    s = lattice.make_system("cubic", (5, 5, 6), 13, 2.0, 21)
    P = 40
    a = B.Analysis.from_system(s)
    budget = resident_bytes(a, 12, 2) + 1024      # fits 12 of the 40 shifts
    srv = Server(budget_bytes=budget, nstreams=2, keep_outputs=True)
    eps = np.array([-0.05, 0.0, 0.07])
    req = Request(system=s, mu=0.0, poles=P, eps=eps)
    say("case: chunked request, budget", budget)
    srv.run([req], realtime=False)
    assert req.chunks > 1
    out, tr = _alone(torch, s, 0.0, P, req.dE)
    got = req.out.cpu().numpy()
    assert np.max(np.abs(got - out)) <= 1e-12 * np.max(np.abs(out))
    assert np.allclose(req.traces, tr, rtol=1e-12, atol=1e-12)
    assert np.all(req.info == 0)
    assert_oracle(s, 0.0, P, req.dE, got, req.traces, what="chunked request")
    assert_counts(s, eps, req.neg_counts)


def test_graph_plan_replays_match_eager_and_oracle(torch_cuda):
    """The captured graph replayed several times (with eager library work and
    synchronisations in between, new pole tables and new H values) gives the
    eager result bit for bit every time, and the oracle's."""
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    s = lattice.make_system("honeycomb", (6, 5), 13, 3.0, 31)
    a = B.Analysis.from_system(s)
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    P = 20
    say("case: graph plan replays")
    plan = B.Plan(a, H, S, P, nsets=2)
    rng = np.random.default_rng(2)
    cur = s
    for rep in range(4):
        mu = float(rng.uniform(-0.1, 0.1))
        if rep == 2:
            cur = dataclasses.replace(s, hval=s.hval * (1.0 + 1e-3 * rng.standard_normal(s.nnz_lower)))
            H.copy_(torch.from_numpy(cur.hval).cuda())
        dE = 1.0 + abs(mu)
        sh, wt = B.poles(BETA, dE, mu, P, 2)
        out_g, tr_g, info = plan.run(sh, wt)
        out_g = out_g.cpu().numpy().copy()
        out_e, tr_e, info_e, _, _ = B.density_matrix(a, H, S, BETA, dE, mu, P, nsets=2)
        torch.cuda.synchronize()
        assert np.array_equal(out_g, out_e.cpu().numpy()), rep
        assert np.array_equal(tr_g, tr_e), rep
        assert np.all(info == 0)
        if rep in (0, 2):
            assert_oracle(cur, mu, P, dE, out_g, tr_g, what=f"plan replay {rep}")


def _alone_hermitian(torch, system, mu, P, dE, analysis=None, nsets=2):
    from paper_1405_0194_amd import binding as B
    a = analysis if analysis is not None else B.Analysis.from_system(system)
    H = torch.from_numpy(system.hval).to("cuda")
    S = torch.from_numpy(system.sval).to("cuda")
    sh, wt = B.poles(BETA, dE, mu, P, nsets)
    f = B.HermitianFactorization(a, H, S, sh)
    f.selinv()
    out, tr = f.pole_sum(wt)
    torch.cuda.synchronize()
    return out.cpu().numpy(), tr


def test_hermitian_plan_replays_match_eager_and_oracle(torch_cuda):
    """The captured L D U + two-sided SelInv + pole sums, replayed with new
    pole tables and new H values (eager library work in between), equal the
    eager Hermitian runs bit for bit every time, and the oracle's
    (M - M^H)/2i."""
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
    cur = s
    for rep in range(4):
        mu = float(rng.uniform(-0.1, 0.1))
        if rep == 2:
            cur = dataclasses.replace(s, hval=s.hval * (1.0 + 1e-3 * rng.standard_normal(s.nnz_lower)))
            H.copy_(torch.from_numpy(cur.hval).cuda())
        dE = 1.0 + abs(mu)
        sh, wt = B.poles(BETA, dE, mu, P, 2)
        out_g, tr_g, info = plan.run(sh, wt)
        out_g = out_g.cpu().numpy().copy()
        f = B.HermitianFactorization(a, H, S, sh)
        f.selinv()
        out_e, tr_e = f.pole_sum(wt)
        torch.cuda.synchronize()
        assert np.array_equal(out_g, out_e.cpu().numpy()), rep
        assert np.array_equal(tr_g, tr_e), rep
        assert np.all(info == 0)
        if rep in (0, 2):
            assert_oracle(cur, mu, P, dE, out_g, tr_g, what=f"hermitian plan replay {rep}")


def test_batch_with_kpoints_equals_individual_runs_and_oracle(torch_cuda):
    """Real systems and four Hermitian 'k-points' (one pattern, one shared
    analysis, different values) in one batch on 3 streams: every result
    equals its run alone and the oracle's."""
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
        got = j.out.cpu().numpy()
        if j.system.hermitian:
            out, tr = _alone_hermitian(torch, j.system, j.mu, j.poles, j.dE, analysis=shared)
        else:
            out, tr = _alone(torch, j.system, j.mu, j.poles, j.dE)
        assert np.array_equal(got, out), j.system.kind
        assert np.array_equal(j.traces, tr)
        assert np.all(j.info == 0)
        assert_oracle(j.system, j.mu, j.poles, j.dE, got, j.traces, what="k-point batch")


@pytest.mark.parametrize("groups,waves", [(1, False), (2, False), (2, True)])
def test_fused_batch_equals_individual_runs_and_oracle(torch_cuda, groups, waves):
    """The fused multi-system execution (one launch per kernel kind holding
    the next panel operation of every system that uses it, captured as one
    graph per group of systems; with `waves`, a budget that splits the
    systems into waves sharing one arena): every system's result is the
    bits of its eager run alone, and the oracle's, over three replays."""
    torch = torch_cuda
    from paper_1405_0194_amd.batch import BatchRunner, Job
    mix = _small_mix(seed=11)
    jobs = [Job(system=s, poles=P, mu=mu) for s, P, mu in mix]
    budget = 8 * 2**30
    if waves:
        from paper_1405_0194_amd import binding as B
        from paper_1405_0194_amd.batch import footprint
        need = [footprint(B.Analysis.from_system(s, selinv_streams=1), P, 2) + 4096 for s, P, _ in mix]
        budget = max(max(need), sum(need) // 2)
    say("case: fused batch of", len(jobs), "systems in", groups, "groups, budget", budget)
    br = BatchRunner(jobs, budget_bytes=budget, nstreams=groups, keep_outputs=True, mode="fused",
                     groups=groups)
    for rep in range(3):
        br.run()
        for j in jobs:
            got = j.out.cpu().numpy()
            assert np.all(j.info == 0)
            out, tr = _alone(torch, j.system, j.mu, j.poles, j.dE)
            assert np.array_equal(got, out), (rep, j.system.kind)
            assert np.array_equal(j.traces, tr), rep
            if rep == 0:
                assert_oracle(j.system, j.mu, j.poles, j.dE, got, j.traces, what=f"fused batch g{groups}")
    say("fused launches", br.fused_launches())
    if waves:
        assert len(br.fused_launches()) >= 2


def test_fused_uneven_batch_sample_against_oracle(torch_cuda):
    """The six-system sample of the uneven batch through the fused path with
    the tuned analyses (as the benchmark runs it): every result against the
    oracle."""
    from paper_1405_0194_amd import tune
    from paper_1405_0194_amd.batch import BatchRunner, Job
    items = lattice.batch_systems(only={6, 7, 9, 26, 28, 41})
    jobs = [Job(system=s, poles=P, mu=0.0) for s, P in items]
    say("case: fused uneven batch sample")
    br = BatchRunner(jobs, budget_bytes=32 * 2**30, nstreams=2, keep_outputs=True,
                     tuned=tune.load_cache() or None, mode="fused", groups=2)
    br.run()
    for j in jobs:
        assert np.all(j.info == 0)
        assert_oracle(j.system, j.mu, j.poles, j.dE, j.out.cpu().numpy(), j.traces, what="fused uneven batch")


def test_server_small_request_after_large_one_finishes_first(torch_cuda):
    """Continuous batching: a small request admitted while a large one runs
    on another stream completes (and is recorded) before the large one."""
    from paper_1405_0194_amd.serve import Request, Server
    big = lattice.make_system("cubic", (7, 7, 7), 13, 2.0, 31)        # N = 4459
    small = lattice.make_system("chain", 40, 4, 2.0, 32)               # N = 160
    reqs = [Request(system=big, mu=0.0, poles=40, arrival=0.0),
            Request(system=small, mu=0.0, poles=20, arrival=0.02)]
    srv = Server(budget_bytes=64 * 2**30, nstreams=2, keep_outputs=True)
    say("case: small after large")
    summary = srv.run(reqs, realtime=True)
    say(summary, [(q.rid, q.t_admit, q.t_done) for q in reqs])
    qb, qs = reqs
    assert qs.t_admit < qb.t_done           # admitted while the large one ran
    assert qs.t_done < qb.t_done            # and finished first
    assert np.all(qb.info == 0) and np.all(qs.info == 0)
    assert_oracle(qs.system, qs.mu, qs.poles, qs.dE, qs.out.cpu().numpy(), qs.traces, what="small request")


def test_server_chunks_a_30k_cubic_request(torch_cuda):
    """A 3D bulk request of 30,576 orbitals (14 x 14 x 12 atoms, 40 poles,
    3.8 GB of factor storage and 16 TF per shift) under a budget that holds
    10 of its 40 shifts: the server runs it in pole chunks added into one
    output; the result equals the same request run alone in one batch, and
    the alone run's selected inverse equals the oracle's Krylov columns on
    sampled entries."""
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import tune
    from paper_1405_0194_amd.serve import Request, Server, resident_bytes
    from oracle import sparse as osparse
    s = lattice.make_system("cubic", (14, 14, 12), 13, 2.0, 1405)
    assert s.n == 30576
    P, mu = 40, 0.0
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    # alone: one batch of 40 shifts (SelInv in shift chunks that fit the device)
    a = tune.fit_to_budget(s, B.Analysis.from_system(s), P, int(240 * 2**30))
    from paper_1405_0194_amd.batch import job_dE
    dE = job_dE(s, mu)
    sh, wt = B.poles(BETA, dE, mu, P, 2)
    say(f"case: 30k cubic alone, SelInv chunk {a.options['selinv_chunk']}")
    f = B.Factorization(a, H, S, sh)
    assert np.all(f.info == 0)
    f.selinv()
    order = np.argsort(sh.imag)
    cols = s.entry_cols()
    rows = s.rowind.astype(np.int64)
    worst = 0.0
    for l in (int(order[-1]), int(order[-2])):
        A = osparse.matrix(s.n, s.colptr, s.rowind, s.hval, s.sval, sh[l])
        z = f.selected(l).cpu().numpy()
        for j in (777, s.n - 5):
            x = osparse.inverse_column(A, j)
            incol = np.nonzero(cols == j)[0]
            inrow = np.nonzero((rows == j) & (cols < j))[0]
            got = np.concatenate([z[incol], z[inrow]])
            want = np.concatenate([x[rows[incol]], x[cols[inrow]]])
            worst = max(worst, float(np.max(odense.entry_error(got, want))))
    say("sampled columns worst entry error", worst)
    assert worst <= TOL
    out_alone, tr_alone = f.pole_sum(wt)
    out_alone = out_alone.cpu().numpy().copy()
    del f
    torch.cuda.empty_cache()
    # served in pole chunks
    a1 = B.Analysis.from_system(s)
    budget = resident_bytes(a1, 10, 2) + a1.info["map_bytes"] + 2**20
    srv = Server(budget_bytes=budget, nstreams=2, keep_outputs=True, max_request_share=1.0)
    req = Request(system=s, mu=mu, poles=P, dE=dE)
    say("case: 30k cubic served in chunks, budget", budget)
    srv.run([req], realtime=False)
    assert req.chunks == 4 and np.all(req.info == 0)
    got = req.out.cpu().numpy()
    assert np.max(np.abs(got - out_alone)) <= 1e-12 * np.max(np.abs(out_alone))
    assert np.allclose(req.traces, tr_alone, rtol=1e-12, atol=1e-12)
    e_rho = opoles.expansion_error(BETA, dE, mu, P)
    e_E = opoles.expansion_error(BETA, dE, mu, P, g="E")
    assert abs(req.traces[0, 1] - req.traces[1, 0]) <= s.n * (e_rho + e_E) + 1e-8 * abs(req.traces[0, 1])
    assert 0.0 < req.traces[0, 0] < 2.0 * s.n
