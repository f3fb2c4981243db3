"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar (per entry): |x - y| / max(|y|, 1e-3 max|y|) <= 1e-10 for selected
inverses and pole sums; integer inertia counts bit-exact.  The oracle draws
its own pole table; the HIP library computes its own.
"""
import sys

import numpy as np
import pytest

from oracle import dense as odense
from oracle import poles as opoles
from paper_1405_0194_amd import lattice

pytestmark = pytest.mark.gpu
TOL = 1e-10
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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _run(torch, system, shifts, **akw):
    from paper_1405_0194_amd import binding as B
    a = B.Analysis.from_system(system, **akw)
    H = _dev(torch, system.hval)
    S = _dev(torch, system.sval)
    f = B.Factorization(a, H, S, shifts)
    return a, f, H, S


def _entries(system, Z):
    cols = system.entry_cols()
    return Z[system.rowind, cols]


def _max_entry_err(x, y):
    return float(np.max(odense.entry_error(x, y)))


def test_chain_selected_inverse_and_pole_sums(torch_cuda):
    torch = torch_cuda
    s = lattice.config_system(0)
    Hd, Sd = s.dense()
    eig = odense.gen_eigh(Hd, Sd)
    mu = odense.half_filling_mu(eig[0])
    dE = 1.0 + abs(mu)
    P = 40
    ow, oom = opoles.pole_table(BETA, dE, mu, P)
    from paper_1405_0194_amd import binding as B
    sh, wt = B.poles(BETA, dE, mu, P, 4)
    say("case: chain N=256 P=40 factor+selinv")
    a, f, H, S = _run(torch, s, sh)
    assert np.all(f.info == 0)
    f.selinv()
    torch.cuda.synchronize()
    worst = 0.0
    for l in range(P):
        z = f.selected(l).cpu().numpy()
        zo = _entries(s, odense.shifted_inverse(Hd, Sd, ow[l]))
        worst = max(worst, _max_entry_err(z, zo))
    say("selected inverse worst entry error", worst)
    assert worst <= TOL
    say("case: chain pole sums (rho, E, F, d)")
    out, tr = f.pole_sum(wt)
    out = out.cpu().numpy()
    G = odense.gamma_route_a(Hd, Sd, ow, oom)
    for g, name in enumerate(opoles.SETS):
        e = _max_entry_err(out[g], _entries(s, G[name]))
        say(name, "worst entry error", e)
        assert e <= TOL
        tS, tH = odense.traces(G[name], Hd, Sd)
        assert abs(tr[g, 0] - tS) <= 1e-10 * max(1.0, abs(tS))
        assert abs(tr[g, 1] - tH) <= 1e-10 * max(1.0, abs(tH))


def test_chain_factor_log_determinant(torch_cuda):
    torch = torch_cuda
    s = lattice.config_system(0)
    Hd, Sd = s.dense()
    shifts = np.array([0.01 + 0.003j, -0.3 + 0.05j, 0.2 + 1.5j])
    say("case: chain logdet via D")
    a, f, H, S = _run(torch, s, shifts)
    for l, w in enumerate(shifts):
        d = f.diag(l).cpu().numpy()
        sign, logabs = np.linalg.slogdet(Hd - w * Sd)
        assert abs(np.sum(np.log(np.abs(d))) - logabs) < 1e-9 * max(1.0, abs(logabs))
        ph = np.angle(np.prod(d / np.abs(d)))
        assert abs(np.angle(np.exp(1j * (ph - np.angle(sign))))) < 1e-9
        # the pivot bound of Im w lambda_min(S) (negative-definite imaginary part)
        assert np.min(np.abs(d)) >= w.imag * np.linalg.eigvalsh(Sd).min() * (1 - 1e-12)


def test_inertia_counts_match_eigenvalues(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    for k, sysm in enumerate([lattice.config_system(0),
                              lattice.make_system("honeycomb", (5, 5), 13, 3.0, 77),
                              lattice.make_system("cubic", (5, 5, 5), 4, 2.0, 78)]):
        Hd, Sd = sysm.dense()
        ev = np.sort(odense.gen_eigh(Hd, Sd)[0])
        rng = np.random.default_rng(100 + k)
        eps = []
        while len(eps) < 16:
            e = rng.uniform(ev[0] - 0.05, ev[-1] + 0.05)
            if np.min(np.abs(ev - e)) > 1e-8:
                eps.append(e)
        eps = np.array(eps)
        say("case: inertia", sysm.kind, sysm.n)
        a = B.Analysis.from_system(sysm)
        neg, info = B.inertia(a, _dev(torch, sysm.hval), _dev(torch, sysm.sval), eps)
        want = np.array([odense.inertia_count(ev, e) for e in eps])
        assert np.array_equal(neg, want), (neg, want)
        assert np.all(info == 0)


@pytest.mark.parametrize("kind,dims,orb,cut,akw", [
    ("honeycomb", (6, 6), 13, 3.0, {}),
    ("cubic", (5, 5, 5), 13, 2.0, {}),
    ("cubic", (4, 5, 6), 5, 2.0, dict(panel_width=23, leaf_cols=40)),
    ("chain", 301, 3, 2.0, dict(panel_width=7, leaf_cols=33)),
    ("honeycomb", (7, 5), 4, 3.0, dict(ordering=1, leaf_cols=70)),
    ("cubic", (5, 5, 5), 13, 2.0, dict(selinv_chunk=7)),
    ("honeycomb", (6, 6), 13, 3.0, dict(tile_rows=128)),
    ("honeycomb", (8, 7), 13, 3.0, dict(selinv_streams=1)),
    ("cubic", (6, 5, 5), 13, 2.0, dict(selinv_streams=8, selinv_chunk=13)),
    ("chain", 301, 3, 2.0, dict(panel_width=7, leaf_cols=33, tile_rows=128)),
    ("cubic", (6, 5, 5), 13, 2.0, dict(sep_cols=130)),
    ("cubic", (5, 5, 6), 5, 2.0, dict(sep_cols=20, panel_width=16, selinv_chunk=9)),
    ("cubic", (6, 5, 5), 13, 2.0, dict(fused_lanes=1)),
    ("chain", 301, 3, 2.0, dict(panel_width=7, leaf_cols=33, fused_lanes=-1)),
    ("honeycomb", (8, 7), 13, 3.0, dict(fused_lanes=1, selinv_streams=8, selinv_chunk=11, tile_rows=128)),
])
def test_lattice_parity_several_tiles(torch_cuda, kind, dims, orb, cut, akw):
    torch = torch_cuda
    s = lattice.make_system(kind, dims, orb, cut, 4242)
    Hd, Sd = s.dense()
    eig = odense.gen_eigh(Hd, Sd)
    mu = odense.half_filling_mu(eig[0])
    dE = 1.0 + abs(mu)
    P = 60
    ow, oom = opoles.pole_table(BETA, dE, mu, P, sets=("rho", "E"))
    from paper_1405_0194_amd import binding as B
    sh, wt = B.poles(BETA, dE, mu, P, 2)
    pick = np.array([0, 7, 19, 29, 30, 44, 59])    # includes the smallest Im w
    say("case:", kind, dims, orb, s.n, akw)
    a, f, H, S = _run(torch, s, sh, **akw)
    assert np.all(f.info == 0)
    f.selinv()
    for l in pick:
        z = f.selected(int(l)).cpu().numpy()
        zo = _entries(s, odense.shifted_inverse(Hd, Sd, ow[l]))
        e = _max_entry_err(z, zo)
        say("shift", l, "worst", e)
        assert e <= TOL
    out, tr = f.pole_sum(wt)
    out = out.cpu().numpy()
    G = odense.gamma_route_b(Hd, Sd, ow, oom, eig=eig)
    for g, name in enumerate(("rho", "E")):
        e = _max_entry_err(out[g], _entries(s, G[name]))
        say(name, e)
        assert e <= TOL


def test_random_pattern_no_blocks_graph_ordering(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    rng = np.random.default_rng(5)
    n = 333
    P = rng.uniform(size=(n, n)) < 0.01
    P = np.triu(P, 1)
    H = np.where(P, rng.standard_normal((n, n)), 0.0)
    S = np.where(P, 0.1 * rng.standard_normal((n, n)), 0.0)
    H = H + H.T + np.diag(rng.standard_normal(n))
    S = S + S.T
    S += np.diag(1.0 + np.abs(S).sum(axis=1))
    H /= np.abs(H).sum(axis=1).max()
    cols, rows, hv, sv = [], [], [], []
    colptr = [0]
    for j in range(n):
        r = [i for i in range(j, n) if (i == j or H[i, j] != 0 or S[i, j] != 0)]
        rows += r
        hv += [H[i, j] for i in r]
        sv += [S[i, j] for i in r]
        colptr.append(len(rows))
    colptr = np.array(colptr, dtype=np.int64)
    rows = np.array(rows, dtype=np.int32)
    hv = np.array(hv)
    sv = np.array(sv)
    a = B.Analysis(n, colptr, rows, leaf_cols=17, panel_width=11)
    shifts = np.array([0.0 + 0.002j, 0.3 + 0.01j, -0.7 + 0.5j])
    say("case: random pattern n=333 graph ND")
    f = B.Factorization(a, _dev(torch, hv), _dev(torch, sv), shifts)
    f.selinv()
    ec = np.repeat(np.arange(n), np.diff(colptr))
    for l, w in enumerate(shifts):
        z = f.selected(l).cpu().numpy()
        zo = np.linalg.inv(H - w * S)[rows, ec]
        assert _max_entry_err(z, zo) <= TOL


def test_diagonal_pencil_and_conjugate_pairs(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    n = 130
    rng = np.random.default_rng(9)
    h = rng.uniform(-0.9, 0.9, n)
    colptr = np.arange(n + 1, dtype=np.int64)
    rows = np.arange(n, dtype=np.int32)
    a = B.Analysis(n, colptr, rows)
    shifts = np.array([0.1 + 0.01j, 0.1 - 0.01j, -0.5 + 0.2j])
    say("case: diagonal pencil")
    f = B.Factorization(a, _dev(torch, h), _dev(torch, np.ones(n)), shifts)
    f.selinv()
    for l, w in enumerate(shifts):
        z = f.selected(l).cpu().numpy()
        assert np.allclose(z, 1.0 / (h - w), rtol=1e-14, atol=0)
    # conjugate shifts of a coupled system: Z(conj w) = conj Z(w)
    s = lattice.make_system("cubic", (4, 4, 4), 4, 2.0, 3)
    sh = np.array([0.05 + 0.004j, 0.05 - 0.004j])
    say("case: conjugate pair")
    a2, f2, _, _ = _run(torch, s, sh)
    f2.selinv()
    z0 = f2.selected(0).cpu().numpy()
    z1 = f2.selected(1).cpu().numpy()
    assert np.max(np.abs(z1 - np.conj(z0))) <= 1e-12 * np.max(np.abs(z0))


def test_tiny_pivot_reported(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    n = 40
    h = np.linspace(-0.5, 0.5, n)
    colptr = np.arange(n + 1, dtype=np.int64)
    rows = np.arange(n, dtype=np.int32)
    a = B.Analysis(n, colptr, rows, ordering=1)
    say("case: tiny pivot")
    neg, info = B.inertia(a, _dev(torch, h), _dev(torch, np.ones(n)), np.array([h[7], 0.013]))
    assert info[0] == 8          # 1-based column of the exact zero pivot
    assert info[1] == 0
    assert neg[1] == int(np.sum(h < 0.013))


def test_single_column(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    a = B.Analysis(1, np.array([0, 1]), np.array([0]))
    f = B.Factorization(a, _dev(torch, np.array([0.3])), _dev(torch, np.array([2.0])),
                        np.array([0.1 + 0.2j]))
    f.selinv()
    z = f.selected(0).cpu().numpy()
    assert abs(z[0] - 1.0 / (0.3 - (0.1 + 0.2j) * 2.0)) < 1e-15


def _diag_identity_residual(system, w, z):
    """max_i |sum_k A_ik Z_ki - 1| with A = H - w S, using only entries of the
    input pattern (every Z_ki needed is on it)."""
    n = system.n
    cols = system.entry_cols()
    rows = system.rowind.astype(np.int64)
    a = system.hval - w * system.sval
    acc = np.zeros(n, dtype=np.complex128)
    mag = np.zeros(n)
    # lower entry (r, c): contributes A_rc Z_cr to row r and A_cr Z_rc to row c
    np.add.at(acc, rows, a * z)
    np.add.at(mag, rows, np.abs(a * z))
    off = rows != cols
    np.add.at(acc, cols[off], a[off] * z[off])
    np.add.at(mag, cols[off], np.abs(a[off] * z[off]))
    return float(np.max(np.abs(acc - 1.0) / np.maximum(mag, 1.0)))


# device memory the benchmark gives factors + workspace (bench.py --hbm-budget-gib)
BENCH_BUDGET = int(270.0 * 2**30)


def _full_size_check(torch, cfg):
    """One density matrix of a full-size workload (mu = 0, 2 weight sets) in
    the benchmark's launch configuration (tuned analysis, SelInv shift
    chunks chosen for the same memory budget): sum_k A_ik Z_ki = 1 on the
    input pattern for the shifts nearest to and farthest from the real
    axis, sampled columns against the oracle, Tr(G H) against Tr(G^E S)
    within the expansion errors, and 0 < Tr(G S) < 2N."""
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import tune
    torch.cuda.empty_cache()
    s = lattice.config_system(cfg)
    mu = 0.0
    dE = 1.0 + abs(mu)
    P = lattice.CONFIG_POLES[cfg]
    a = tune.fit_to_budget(s, tune.tuned_analysis(s, P), P, BENCH_BUDGET)
    akw = a.options
    H = _dev(torch, s.hval)
    S = _dev(torch, s.sval)
    sh, wt = B.poles(BETA, dE, mu, P, 2)
    say(f"case: full-size config {cfg} N={s.n} P={P} {akw}")
    f = B.Factorization(a, H, S, sh)
    assert np.all(f.info == 0)
    f.selinv()
    order = np.argsort(sh.imag)
    for l in list(order[:2]) + [int(order[P // 2]), int(order[-1])]:
        z = f.selected(int(l)).cpu().numpy()
        r = _diag_identity_residual(s, sh[l], z)
        say("shift", l, "Im w", sh[l].imag, "diag(AZ)-1 residual", r)
        assert r <= 1e-11
    # sampled entries one by one: columns of A^{-1} from the oracle's Krylov
    # solve, against the selected inverse on the column's and the row's
    # input entries (shifts far from and nearer to the real axis)
    worst = _sampled_columns_error(f, s, sh, [int(order[-1]), int(order[P * 3 // 4])],
                                   [1234 % s.n, s.n - 77])
    say("sampled columns worst entry error", worst)
    assert worst <= TOL
    out, tr = f.pole_sum(wt)
    e_rho = opoles.expansion_error(BETA, dE, mu, P)
    e_E = opoles.expansion_error(BETA, dE, mu, P, g="E")
    bound = s.n * (1.0 * e_rho + e_E) + 1e-8 * abs(tr[0, 1])
    say("traces", tr, "bound", bound)
    assert abs(tr[0, 1] - tr[1, 0]) <= bound
    assert 0.0 < tr[0, 0] < 2.0 * s.n
    del f, H, S
    torch.cuda.empty_cache()


def _sampled_columns_error(f, s, sh, shifts, cols_j, upper=None):
    """Worst per-entry error of Z_l[:, j] on the input pattern against the
    oracle's column A_l^{-1} e_j: entries (i, j), i >= j, from the lower
    extraction; entries (j, k), k < j, hold Z[j][k], which equals Z[k][j]
    for complex symmetric A (or comes from the upper extraction, given as
    upper(l), for Hermitian A)."""
    from oracle import sparse as osparse
    cols = s.entry_cols()
    rows = s.rowind.astype(np.int64)
    worst = 0.0
    for l in shifts:
        A = osparse.matrix(s.n, s.colptr, s.rowind, s.hval, s.sval, sh[l])
        zl = f.selected(int(l)).cpu().numpy()
        zu = upper(int(l)) if upper is not None else zl
        for j in cols_j:
            x = osparse.inverse_column(A, j)
            incol = np.nonzero(cols == j)[0]
            inrow = np.nonzero((rows == j) & (cols < j))[0]
            got = np.concatenate([zl[incol], zu[inrow]])
            want = np.concatenate([x[rows[incol]], x[cols[inrow]]])
            worst = max(worst, float(np.max(odense.entry_error(got, want))))
    return worst


def test_full_size_honeycomb_bench_configuration(torch_cuda):
    """The benchmark workload itself (honeycomb N=26,624, 60 poles in one
    batch, the launch configuration the benchmark times)."""
    _full_size_check(torch_cuda, 1)


def test_full_size_cubic_configuration(torch_cuda):
    """The cubic bulk (N=22,464, 80 poles, mu inside the dense spectrum) at
    full size: 145 GiB of factors (separators cut at 832 columns), SelInv in
    the benchmark's shift chunks (40 under 270 GiB)."""
    _full_size_check(torch_cuda, 2)


@pytest.mark.parametrize("fused", [-1, 1])
def test_graph_plan_replays_match_eager(torch_cuda, fused):
    """The captured graph replayed several times (with eager library work and
    synchronisations in between, new pole tables and new H values) gives the
    eager result bit for bit every time (SelInv lanes fused into the
    capturing stream, or that stream alone)."""
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    s = lattice.make_system("honeycomb", (6, 5), 13, 3.0, 31)
    a = B.Analysis.from_system(s, fused_lanes=fused)
    H = _dev(torch, s.hval)
    S = _dev(torch, s.sval)
    P = 20
    say("case: graph plan replays, fused lanes", fused)
    plan = B.Plan(a, H, S, P, nsets=2)
    rng = np.random.default_rng(2)
    for rep in range(4):
        mu = float(rng.uniform(-0.1, 0.1))
        if rep == 2:
            H.copy_(_dev(torch, s.hval * (1.0 + 1e-3 * rng.standard_normal(s.nnz_lower))))
        sh, wt = B.poles(BETA, 1.0 + abs(mu), mu, P, 2)
        out_g, tr_g, info = plan.run(sh, wt)
        out_g = out_g.cpu().numpy().copy()
        # eager library work on other buffers between replays
        out_e, tr_e, info_e, _, _ = B.density_matrix(a, H, S, BETA, 1.0 + abs(mu), mu, P, nsets=2)
        torch.cuda.synchronize()
        assert np.array_equal(out_g, out_e.cpu().numpy()), rep
        assert np.array_equal(tr_g, tr_e), rep
        assert np.all(info == 0)


def test_results_do_not_depend_on_the_subtree_streams(torch_cuda):
    """Eager factorization and selected inversion on 1, 2, 4 or 8 subtree
    streams (and the in-order path of a single stream), or with 4 or 8
    subtree lanes fused on one stream, give the same factors, selected
    inverses, pole sums, traces and inertia counts bit for bit: the
    supernodes are issued in one order on every path and every entry
    receives its scatters in that order."""
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    s = lattice.make_system("honeycomb", (9, 8), 13, 3.0, 77)
    H = _dev(torch, s.hval)
    S = _dev(torch, s.sval)
    P = 24
    sh, wt = B.poles(BETA, 1.0, 0.0, P, 2)
    eps = np.array([-0.3, -0.01, 0.0, 0.2])
    ref = None
    for ns, fused in ((1, -1), (2, -1), (4, -1), (8, -1), (4, 1), (8, 1)):
        say("case: subtree streams", ns, "fused lanes", fused, "N", s.n)
        a = B.Analysis.from_system(s, selinv_streams=ns, fused_lanes=fused)
        f = B.Factorization(a, H, S, sh)
        d = f.diag(5).cpu().numpy().copy()
        f.selinv()
        z = f.selected(3).cpu().numpy().copy()
        out, tr = f.pole_sum(wt)
        neg, info = B.inertia(a, H, S, eps)
        got = (d, z, out.cpu().numpy().copy(), np.asarray(tr).copy(), np.asarray(neg).copy())
        assert np.all(f.info == 0) and np.all(np.asarray(info) == 0)
        if ref is None:
            ref = got
            continue
        for x, y in zip(got, ref):
            assert np.array_equal(np.asarray(x), np.asarray(y)), (ns, fused)


def test_maximum_batch_of_shifts(torch_cuda):
    """4096 shifts (the largest batch) in one factorization + SelInv;
    sampled shifts against the dense inverse."""
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    s = lattice.config_system(0)
    Hd, Sd = s.dense()
    rng = np.random.default_rng(4096)
    shifts = rng.uniform(-1.2, 1.2, 4096) + 1j * rng.uniform(1e-3, 0.5, 4096)
    say("case: chain N=256 with 4096 shifts")
    a, f, H, S = _run(torch, s, shifts)
    assert np.all(f.info == 0)
    f.selinv()
    torch.cuda.synchronize()
    worst = 0.0
    for l in (0, 1, 1000, 2047, 4094, 4095):
        z = f.selected(l).cpu().numpy()
        zo = _entries(s, odense.shifted_inverse(Hd, Sd, shifts[l]))
        worst = max(worst, _max_entry_err(z, zo))
    say("max batch worst entry error", worst)
    assert worst <= TOL


def test_two_pole_density_matrix(torch_cuda):
    """The smallest pole table (P = 2) through the fused call."""
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    s = lattice.config_system(0)
    Hd, Sd = s.dense()
    say("case: chain density matrix with P = 2")
    a = B.Analysis.from_system(s)
    H, S = _dev(torch, s.hval), _dev(torch, s.sval)
    out, tr, info, sh, wt = B.density_matrix(a, H, S, BETA, 1.0, 0.0, 2, nsets=2)
    assert np.all(info == 0)
    ow, oom = opoles.pole_table(BETA, 1.0, 0.0, 2)
    G = odense.gamma_route_a(Hd, Sd, ow, {k: oom[k] for k in ("rho", "E")})
    cols = s.entry_cols()
    out = out.cpu().numpy()
    for g, name in enumerate(("rho", "E")):
        assert _max_entry_err(out[g], G[name][s.rowind, cols]) <= TOL
