"""GPU parity of the chemical-potential search (Sec. II.C) against the
oracle: inertia bracketing from device counts equals the oracle's bracketing
from eigenvalue counts; Newton converges to the oracle's exact root of
N_P(mu) = N_e; a bracket reused across an SCF-style change of H still
converges, also when mu has left it."""
import sys

import numpy as np
import pytest

from oracle import chempot as oc
from oracle import dense as odense
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


def _systems():
    return {"chain": lattice.config_system(0),
            "honeycomb": lattice.make_system("honeycomb", (4, 3), 13, 3.0, 77)}


@pytest.mark.parametrize("name,frac", [("chain", 0.5), ("chain", 0.23), ("honeycomb", 0.5), ("honeycomb", 0.71)])
def test_bracket_and_newton_match_oracle(torch_cuda, name, frac):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import chempot as pc
    s = _systems()[name]
    Hd, Sd = s.dense()
    ev = odense.gen_eigh(Hd, Sd)[0]
    Ne = float(2 * round(frac * s.n)) + 0.37
    say(f"case: chempot {name} N={s.n} Ne={Ne}")
    a = B.Analysis.from_system(s).bind()
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    br = pc.inertia_bracket(a, H, S, Ne, -1.0, 1.0, BETA, Q=16, dN=0.1, rounds=3)
    olo, ohi, omu, samples = oc.bracket(oc.counts_from_eigenvalues(ev), Ne, -1.0, 1.0, BETA, Q=16, dN=0.1,
                                        rounds=3)
    say("bracket", br.lo, br.hi, br.mu, "oracle", olo, ohi, omu)
    assert abs(br.lo - olo) <= 1e-12 and abs(br.hi - ohi) <= 1e-12 and abs(br.mu - omu) <= 1e-12
    P = 40
    res = pc.newton_mu(a, H, S, Ne, br.mu, br.lo, br.hi, BETA, P, tol_ne=1e-8)
    mu_star = oc.mu_exact(ev, Ne, BETA, P, (-1.0, 1.0), br.lo, br.hi)
    Np, dNp = oc.n_pole(ev, res.mu, BETA, P, (-1.0, 1.0))
    say("newton", res.mu, res.N, res.dN, res.iterations, "oracle mu*", mu_star, "N_P", Np, dNp)
    assert abs(res.N - Ne) <= 1e-8
    assert abs(Np - res.N) <= 1e-9 * s.n
    assert abs(dNp - res.dN) <= 1e-9 * max(1.0, abs(dNp)) * s.n
    assert abs(res.mu - mu_star) <= 2e-8 / max(dNp, 1e-3) + 1e-12
    assert res.iterations < 30


def test_reused_bracket_recovers_when_mu_moves(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import chempot as pc
    s = _systems()["honeycomb"]
    Ne = float(s.n) + 0.37
    a = B.Analysis.from_system(s).bind()
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    say("case: SCF reuse, first solve")
    br, res = pc.solve_mu(a, H, S, Ne, BETA, 40, spectrum=(-1.0, 1.0))
    assert abs(res.N - Ne) <= 1e-8
    # next "SCF step": H' = 0.8 H + 0.15 S moves every eigenvalue e -> 0.8 e + 0.15
    say("case: SCF reuse, shifted H with the previous bracket")
    H2 = 0.8 * H + 0.15 * S
    br2, res2 = pc.solve_mu(a, H2, S, Ne, BETA, 40, spectrum=(-1.0, 1.0), previous=br, margin=0.01)
    assert br2.counts == 0
    Hd, Sd = s.dense()
    ev2 = odense.gen_eigh(0.8 * Hd + 0.15 * Sd, Sd)[0]
    mu_star = oc.mu_exact(ev2, Ne, BETA, 40, (-1.0, 1.0), -0.99, 0.99)
    say("reuse", res2.mu, res2.N, res2.iterations, "oracle", mu_star)
    assert abs(res2.N - Ne) <= 1e-8
    assert abs(res2.mu - mu_star) <= 2e-8 / max(res2.dN, 1e-3) + 1e-12


def test_hermitian_inertia_counts_match_eigenvalues(torch_cuda):
    """Counts of a complex Hermitian pencil from the signs of its L D U
    pivots equal the eigenvalue counts exactly."""
    torch = torch_cuda
    from oracle import hermitian as oherm
    from paper_1405_0194_amd import binding as B
    s = lattice.make_hermitian_system("honeycomb", (4, 3), 13, 3.0, 78)
    Hd, Sd = s.dense()
    ev = oherm.gen_eigh(Hd, Sd)[0]
    rng = np.random.default_rng(78)
    eps = np.sort(rng.uniform(-1.05, 1.05, 24))
    say(f"case: hermitian inertia N={s.n} {len(eps)} shifts")
    a = B.Analysis.from_system(s).bind()
    neg, info = B.inertia_hermitian(a, torch.from_numpy(s.hval).cuda(), torch.from_numpy(s.sval).cuda(), eps)
    want = np.array([odense.inertia_count(ev, e) for e in eps])
    assert np.all(info == 0)
    assert np.array_equal(neg, want), (neg, want)


def test_hermitian_bracket_and_newton_match_oracle(torch_cuda):
    """The mu search on a complex Hermitian pencil: bracket from the device
    counts equals the oracle's bracket from eigenvalue counts, Newton on the
    two-sided density matrices lands on the oracle's root."""
    torch = torch_cuda
    from oracle import hermitian as oherm
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import chempot as pc
    s = lattice.make_hermitian_system("honeycomb", (4, 3), 13, 3.0, 79)
    Hd, Sd = s.dense()
    ev = oherm.gen_eigh(Hd, Sd)[0]
    Ne = float(s.n) + 0.37
    say(f"case: hermitian chempot N={s.n} Ne={Ne}")
    a = B.Analysis.from_system(s).bind()
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    br = pc.inertia_bracket(a, H, S, Ne, -1.0, 1.0, BETA, Q=16, dN=0.1, rounds=3)
    olo, ohi, omu, _ = oc.bracket(oc.counts_from_eigenvalues(ev), Ne, -1.0, 1.0, BETA, Q=16, dN=0.1, rounds=3)
    say("bracket", br.lo, br.hi, br.mu, "oracle", olo, ohi, omu)
    assert abs(br.lo - olo) <= 1e-12 and abs(br.hi - ohi) <= 1e-12 and abs(br.mu - omu) <= 1e-12
    P = 40
    res = pc.newton_mu(a, H, S, Ne, br.mu, br.lo, br.hi, BETA, P, tol_ne=1e-8)
    mu_star = oc.mu_exact(ev, Ne, BETA, P, (-1.0, 1.0), br.lo, br.hi)
    Np, dNp = oc.n_pole(ev, res.mu, BETA, P, (-1.0, 1.0))
    say("newton", res.mu, res.N, res.dN, res.iterations, "oracle mu*", mu_star, "N_P", Np, dNp)
    assert abs(res.N - Ne) <= 1e-8
    assert abs(Np - res.N) <= 1e-9 * s.n
    assert abs(dNp - res.dN) <= 1e-9 * max(1.0, abs(dNp)) * s.n
    assert abs(res.mu - mu_star) <= 2e-8 / max(dNp, 1e-3) + 1e-12
