"""GPU parity of the complex Hermitian path (L D U factorization and
two-sided selected inversion) against the oracle: both triangles of every
selected inverse against the dense inverse, the pole-expanded density matrix
(the matrix imaginary part of the pole sum) against the oracle's inverse
route, its traces, and the real-pencil special case against the symmetric
path."""
import sys

import numpy as np
import pytest

from oracle import dense as odense
from oracle import hermitian as oherm
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


def _err(x, y):
    return float(np.max(odense.entry_error(x, y)))


CASES = {
    "chain": lambda: lattice.make_hermitian_system("chain", 64, 4, 2.0, 11),
    "honeycomb": lambda: lattice.make_hermitian_system("honeycomb", (6, 5), 13, 3.0, 12),
}


@pytest.mark.parametrize("name,akw", [("chain", {}), ("honeycomb", {}),
                                      ("honeycomb", dict(leaf_cols=256, panel_width=32))])
def test_hermitian_selected_inverse_both_triangles(torch_cuda, name, akw):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    s = CASES[name]()
    Hd, Sd = s.dense()
    rng = np.random.default_rng(5)
    shifts = rng.uniform(-0.3, 0.3, 5) + 1j * rng.uniform(1e-3, 0.2, 5)
    a = B.Analysis.from_system(s, **akw)
    say(f"case: hermitian {name} N={s.n} nsuper={a.info['nsuper']} npanel={a.info['npanel']} {akw}")
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    f = B.HermitianFactorization(a, H, S, shifts)
    assert np.all(f.info == 0)
    # log|det| from the pivots against the dense determinant
    for l in (0, 3):
        d = f.diag(l).cpu().numpy()
        sign, logdet = np.linalg.slogdet(Hd - shifts[l] * Sd)
        assert abs(np.sum(np.log(np.abs(d))) - logdet) <= 1e-9 * max(1.0, abs(logdet))
    f.selinv()
    cols = s.entry_cols()
    worst = 0.0
    for l in range(len(shifts)):
        Z = odense.shifted_inverse(Hd, Sd, shifts[l])
        lo = f.selected(l).cpu().numpy()
        up = f.selected(l, upper=True).cpu().numpy()
        worst = max(worst, _err(lo, Z[s.rowind, cols]), _err(up, Z[cols, s.rowind]))
    say("hermitian worst entry error", worst)
    assert worst <= TOL


def test_hermitian_density_matrix_and_traces(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    s = CASES["honeycomb"]()
    Hd, Sd = s.dense()
    eig = oherm.gen_eigh(Hd, Sd)
    mu = float(np.median(eig[0]))
    dE = 1.0 + abs(mu)
    P = 40
    sh, wt = B.poles(BETA, dE, mu, P, 2)
    osh, ow = opoles.pole_table(BETA, dE, mu, P, sets=("rho", "E"))
    say(f"case: hermitian density matrix N={s.n} P={P}")
    a = B.Analysis.from_system(s)
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    f = B.HermitianFactorization(a, H, S, sh)
    f.selinv()
    out, tr = f.pole_sum(wt)
    out = out.cpu().numpy()
    G = oherm.gamma_route_a(Hd, Sd, osh, ow)
    cols = s.entry_cols()
    for g, name in enumerate(("rho", "E")):
        err = _err(out[g], G[name][s.rowind, cols])
        say(name, "worst entry error", err)
        assert err <= TOL
        tS, tH = oherm.traces(G[name], Hd, Sd)
        assert abs(tr[g, 0] - tS) <= TOL * max(1.0, abs(tS))
        assert abs(tr[g, 1] - tH) <= TOL * max(1.0, abs(tH))


def test_real_pencil_through_hermitian_path_matches_symmetric_path(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    s = lattice.make_system("honeycomb", (5, 4), 13, 3.0, 13)
    shifts = np.array([0.05 + 0.01j, -0.2 + 0.3j])
    a = B.Analysis.from_system(s)
    say(f"case: real pencil, hermitian vs symmetric path N={s.n}")
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    fs = B.Factorization(a, H, S, shifts)
    fs.selinv()
    fh = B.HermitianFactorization(a, H.to(torch.complex128), S.to(torch.complex128), shifts)
    fh.selinv()
    for l in range(2):
        zs = fs.selected(l).cpu().numpy()
        assert _err(fh.selected(l).cpu().numpy(), zs) <= TOL
        assert _err(fh.selected(l, upper=True).cpu().numpy(), zs) <= TOL
