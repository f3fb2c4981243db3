"""GPU parity of the high-level entry (paper_1405_0194_amd.api) against the
oracle: sparse torch / scipy inputs in, the pole-expanded matrices of every
weight set and the traces out, for a real symmetric and a complex Hermitian
pencil; the symbolic analysis is reused for a second mu on the same
pattern."""
import sys

import numpy as np
import pytest
import scipy.sparse as sps

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


def _lower_values(M, Dense):
    """(values of the sparse CSC result, the dense matrix at its entries)."""
    cp = M.ccol_indices().cpu().numpy()
    rows = M.row_indices().cpu().numpy()
    cols = np.repeat(np.arange(cp.shape[0] - 1), np.diff(cp))
    return M.values().cpu().numpy(), Dense[rows, cols]


def test_api_real_pencil_all_sets(torch_cuda):
    torch = torch_cuda
    from paper_1405_0194_amd import api
    s = lattice.make_system("honeycomb", (4, 3), 13, 3.0, 41)
    Hd, Sd = s.dense()
    eig = odense.gen_eigh(Hd, Sd)
    mu = odense.half_filling_mu(eig[0])
    P = 40
    Ht = torch.from_numpy(Hd).to_sparse_csr().cuda()
    St = torch.from_numpy(Sd).to_sparse_csr().cuda()
    say(f"case: api real honeycomb N={s.n} P={P}")
    solver = api.Solver()
    rho, E, F, d, tr = solver.density_matrix(Ht, St, mu, BETA, P, outputs=("rho", "E", "F", "d"))
    assert np.all(tr["info"] == 0)
    assert tr["dE"] >= np.max(np.abs(eig[0] - mu))
    ow, oom = opoles.pole_table(BETA, tr["dE"], mu, P)
    G = odense.gamma_route_a(Hd, Sd, ow, oom)
    for M, name in zip((rho, E, F, d), opoles.SETS):
        assert M.layout == torch.sparse_csc and M.shape == (s.n, s.n)
        x, y = _lower_values(M, G[name])
        err = float(np.max(odense.entry_error(x, y)))
        say(name, "worst entry error", err)
        assert err <= TOL
    tS, tH = odense.traces(G["rho"], Hd, Sd)
    assert abs(tr["N"] - tS) <= 1e-10 * abs(tS)
    assert abs(tr["Eband"] - tH) <= 1e-10 * max(1.0, abs(tH))
    assert abs(tr["TrES"] - odense.traces(G["E"], Hd, Sd)[0]) <= 1e-10 * max(1.0, abs(tH))
    fo = odense.traces(G["F"], Hd, Sd)[0] + mu * tS
    assert abs(tr["free_energy"] - fo) <= 1e-10 * max(1.0, abs(fo))
    dn = odense.traces(G["d"], Hd, Sd)[0]
    assert abs(tr["dN_dmu"] - dn) <= 1e-10 * abs(dn)
    # same pattern, another mu: the analysis is reused
    mu2 = mu + 0.01
    (rho2, tr2) = solver.density_matrix(Ht, St, mu2, BETA, P, outputs=("rho",))
    assert len(solver._cache) == 1
    ow2, oom2 = opoles.pole_table(BETA, tr2["dE"], mu2, P, sets=("rho",))
    G2 = odense.gamma_route_a(Hd, Sd, ow2, oom2)["rho"]
    x, y = _lower_values(rho2, G2)
    assert float(np.max(odense.entry_error(x, y))) <= TOL


def test_api_hermitian_pencil(torch_cuda):
    from paper_1405_0194_amd import api
    s = lattice.make_hermitian_system("honeycomb", (3, 2), 5, 3.0, 42)
    Hd, Sd = s.dense()
    eig = oherm.gen_eigh(Hd, Sd)
    mu = float(np.median(eig[0]))
    P = 30
    say(f"case: api hermitian honeycomb N={s.n} P={P}")
    rho, E, tr = api.Solver().density_matrix(sps.csr_matrix(Hd), sps.csr_matrix(Sd), mu, BETA, P)
    ow, oom = opoles.pole_table(BETA, tr["dE"], mu, P, sets=("rho", "E"))
    G = oherm.gamma_route_a(Hd, Sd, ow, oom)
    for M, name in ((rho, "rho"), (E, "E")):
        x, y = _lower_values(M, G[name])
        err = float(np.max(odense.entry_error(x, y)))
        say("hermitian", name, "worst entry error", err)
        assert err <= TOL
    tS, tH = oherm.traces(G["rho"], Hd, Sd)
    assert abs(tr["N"] - tS) <= 1e-10 * abs(tS)
    assert abs(tr["Eband"] - tH) <= 1e-10 * max(1.0, abs(tH))


@pytest.mark.parametrize("hermitian", [False, True])
def test_overlap_check_counts_negative_eigenvalues(torch_cuda, hermitian):
    """S shifted down by c I has #{lambda_i(S) < c} negative pivots
    (Sylvester); the unshifted S passes."""
    import scipy.linalg as sla
    from paper_1405_0194_amd import api
    mk = lattice.make_hermitian_system if hermitian else lattice.make_system
    s = mk("honeycomb", (3, 2), 5, 3.0, 43)
    Hd, Sd = s.dense()
    lam = sla.eigvalsh(Sd)
    solver = api.Solver()
    say(f"case: overlap check hermitian={hermitian} N={s.n}")
    ok, bad, info = solver.check_overlap(sps.csr_matrix(Hd), sps.csr_matrix(Sd))
    assert ok and bad == 0 and info == 0
    c = 0.5 * (lam[3] + lam[4])          # four eigenvalues below c
    Sbad = Sd - c * np.eye(s.n)
    ok, bad, info = solver.check_overlap(sps.csr_matrix(Hd), sps.csr_matrix(Sbad))
    assert not ok and info == 0 and bad == 4
    with pytest.raises(ValueError):
        solver.density_matrix(sps.csr_matrix(Hd), sps.csr_matrix(Sbad), 0.0, BETA, 10, dE=2.0,
                              check_overlap=True)


def test_api_runs_are_bitwise_reproducible(torch_cuda):
    """Two calls on the same input give identical bits (owner-computes
    updates, fixed reduction orders, SelInv on several streams)."""
    import torch
    from paper_1405_0194_amd import api
    s = lattice.make_system("honeycomb", (6, 5), 13, 3.0, 44)
    Hd, Sd = s.dense()
    Ht = torch.from_numpy(Hd).to_sparse_csr().cuda()
    St = torch.from_numpy(Sd).to_sparse_csr().cuda()
    solver = api.Solver(leaf_cols=64, selinv_streams=4)
    say(f"case: run-twice determinism N={s.n}")
    r1, e1, t1 = solver.density_matrix(Ht, St, 0.0, BETA, 40)
    v1, w1 = r1.values().clone(), e1.values().clone()
    r2, e2, t2 = solver.density_matrix(Ht, St, 0.0, BETA, 40)
    assert torch.equal(v1, r2.values()) and torch.equal(w1, e2.values())
    assert t1["N"] == t2["N"] and t1["Eband"] == t2["Eband"]
    # a caller's side stream: uploads, buffers and launches all on it
    side = torch.cuda.Stream()
    r3, e3, t3 = solver.density_matrix(Ht, St, 0.0, BETA, 40, stream=side)
    side.synchronize()
    assert torch.equal(v1, r3.values()) and torch.equal(w1, e3.values())
    assert t1["N"] == t3["N"]
