"""Pins of the oracle's dense routes (Sec. II.A eqs. gammaeq, gammapole,
gammaF; Sec. II.C eq. Nmu and inertia counting).

Each pin compares against something other than the routine under test:
a second algorithm (inverse vs eigen-decomposition), a closed form, a bound
the mathematics fixes, or a pencil built with a known spectrum.
"""
import numpy as np
import pytest

from oracle import dense, poles, fermi
from paper_1405_0194_amd import lattice

BETA = lattice.BETA_300K


@pytest.fixture(scope="module")
def chain():
    s = lattice.config_system(0)
    H, S = s.dense()
    eig = dense.gen_eigh(H, S)
    mu = dense.half_filling_mu(eig[0])
    return s, H, S, eig, mu


def test_route_a_equals_route_b(chain):
    s, H, S, eig, mu = chain
    dE = 1.0 + abs(mu)
    w, om = poles.pole_table(BETA, dE, mu, 40, sets=("rho", "E"))
    ga = dense.gamma_route_a(H, S, w, om)
    gb = dense.gamma_route_b(H, S, w, om, eig=eig)
    for g in ("rho", "E"):
        err = np.max(np.abs(ga[g] - gb[g])) / np.max(np.abs(gb[g]))
        assert err < 1e-12, (g, err)


def test_pole_density_matrix_within_expansion_error_of_fermi_dirac(chain):
    s, H, S, eig, mu = chain
    dE = 1.0 + abs(mu)
    for P in (40, 60):
        w, om = poles.pole_table(BETA, dE, mu, P, sets=("rho",))
        gP = dense.gamma_route_a(H, S, w, om)["rho"]
        gFD, _ = dense.gamma_fermi_dirac(H, S, mu, BETA, eig=eig)
        e_p = poles.expansion_error(BETA, dE, mu, P, extra=eig[0])
        sinv = np.diag(np.linalg.inv(S))
        bound = e_p * np.sqrt(np.outer(sinv, sinv))   # |C r C^T - C f C^T| <= e_P sqrt(Sinv_ii Sinv_jj)
        assert np.all(np.abs(gP - gFD) <= bound * (1 + 1e-9) + 1e-14)


def test_traces_and_electron_count(chain):
    s, H, S, eig, mu = chain
    eps = eig[0]
    dE = 1.0 + abs(mu)
    w, om = poles.pole_table(BETA, dE, mu, 60, sets=("rho", "E"))
    g = dense.gamma_route_a(H, S, w, om)
    tGS, tGH = dense.traces(g["rho"], H, S)
    tES, _ = dense.traces(g["E"], H, S)
    r = poles.rational(eps, w, om["rho"])
    rE = poles.rational(eps, w, om["E"])
    # exact identities: Tr(Gamma S) = sum r(eps_i), Tr(Gamma H) = sum eps_i r(eps_i)
    assert abs(tGS - r.sum()) < 1e-10
    assert abs(tGH - (eps * r).sum()) < 1e-10
    assert abs(tES - rE.sum()) < 1e-10
    # half filling: mid-gap mu leaves N/2 states below it; the random
    # spectrum's gap is comparable to k_B T, so only the two states next to
    # mu are partially occupied
    e_p = poles.expansion_error(BETA, dE, mu, 60, extra=eps)
    Ntrue = dense.electron_number(eps, mu, BETA)
    assert abs(Ntrue - s.n) < 2.0
    assert abs(tGS - Ntrue) <= s.n * e_p + 1e-10
    e_pE = poles.expansion_error(BETA, dE, mu, 60, g="E", extra=eps)
    assert abs(tGH - tES) <= s.n * (np.max(np.abs(eps)) * e_p + e_pE) + 1e-10


def test_diagonal_pencil_closed_form():
    rng = np.random.default_rng(7)
    h = np.sort(rng.uniform(-0.9, 0.9, 12))
    H = np.diag(h)
    S = np.eye(12)
    mu = 0.01
    w, om = poles.pole_table(BETA, 1.0 + abs(mu), mu, 40, sets=("rho",))
    for l in (0, 7, 39):
        Z = dense.shifted_inverse(H, S, w[l])
        assert np.allclose(np.diag(Z), 1.0 / (h - w[l]), rtol=1e-14, atol=0)
        assert np.count_nonzero(Z - np.diag(np.diag(Z))) == 0
    g = dense.gamma_route_a(H, S, w, om)["rho"]
    r = np.imag(sum(om["rho"][l] / (h - w[l]) for l in range(40)))
    assert np.allclose(np.diag(g), r, atol=1e-13)


def test_two_by_two_inverse_closed_form():
    H = np.array([[0.3, -0.2], [-0.2, -0.1]])
    S = np.array([[1.2, 0.1], [0.1, 1.1]])
    w = 0.05 + 0.01j
    A = H - w * S
    det = A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0]
    Zc = np.array([[A[1, 1], -A[0, 1]], [-A[1, 0], A[0, 0]]]) / det
    assert np.allclose(dense.shifted_inverse(H, S, w), Zc, rtol=1e-14)


def test_conjugate_shift_symmetry(chain):
    s, H, S, eig, mu = chain
    w = mu + 0.3 + 0.004j
    Z1 = dense.shifted_inverse(H, S, w)
    Z2 = dense.shifted_inverse(H, S, np.conj(w))
    assert np.allclose(Z2, np.conj(Z1), rtol=1e-12, atol=1e-12 * np.abs(Z1).max())
    assert np.allclose(Z1, Z1.T, rtol=0, atol=1e-12 * np.abs(Z1).max())   # complex symmetric


def test_inertia_on_pencil_with_known_spectrum():
    rng = np.random.default_rng(11)
    n = 40
    lam = np.sort(rng.uniform(-1, 1, n))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = rng.standard_normal((n, n)) * 0.1 + np.eye(n)
    S = B @ B.T                         # SPD
    # H = S^{1/2} Q diag(lam) Q^T S^{1/2} has pencil eigenvalues lam
    ws, V = np.linalg.eigh(S)
    Sh = (V * np.sqrt(ws)) @ V.T
    H = Sh @ (Q * lam) @ Q.T @ Sh
    eps, _ = dense.gen_eigh(H, S)
    assert np.allclose(eps, lam, atol=1e-12)
    for e in rng.uniform(-1.2, 1.2, 25):
        assert dense.inertia_count(eps, e) == int(np.sum(lam < e))


def test_entry_error_floor():
    y = np.array([1.0, 1e-9, -0.5])
    x = y + np.array([1e-12, 1e-12, 0.0])
    err = dense.entry_error(x, y)
    assert err[1] == pytest.approx(1e-12 / 1e-3)


@pytest.mark.parametrize("kind,dims,orb,cut,herm", [("honeycomb", (4, 3), 5, 3.0, False),
                                                    ("cubic", (3, 3, 3), 4, 2.0, False),
                                                    ("honeycomb", (4, 3), 5, 3.0, True)])
def test_sparse_inverse_column_equals_dense_inverse(kind, dims, orb, cut, herm):
    """The Krylov column of A^{-1} (used at sizes the dense routes cannot
    reach) against the dense LU inverse, for a shift far from and one near
    the real axis."""
    from oracle import sparse
    mk = lattice.make_hermitian_system if herm else lattice.make_system
    s = mk(kind, dims, orb, cut, 17)
    H, S = s.dense()
    for w in (0.1 + 0.5j, -0.05 + 0.04j):
        A = sparse.matrix(s.n, s.colptr, s.rowind, s.hval, s.sval, w)
        assert np.abs(A.toarray() - (H - w * S)).max() == 0.0
        Z = dense.shifted_inverse(H, S, w)
        for j in (0, s.n // 2, s.n - 1):
            x = sparse.inverse_column(A, j)
            assert np.max(np.abs(x - Z[:, j])) <= 1e-12 * np.max(np.abs(Z[:, j]))
