"""Pins of the Hermitian-pencil oracle: the inverse route equals the
eigenbasis route; the result is Hermitian; for real symmetric input it
reduces to the entrywise imaginary part used for real pencils; the traces
equal the sums of r over the spectrum; the pole-expanded matrix is within the
expansion error of the Fermi-Dirac density matrix."""
import numpy as np
import pytest

from oracle import dense as od
from oracle import hermitian as oh
from oracle import poles as op
from paper_1405_0194_amd import lattice

BETA = lattice.BETA_300K


def _small(seed, imag=0.5):
    return lattice.make_hermitian_system("honeycomb", (3, 2), 5, 3.0, seed, imag_scale=imag)


@pytest.mark.parametrize("seed", [1, 2])
def test_routes_agree_and_are_hermitian(seed):
    s = _small(seed)
    H, S = s.dense()
    assert np.abs(H - H.conj().T).max() == 0 and np.abs(H.imag).max() > 0
    eig = oh.gen_eigh(H, S)
    mu = float(np.median(eig[0]))
    sh, w = op.pole_table(BETA, 1.0 + abs(mu), mu, 40, sets=("rho", "E"))
    A = oh.gamma_route_a(H, S, sh, w)
    Bm = oh.gamma_route_b(H, S, sh, w, eig)
    for g in ("rho", "E"):
        scale = np.abs(Bm[g]).max()
        assert np.abs(A[g] - Bm[g]).max() <= 1e-11 * scale
        assert np.abs(A[g] - A[g].conj().T).max() <= 1e-12 * scale
    trS, trH = oh.traces(A["rho"], H, S)
    r = op.rational(eig[0], sh, w["rho"])
    assert abs(trS - r.sum()) <= 1e-10 * len(r)
    assert abs(trH - (eig[0] * r).sum()) <= 1e-10 * len(r)


def test_real_input_reduces_to_entrywise_imaginary_part():
    s = lattice.make_system("honeycomb", (3, 2), 5, 3.0, 3)
    H, S = s.dense()
    sh, w = op.pole_table(BETA, 1.0, 0.0, 20, sets=("rho",))
    A = oh.gamma_route_a(H, S, sh, w)["rho"]
    R = od.gamma_route_a(H, S, sh, w)["rho"]
    assert np.abs(A.imag).max() <= 1e-13 * np.abs(R).max()
    assert np.abs(A.real - R).max() <= 1e-12 * np.abs(R).max()


def test_close_to_fermi_dirac_within_expansion_error():
    s = _small(4)
    H, S = s.dense()
    eig = oh.gen_eigh(H, S)
    mu = float(np.median(eig[0]))
    dE = 1.0 + abs(mu)
    P = 60
    sh, w = op.pole_table(BETA, dE, mu, P, sets=("rho",))
    G = oh.gamma_route_b(H, S, sh, w, eig)["rho"]
    F = oh.gamma_fermi_dirac(H, S, mu, BETA, eig)
    eP = op.expansion_error(BETA, dE, mu, P, extra=eig[0])
    Sinv = np.linalg.inv(S)
    d = np.sqrt(np.abs(np.real(np.diag(Sinv))))
    assert np.all(np.abs(G - F) <= eP * np.outer(d, d) + 1e-14)
