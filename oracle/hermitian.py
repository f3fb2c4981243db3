"""Complex Hermitian pencils (oracle; test infrastructure only).

For Hermitian H and Hermitian positive definite S (k-point Hamiltonians, the
variant the paper names as future work in its conclusion), A_l = H - w_l S is
structurally symmetric but not symmetric, so the pole expansion cannot take
the entrywise imaginary part of sum_l omega_l Z_l.  Reading: with
H C = S C Xi, C^H S C = I, every inverse is Z_l = C (Xi - w_l)^{-1} C^H, so
M = sum_l omega_l Z_l = C diag(q) C^H with Im q_i = r(eps_i) ~ f(eps_i), and
the matrix imaginary part (M - M^H) / (2i) = C diag(r(Xi)) C^H is the pole
expansion of the density matrix (route A).  Entrywise,
Gamma_ij = (M_ij - conj(M_ji)) / (2i); for real symmetric H, S this reduces
to Im M_ij.  Route B applies r in the eigenbasis.
"""
import numpy as np
import scipy.linalg as sla

from . import dense
from . import fermi
from . import poles as _poles


def gen_eigh(H, S):
    """Eigenpairs of the Hermitian pencil (eps ascending, C^H S C = I)."""
    return sla.eigh(H, S)


def gamma_route_a(H, S, shifts, weights):
    """(M - M^H) / (2i), M = sum_l omega_l (H - w_l S)^{-1}, per weight set."""
    acc = {g: np.zeros(H.shape, dtype=np.complex128) for g in weights}
    for l, w in enumerate(shifts):
        Z = dense.shifted_inverse(H, S, w)
        for g, om in weights.items():
            acc[g] += om[l] * Z
    return {g: (a - a.conj().T) / 2j for g, a in acc.items()}


def gamma_route_b(H, S, shifts, weights, eig=None):
    """C diag(r^g(Xi)) C^H."""
    eps, C = gen_eigh(H, S) if eig is None else eig
    return {g: (C * _poles.rational(eps, shifts, om)[None, :]) @ C.conj().T for g, om in weights.items()}


def gamma_fermi_dirac(H, S, mu, beta, eig=None):
    """C f_beta(Xi - mu) C^H."""
    eps, C = gen_eigh(H, S) if eig is None else eig
    return (C * fermi.fermi(eps - mu, beta)[None, :]) @ C.conj().T


def traces(G, H, S):
    """Tr(G S) and Tr(G H) (real for Hermitian G, H, S)."""
    return float(np.real(np.sum(G * S.T))), float(np.real(np.sum(G * H.T)))
