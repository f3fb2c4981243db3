"""Density of states and local density of states (oracle; test
infrastructure only).

Sec. II.D:
* eq. DOS: g(eps) = 2 sum_i delta(eps - eps_i); eq. cdos: its integral
  C(eps) is N_inf(eps), the zero-temperature count.  The DOS follows from
  samples of N_inf by interpolation and numerical differentiation.  Reading:
  on a grid of bin edges the derivative of the linear interpolant is the bin
  average (C(e_{b+1}) - C(e_b)) / (e_{b+1} - e_b), exact for each bin.
* eq. LDOSgreen / LDOSGreen: with a small eta > 0 the local DOS in the
  basis is G(eps) = (2/pi) Im [H - (eps + i eta) S]^{-1} (the imaginary part
  taken entrywise; reading: the printed formula leaves Im implicit, and the
  sign follows from the Plemelj formula, eq. ImPlemlj).
Independent routes used by the pins: the eigen-decomposition
G(eps) = C diag((2/pi) eta / ((eps_i - eps)^2 + eta^2)) C^T, whose trace
against S is the Lorentzian-broadened DOS.
"""
import numpy as np

from . import dense


def dos_bins(eig_sorted, edges):
    """Bin averages of g: 2 * #{eps_i in [e_b, e_{b+1})} / (e_{b+1} - e_b)."""
    ev = np.asarray(eig_sorted)
    edges = np.asarray(edges, dtype=np.float64)
    c = np.searchsorted(ev, edges, side="left")
    return 2.0 * np.diff(c) / np.diff(edges)


def ldos_dense(H, S, eps, eta):
    """(2/pi) Im [H - (eps + i eta) S]^{-1} by dense LU."""
    return (2.0 / np.pi) * np.imag(dense.shifted_inverse(H, S, eps + 1j * eta))


def ldos_eig(H, S, eps, eta, eig=None):
    """The same matrix from the generalised eigenpairs."""
    ev, C = dense.gen_eigh(H, S) if eig is None else eig
    w = (2.0 / np.pi) * eta / ((ev - eps) ** 2 + eta ** 2)
    return (C * w[None, :]) @ C.T


def broadened_dos(eig, eps, eta):
    """Tr[G(eps) S] = (2/pi) sum_i eta / ((eps - eps_i)^2 + eta^2)."""
    ev = np.asarray(eig)[None, :]
    e = np.atleast_1d(np.asarray(eps, dtype=np.float64))[:, None]
    return ((2.0 / np.pi) * eta / ((e - ev) ** 2 + eta ** 2)).sum(axis=1)
