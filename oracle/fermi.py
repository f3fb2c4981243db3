"""Occupation functions of the pole expansions (oracle; test infrastructure).

All functions take x = epsilon - mu (real or complex) and beta.

* rho: the Fermi-Dirac occupation with the spin factor 2,
  f_beta(x) = 2 / (1 + exp(beta x))                 (Sec. II.A, eq. fermidirac)
* E:   the energy-weighted occupation (x + mu) f_beta(x), whose expansion
  gives the energy-density matrix Gamma^E             (Sec. II.A, eq. gammaF)
* F:   the free-energy occupation -(2/beta) ln(1 + exp(-beta x)), whose
  expansion gives Gamma^F in the free energy Tr[Gamma^F S] + mu N_e
                                                     (Sec. II.A, eqs.
                                                      Helmholtzpole, gammaF)
* d:   d f_beta(epsilon - mu) / d mu = -f_beta'(x), whose expansion gives
  N'_beta(mu) = Tr[Gamma^d S]                        (Sec. II.C)

The complex versions are the analytic continuations used at the quadrature
nodes; each branch below is chosen so that exp() never overflows.
"""
import numpy as np


def fermi(x, beta):
    """f_beta(x) = 2/(1+exp(beta x)), real or complex x."""
    x = np.asarray(x)
    bx = beta * x
    out = np.empty(np.broadcast(bx).shape, dtype=np.result_type(bx, np.float64))
    pos = np.real(bx) > 0
    e = np.exp(-bx[pos])
    out[pos] = 2.0 * e / (1.0 + e)
    out[~pos] = 2.0 / (1.0 + np.exp(bx[~pos]))
    return out


def energy_occ(x, beta, mu):
    """(x + mu) f_beta(x) = epsilon f_beta(epsilon - mu)."""
    return (np.asarray(x) + mu) * fermi(x, beta)


def free_occ(x, beta):
    """-(2/beta) ln(1 + exp(-beta x)), continued analytically off the real
    axis within |Im x| < pi/beta of the real axis and for Re x far from 0."""
    x = np.asarray(x)
    bx = beta * x
    out = np.empty(np.broadcast(bx).shape, dtype=np.result_type(bx, np.float64))
    pos = np.real(bx) > 0
    out[pos] = -(2.0 / beta) * np.log1p(np.exp(-bx[pos]))
    # ln(1 + e^{-y}) = -y + ln(1 + e^{y})
    out[~pos] = 2.0 * x[~pos] - (2.0 / beta) * np.log1p(np.exp(bx[~pos]))
    return out


def dfermi_dmu(x, beta):
    """d/dmu f_beta(epsilon - mu) = -f_beta'(x) = (beta/2) f (2 - f)."""
    f = fermi(x, beta)
    return 0.5 * beta * f * (2.0 - f)


def occupation(kind, x, beta, mu):
    if kind == "rho":
        return fermi(x, beta)
    if kind == "E":
        return energy_occ(x, beta, mu)
    if kind == "F":
        return free_occ(x, beta)
    if kind == "d":
        return dfermi_dmu(x, beta)
    raise ValueError(kind)
