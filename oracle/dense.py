"""Dense CPU routes to the quantities the hot path computes (oracle; test
infrastructure).

Given dense real symmetric H, S (S positive definite), mu, beta and a pole
table {w_l = z_l + mu, omega_l^g}:

* selected inverse of one shift: Z_l = (H - w_l S)^{-1}
  (Sec. II.A: the exact inverse restricted to the selected pattern; selected
  inversion is exact up to roundoff) -- dense complex LU inverse;
* route A: Gamma^g = Im sum_l omega_l^g Z_l   (eqs. gammapole, gammaF);
* route B: H C = S C Xi, C^T S C = I, Gamma^g = C diag(r^g(Xi)) C^T with
  r^g(eps) = Im sum_l omega_l^g/(eps - w_l)   (the same expansion applied in
  the eigenbasis, since (H - wS)^{-1} = C (Xi - w)^{-1} C^T);
* Fermi-Dirac truth Gamma_FD = C f_beta(Xi - mu) C^T (eq. gammaeq) and
  N_beta(mu) = sum_i f_beta(eps_i - mu) = Tr[Gamma_FD S] (eq. Nmu);
* traces Tr(Gamma S), Tr(Gamma H), Tr(Gamma^E S);
* inertia: count(eps) = #{i : eps_i < eps}, N_infinity = 2 count (Sec. II.C,
  Sylvester's law of inertia; Sec. II.D, eq. cdos).
"""
import numpy as np
import scipy.linalg as sla

from . import fermi
from . import poles as _poles


def shifted_inverse(H, S, w):
    """(H - w S)^{-1} for complex w, by dense LU."""
    A = H.astype(np.complex128) - w * S
    return np.linalg.inv(A)


def gamma_route_a(H, S, shifts, weights):
    """Im sum_l omega_l Z_l for each weight set (dict name -> array)."""
    acc = {g: np.zeros(H.shape, dtype=np.complex128) for g in weights}
    for l, w in enumerate(shifts):
        Z = shifted_inverse(H, S, w)
        for g, om in weights.items():
            acc[g] += om[l] * Z
    return {g: np.imag(a) for g, a in acc.items()}


def gen_eigh(H, S):
    """Generalised eigenpairs (eps ascending, C with C^T S C = I)."""
    return sla.eigh(H, S)


def gamma_route_b(H, S, shifts, weights, eig=None):
    eps, C = gen_eigh(H, S) if eig is None else eig
    out = {}
    for g, om in weights.items():
        r = _poles.rational(eps, shifts, om)
        out[g] = (C * r[None, :]) @ C.T
    return out


def gamma_fermi_dirac(H, S, mu, beta, eig=None):
    """Gamma_FD and Gamma^E_FD from the eigen-decomposition."""
    eps, C = gen_eigh(H, S) if eig is None else eig
    f = fermi.fermi(eps - mu, beta)
    return (C * f[None, :]) @ C.T, (C * (eps * f)[None, :]) @ C.T


def electron_number(eps, mu, beta):
    """N_beta(mu) = sum_i f_beta(eps_i - mu)."""
    return float(np.sum(fermi.fermi(np.asarray(eps) - mu, beta)))


def traces(G, H, S):
    """Tr(G S) and Tr(G H) for symmetric G."""
    return float(np.sum(G * S)), float(np.sum(G * H))


def inertia_count(eps_sorted, shift):
    """#{i : eps_i < shift} (zero-temperature CDOS / 2)."""
    return int(np.searchsorted(np.asarray(eps_sorted), shift, side="left"))


def half_filling_mu(eps_sorted):
    """Mid-gap between the N/2-th and (N/2+1)-th eigenvalue."""
    e = np.asarray(eps_sorted)
    h = e.shape[0] // 2
    return 0.5 * (float(e[h - 1]) + float(e[h]))


def entry_error(x, y, floor_frac=1e-3):
    """Per-entry relative error |x - y| / max(|y|, floor_frac * max|y|)
    (the floor keeps near-zero entries from dominating)."""
    x = np.asarray(x)
    y = np.asarray(y)
    den = np.maximum(np.abs(y), floor_frac * np.max(np.abs(y)))
    return np.abs(x - y) / den
