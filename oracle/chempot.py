"""Chemical potential search (oracle; test infrastructure only).

Follows Sec. II.C in the paper's order:
  1. N_e = N_beta(mu) = Tr[Gamma S], non-decreasing in mu (eq. Nmu).
  2. N'_beta(mu) = Tr[Gamma^d S] with Gamma^d from the derivative weights on
     the same poles; Newton's method with bisection as the safeguard.
  3. N_inf(eps) = count of eigenvalues below eps (times 2 for spin), from an
     LDL^T inertia count; here from the eigenvalues directly.
  4. N_beta(mu) = -int f'_beta(eps - mu) N_inf(eps) d eps (integration by
     parts), from Q samples of N_inf.  Reading: N_inf is interpolated
     linearly between samples and held constant outside them, and f here is
     the per-spin occupation 1/(1 + e^{beta x}) since N_inf already carries
     the factor 2.
  5. Roots N_beta(eps_l) = N_e - dN and N_beta(eps_h) = N_e + dN (band-edge
     estimates), mu = (eps_l + eps_h)/2; the interval is narrowed and the
     sampling repeated.  Reading: the next interval is [eps_l - h, eps_h + h]
     with h the sample spacing; an interval whose end samples do not bracket
     N_e -+ dN is first widened by its own width on the failing side.
The exact answer of the Newton stage is the root of N_P(mu) = N_e, where
N_P(mu) = sum_i r^rho(eps_i; mu) uses the pole expansion (what the method
evaluates), found here by Brent's method on the eigenvalues.
"""
import numpy as np
from scipy.optimize import brentq

from . import poles


def _fermi1(x, beta):
    """Per-spin occupation 1/(1 + e^{beta x})."""
    return 0.5 * (1.0 - np.tanh(0.5 * beta * np.asarray(x, dtype=np.float64)))


def _int_fermi1(x, beta):
    """Antiderivative of the per-spin occupation that vanishes at +inf:
    G(x) = x - (1/beta) ln(1 + e^{beta x}) = -(1/beta) ln(1 + e^{-beta x})."""
    x = np.asarray(x, dtype=np.float64)
    bx = beta * x
    return np.where(bx > 0, -np.log1p(np.exp(-np.abs(bx))) / beta,
                    x - np.log1p(np.exp(-np.abs(bx))) / beta)


def n_beta_from_samples(eps, ninf, mu, beta):
    """Step 4, segment by segment:
    N = N_1 (1 - f(e_1 - mu)) + N_Q f(e_Q - mu)
        + sum_s ( [-f(e - mu) N(e)]_{e_s}^{e_s+1} + g_s [G(e - mu)]_{e_s}^{e_s+1} ),
    g_s the slope of the linear interpolant on segment s."""
    eps = np.asarray(eps, dtype=np.float64)
    ninf = np.asarray(ninf, dtype=np.float64)
    total = ninf[0] * (1.0 - _fermi1(eps[0] - mu, beta)) + ninf[-1] * _fermi1(eps[-1] - mu, beta)
    for s in range(len(eps) - 1):
        a, b = eps[s], eps[s + 1]
        na, nb = ninf[s], ninf[s + 1]
        g = (nb - na) / (b - a)
        total += -_fermi1(b - mu, beta) * nb + _fermi1(a - mu, beta) * na
        total += g * (_int_fermi1(b - mu, beta) - _int_fermi1(a - mu, beta))
    return float(total)


def _bisect_increasing(fn, a, b, target, iters=200):
    for _ in range(iters):
        m = 0.5 * (a + b)
        if m == a or m == b:
            break
        if fn(m) >= target:
            b = m
        else:
            a = m
    return 0.5 * (a + b)


def bracket(count_fn, Ne, lo, hi, beta, Q=16, dN=0.1, rounds=3, max_expand=30):
    """Step 5 repeated `rounds` times (plus any widening); returns
    (lo, hi, mu, list of (eps samples, N_inf samples))."""
    samples = []
    mu = 0.5 * (lo + hi)
    r = 0
    widen = 0
    while r < rounds:
        e = np.linspace(lo, hi, Q)
        n = 2.0 * np.asarray(count_fn(e), dtype=np.float64)
        samples.append((e, n))
        low_bad = n[0] > Ne - dN
        high_bad = n[-1] < Ne + dN
        if low_bad or high_bad:
            widen += 1
            if widen > max_expand:
                raise RuntimeError("no bracket")
            w = hi - lo
            lo, hi = (lo - w if low_bad else lo), (hi + w if high_bad else hi)
            continue
        el = _bisect_increasing(lambda x: n_beta_from_samples(e, n, x, beta), e[0], e[-1], Ne - dN)
        eh = _bisect_increasing(lambda x: n_beta_from_samples(e, n, x, beta), e[0], e[-1], Ne + dN)
        mu = 0.5 * (el + eh)
        h = e[1] - e[0]
        lo, hi = el - h, eh + h
        r += 1
    return lo, hi, mu, samples


def counts_from_eigenvalues(eig_sorted):
    """Step 3 from the spectrum: eps -> #{i : eps_i < eps}."""
    ev = np.asarray(eig_sorted)
    return lambda e: np.searchsorted(ev, np.asarray(e), side="left")


def n_pole(eig, mu, beta, P, spectrum):
    """N_P(mu) = sum_i r^rho(eps_i) with the pole table at mu (what
    Tr[Gamma S] evaluates to exactly), and sum_i r^d(eps_i) (= Tr[Gamma^d S])."""
    dE = max(abs(spectrum[0] - mu), abs(spectrum[1] - mu))
    sh, w = poles.pole_table(beta, dE, mu, P, sets=("rho", "d"))
    return (float(poles.rational(eig, sh, w["rho"]).sum()), float(poles.rational(eig, sh, w["d"]).sum()))


def mu_exact(eig, Ne, beta, P, spectrum, lo, hi, xtol=1e-14):
    """Root of N_P(mu) = Ne in [lo, hi] (Brent)."""
    return brentq(lambda m: n_pole(eig, m, beta, P, spectrum)[0] - Ne, lo, hi, xtol=xtol, rtol=1e-15,
                  maxiter=500)
