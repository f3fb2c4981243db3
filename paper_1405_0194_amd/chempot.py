"""Chemical potential: inertia-count bracketing, then safeguarded Newton.

Sec. II.C: N_e = N_beta(mu) = Tr[Gamma S] is non-decreasing in mu.
  * Bracketing.  N_inf(eps), the zero-temperature electron count below eps,
    is 2 x (number of negative pivots of H - eps S = L D L^T) by Sylvester's
    law of inertia; a batch of Q real factorizations samples it on a grid.
    Integration by parts gives N_beta(mu) = -int f'(eps - mu) N_inf(eps)
    d eps, evaluated here in closed form with N_inf interpolated linearly
    between the samples and held constant outside them.  The roots of
    N_beta = N_e -+ dN (band-edge estimates when there is a gap) give
    mu = their midpoint, and the interval narrows around them for the next
    round.  An interval that does not bracket N_e is widened first.
  * Newton.  Each iterate is one density-matrix evaluation with the weight
    sets rho and d on the same poles: N(mu) = Tr[Gamma S] and
    N'(mu) = Tr[Gamma^d S].  A step that leaves the current bracket, or a
    vanishing N', is replaced by bisection.
Host logic only: every count and trace comes from the library's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import binding as B


def _smoothed_ramp(x, beta):
    """F(x) = -(1/beta) ln(1 + exp(-beta x)); F' = 1/(1 + exp(beta x)) is
    the occupation per spin state, F(x) -> min(x, 0) as beta -> inf."""
    bx = beta * np.asarray(x, dtype=np.float64)
    return -np.logaddexp(0.0, -bx) / beta


def n_beta_from_counts(eps, n_inf, mu, beta):
    """N_beta(mu) from samples N_inf(eps_m) on an increasing grid.

    With N_inf linear on each [eps_m, eps_m+1] (slope g_m) and constant
    outside [eps_1, eps_Q], -int f'(eps - mu) N_inf(eps) d eps telescopes to
    N_inf(eps_1) + sum_m g_m [F(eps_m+1 - mu) - F(eps_m - mu)]."""
    eps = np.asarray(eps, dtype=np.float64)
    n_inf = np.asarray(n_inf, dtype=np.float64)
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    g = np.diff(n_inf) / np.diff(eps)
    F = _smoothed_ramp(eps[None, :] - mu[:, None], beta)
    out = n_inf[0] + (np.diff(F, axis=1) * g[None, :]).sum(axis=1)
    return out


def _root(fn, lo, hi, target, iters=200):
    """Bisection for fn(x) = target on [lo, hi] with fn non-decreasing."""
    a, b = lo, hi
    for _ in range(iters):
        m = 0.5 * (a + b)
        if m <= a or m >= b:
            break
        if fn(m) < target:
            a = m
        else:
            b = m
    return 0.5 * (a + b)


@dataclasses.dataclass
class Bracket:
    lo: float
    hi: float
    mu: float
    counts: int = 0            # real factorizations spent
    rounds: list = dataclasses.field(default_factory=list)


def bracket_from_counts(count_fn, Ne, lo, hi, beta, Q=16, dN=0.1, rounds=3, max_expand=30, tol=None):
    """The bracketing procedure on an arbitrary count function
    count_fn(eps array) -> #negative pivots (int array)."""
    if not hi > lo:
        raise ValueError("need lo < hi")
    if Q < 2:
        raise ValueError("need Q >= 2 samples")
    res = Bracket(lo, hi, 0.5 * (lo + hi))
    done = 0
    expand = 0
    mu_prev = None
    while done < rounds:
        eps = np.linspace(lo, hi, Q)
        ninf = 2.0 * np.asarray(count_fn(eps), dtype=np.float64)
        res.counts += Q
        width = hi - lo
        if ninf[0] > Ne - dN or ninf[-1] < Ne + dN:
            expand += 1
            if expand > max_expand:
                raise RuntimeError("could not bracket the electron count")
            if ninf[0] > Ne - dN:
                lo -= width
            if ninf[-1] < Ne + dN:
                hi += width
            res.rounds.append(dict(lo=float(eps[0]), hi=float(eps[-1]), action="widen"))
            continue

        def nb(x):
            return float(n_beta_from_counts(eps, ninf, x, beta)[0])

        el = _root(nb, eps[0], eps[-1], Ne - dN)
        eh = _root(nb, eps[0], eps[-1], Ne + dN)
        mu = 0.5 * (el + eh)
        h = eps[1] - eps[0]
        res.rounds.append(dict(lo=float(eps[0]), hi=float(eps[-1]), el=el, eh=eh, mu=mu))
        res.lo, res.hi, res.mu = el - h, eh + h, mu
        done += 1
        stop = tol is not None and mu_prev is not None and abs(mu - mu_prev) <= tol
        mu_prev = mu
        lo, hi = res.lo, res.hi
        if stop:
            break
    return res


def inertia_counts(analysis, H, S, eps, L=None, work=None, stream=None, max_retry=4):
    """#negative pivots of H - eps_q S for every q (batched real LDL^T on the
    device; for complex Hermitian H, S the batched L D U, whose pivots are
    real at real shifts).  A shift that hits a tiny pivot is moved by 1e-9
    relative and counted again (the count is piecewise constant in eps)."""
    eps = np.array(eps, dtype=np.float64)
    count = B.inertia_hermitian if H.is_complex() else B.inertia
    neg, info = count(analysis, H, S, eps, L=L, work=work, stream=stream)
    for _ in range(max_retry):
        bad = np.nonzero(info)[0]
        if not len(bad):
            break
        scale = max(1.0, float(np.abs(eps).max()))
        eps[bad] += 1e-9 * scale
        neg2, info2 = count(analysis, H, S, eps[bad], L=L, work=work, stream=stream)
        neg[bad] = neg2
        info[bad] = info2
    if np.any(info):
        raise B.PxsError("inertia_counts", B.PXS_TINY_PIVOT, "tiny pivot persists after shifting")
    return neg


def inertia_bracket(analysis, H, S, Ne, lo, hi, beta, Q=16, dN=0.1, rounds=3, tol=None, L=None, work=None,
                    stream=None, max_retry=4):
    """Bracketing with N_inf from batched inertia counts on the device
    (real LDL^T, or L D U for complex Hermitian H, S)."""
    if L is None or work is None:
        L, work = _buffers(analysis, Q, H, real=True)

    def count(eps):
        return inertia_counts(analysis, H, S, eps, L=L, work=work, stream=stream, max_retry=max_retry)

    return bracket_from_counts(count, Ne, lo, hi, beta, Q=Q, dN=dN, rounds=rounds, tol=tol)


@dataclasses.dataclass
class NewtonResult:
    mu: float
    N: float
    dN: float
    iterations: int
    lo: float
    hi: float
    history: list
    out: object = None          # (4, nnz_lower) Gamma, Gamma^E, Gamma^F, Gamma^d at the final mu
    traces: object = None       # (4, 2): Tr(G S), Tr(G H) per set


def newton_from(evaluate, Ne, mu0, lo, hi, spectrum=(-1.0, 1.0), tol_ne=1e-8, maxit=30):
    """Safeguarded Newton for N(mu) = Ne inside [lo, hi]; evaluate(mu)
    returns (N, N', payload).  Returns (mu, N, N', iterations, lo, hi,
    history, payload of the last evaluation)."""
    hist = []
    mu = float(mu0)
    if not lo <= mu <= hi:
        mu = 0.5 * (lo + hi)
    # an end of [lo, hi] is confirmed once N has been evaluated there.  While
    # the root may lie past an unconfirmed end (mu left a reused bracket) that
    # end is widened geometrically and probed; otherwise a step outside the
    # interval is replaced by bisection.  Nothing leaves the spectrum's
    # range, outside which N is constant.
    lo_ok = hi_ok = False
    smin = spectrum[0] - 1e-3 * (spectrum[1] - spectrum[0])
    smax = spectrum[1] + 1e-3 * (spectrum[1] - spectrum[0])
    grow = max(hi - lo, 1e-3 * (smax - smin))    # doubles with every widening
    payload = None
    N = dN = float("nan")
    for it in range(1, maxit + 1):
        N, dN, payload = evaluate(mu)
        hist.append(dict(mu=mu, N=N, dN=dN))
        if abs(N - Ne) <= tol_ne:
            return mu, N, dN, it, lo, hi, hist, payload
        if N < Ne:
            lo, lo_ok = mu, True
        else:
            hi, hi_ok = mu, True
        # Newton step; far from mu* the expansion of N' can be unreliable
        # (even negative), so only a positive N' gives a step
        step = mu - (N - Ne) / dN if dN > 0 else float("nan")
        if np.isfinite(step):
            step = min(max(step, smin), smax)
        probe = None
        if N < Ne and not hi_ok and not (np.isfinite(step) and step < hi):
            # mu* may lie above the guessed upper end: widen it and probe it
            hi = min(smax, hi + grow)
            grow *= 2.0
            probe = hi
        elif N > Ne and not lo_ok and not (np.isfinite(step) and step > lo):
            lo = max(smin, lo - grow)
            grow *= 2.0
            probe = lo
        if probe is not None:
            mu = probe
        elif np.isfinite(step) and lo < step < hi:
            mu = step
        else:
            mu = 0.5 * (lo + hi)
        if lo_ok and hi_ok and hi - lo <= 4 * np.finfo(float).eps * max(1.0, abs(mu)):
            break
    return mu, N, dN, len(hist), lo, hi, hist, payload


def _buffers(analysis, nshift, H, real=False):
    """Factor storage and workspace for nshift shifts of the path H takes."""
    if H.is_complex():
        import torch
        lb, wb = B.hermitian_sizes(analysis, nshift)
        return (torch.empty(lb, dtype=torch.uint8, device=H.device),
                torch.empty(wb, dtype=torch.uint8, device=H.device))
    return analysis.buffers(nshift, real=real, device=H.device)


def newton_mu(analysis, H, S, Ne, mu0, lo, hi, beta, P, spectrum=(-1.0, 1.0), tol_ne=1e-8, maxit=30,
              L=None, work=None, stream=None):
    """Newton for Tr[Gamma_P(mu) S] = Ne; every iterate is one density
    matrix (weight sets rho, E, F, d) on the device (for complex Hermitian
    H, S through the L D U path, Gamma = (M - M^H)/2i).  spectrum bounds the
    pencil's eigenvalues; Delta E = max |bound - mu|."""
    if L is None or work is None:
        L, work = _buffers(analysis, P, H)

    def evaluate(mu):
        dE = max(abs(spectrum[0] - mu), abs(spectrum[1] - mu))
        if H.is_complex():
            sh, wt = B.poles(beta, dE, mu, P, 4)
            f = B.HermitianFactorization(analysis, H, S, sh, L=L, work=work, stream=stream)
            info = f.info.copy()
            f.selinv(stream=stream)
            out, tr = f.pole_sum(wt, stream=stream)
        else:
            out, tr, info, _, _ = B.density_matrix(analysis, H, S, beta, dE, mu, P, nsets=4, L=L, work=work,
                                                   stream=stream)
        if np.any(info):
            raise B.PxsError("newton_mu", B.PXS_TINY_PIVOT, f"tiny pivot at mu={mu}")
        return float(tr[0, 0]), float(tr[3, 0]), (out, tr)

    mu, N, dN, it, lo, hi, hist, payload = newton_from(evaluate, Ne, mu0, lo, hi, spectrum, tol_ne, maxit)
    out, tr = payload if payload is not None else (None, None)
    return NewtonResult(mu, N, dN, it, lo, hi, hist, out, tr)


def solve_mu(analysis, H, S, Ne, beta, P, lo=-1.0, hi=1.0, spectrum=(-1.0, 1.0), Q=16, dN=0.1, rounds=3,
             tol_ne=1e-8, maxit=30, previous: Optional[Bracket] = None, margin=0.05, stream=None):
    """Inertia bracketing (skipped when a previous bracket is given: it is
    reused, widened by `margin`, as across SCF steps) followed by Newton
    from the bracket's mu."""
    if previous is not None:
        br = Bracket(previous.lo - margin, previous.hi + margin, previous.mu)
    else:
        br = inertia_bracket(analysis, H, S, Ne, lo, hi, beta, Q=Q, dN=dN, rounds=rounds, stream=stream)
    res = newton_mu(analysis, H, S, Ne, br.mu, br.lo, br.hi, beta, P, spectrum=spectrum, tol_ne=tol_ne,
                    maxit=maxit, stream=stream)
    return br, res
