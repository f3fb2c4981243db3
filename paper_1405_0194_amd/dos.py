"""Density of states and local density of states (Sec. II.D).

* DOS.  The cumulative DOS C(eps) (eq. cdos) is N_inf(eps) = 2 x #negative
  pivots of H - eps S (Sylvester's law of inertia), sampled at bin edges by
  batched real LDL^T factorizations on the device.  The DOS is its numerical
  derivative: on bin edges e_0 < ... < e_n the derivative of the linear
  interpolant of C is the bin average g_b = (C(e_{b+1}) - C(e_b)) /
  (e_{b+1} - e_b), exact for every bin (twice the number of eigenvalues in
  it, per unit energy).
* LDOS.  In the basis, G(eps) = (2/pi) Im [H - (eps + i eta) S]^{-1}
  (eqs. LDOSgreen, LDOSGreen with Im taken entrywise, eta > 0 small): one
  complex shift eps + i eta per energy, batched into one factorization and
  one selected inversion, then pole sums with weight 2/pi on each energy's
  own shift (up to four energies per pass).  Tr[G(eps) S] is the
  Lorentzian-broadened DOS.
Complex Hermitian pencils take the L D U path: counts from the signs of its
real pivots at real shifts, and G(eps) = (2/pi) (M - M^H) / 2i with
M = [H - (eps + i eta) S]^{-1}, which is the entrywise Im for real pencils.
Host orchestration only: every factorization, selected inversion and sum
runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import binding as B
from .chempot import _buffers, inertia_counts


def cdos(analysis, H, S, eps, batch=32, stream=None):
    """C(eps) = N_inf(eps) at the given energies (batches of `batch` real
    factorizations)."""
    eps = np.asarray(eps, dtype=np.float64)
    q = min(batch, max(1, len(eps)))
    L, W = _buffers(analysis, q, H, real=True)
    out = np.empty(len(eps), dtype=np.int64)
    for i in range(0, len(eps), q):
        out[i:i + q] = 2 * inertia_counts(analysis, H, S, eps[i:i + q], L=L, work=W, stream=stream)
    return out


def dos(analysis, H, S, edges, batch=32, stream=None):
    """Bin averages of the DOS on the given increasing bin edges; returns
    (bin centres, g, C at the edges)."""
    edges = np.asarray(edges, dtype=np.float64)
    if edges.ndim != 1 or len(edges) < 2 or np.any(np.diff(edges) <= 0):
        raise ValueError("edges must be an increasing 1-D array of at least two energies")
    c = cdos(analysis, H, S, edges, batch=batch, stream=stream)
    return 0.5 * (edges[1:] + edges[:-1]), np.diff(c) / np.diff(edges), c


def ldos(analysis, H, S, energies, eta, stream=None):
    """G(eps_j) on the lower pattern for each energy; returns
    (out: (m, nnz_lower) tensor, float64, complex128 for Hermitian input;
    traces: (m, 2) with Tr[G S] and Tr[G H]; info)."""
    import torch
    energies = np.asarray(energies, dtype=np.float64)
    if eta <= 0:
        raise ValueError("eta must be positive")
    m = len(energies)
    shifts = energies + 1j * eta
    herm = H.is_complex()
    F = B.HermitianFactorization if herm else B.Factorization
    f = F(analysis, H, S, shifts, stream=stream)
    f.selinv(stream=stream)
    nnz = analysis.info["nnz_lower"]
    out = torch.empty((m, nnz), dtype=torch.complex128 if herm else torch.float64, device=H.device)
    traces = np.zeros((m, 2))
    for g0 in range(0, m, 4):
        g1 = min(m, g0 + 4)
        w = np.zeros((g1 - g0, m), dtype=np.complex128)
        for g in range(g0, g1):
            w[g - g0, g] = 2.0 / np.pi
        o, tr = f.pole_sum(w, stream=stream)
        out[g0:g1].copy_(o)
        traces[g0:g1] = tr
    info = f.info
    del f
    return out, traces, info
