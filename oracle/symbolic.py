"""Brute-force symbolic elimination (oracle; test infrastructure).

Sec. II.B: step 2 of selected inversion finds the nonzero locations of L in
A = L D L^T; the elimination tree has parent(J) = min{I > J : L_{I,J} != 0}
(eq. parent).  Here both are computed by the plainest means: symmetric
Gaussian elimination on a dense boolean matrix (no cancellation assumed).
Small patterns only.
"""
import numpy as np


def dense_pattern_from_lower_csc(n, colptr, rowind):
    P = np.zeros((n, n), dtype=bool)
    for j in range(n):
        for p in range(colptr[j], colptr[j + 1]):
            i = rowind[p]
            P[i, j] = True
            P[j, i] = True
    return P


def fill_pattern(P):
    """Lower-triangular pattern of L (incl. diagonal) for symmetric pattern
    P eliminated in natural order: eliminating column k connects every pair
    of rows that are nonzero in it below k."""
    n = P.shape[0]
    L = np.tril(P.copy())
    np.fill_diagonal(L, True)
    for k in range(n):
        rows = np.nonzero(L[k + 1:, k])[0] + k + 1
        for a in rows:
            L[a, rows[rows <= a]] = True
    return L


def etree(Lpat):
    """parent[j] = min{i > j : L[i, j]} or -1 (eq. parent, column level)."""
    n = Lpat.shape[0]
    par = np.full(n, -1, dtype=np.int64)
    for j in range(n):
        below = np.nonzero(Lpat[j + 1:, j])[0]
        if below.size:
            par[j] = j + 1 + below[0]
    return par


def permute(P, perm):
    """Pattern of A[perm][:, perm] (perm[new] = old)."""
    return P[np.ix_(perm, perm)]
