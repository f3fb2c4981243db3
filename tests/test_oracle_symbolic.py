"""Pins of the brute-force symbolic elimination (Sec. II.B steps 1-2,
eq. parent): textbook special cases and the nonzero pattern of a numeric
Cholesky factor of a random SPD matrix with the same pattern."""
import numpy as np
import scipy.linalg as sla

from oracle import symbolic


def _lower_csc(P):
    n = P.shape[0]
    colptr = [0]
    rows = []
    for j in range(n):
        r = [i for i in range(j, n) if P[i, j]]
        rows += r
        colptr.append(len(rows))
    return np.array(colptr), np.array(rows)


def test_tridiagonal_no_fill_chain_etree():
    n = 9
    P = np.eye(n, dtype=bool) | np.eye(n, k=1, dtype=bool) | np.eye(n, k=-1, dtype=bool)
    L = symbolic.fill_pattern(P)
    assert np.array_equal(L, np.tril(P))
    assert list(symbolic.etree(L)) == list(range(1, n)) + [-1]


def test_arrow_matrices():
    n = 7
    P = np.eye(n, dtype=bool)
    P[0, :] = P[:, 0] = True            # arrow at the top: full fill
    L = symbolic.fill_pattern(P)
    assert np.array_equal(L, np.tril(np.ones((n, n), dtype=bool)))
    Q = np.eye(n, dtype=bool)
    Q[-1, :] = Q[:, -1] = True          # arrow at the bottom: no fill
    L2 = symbolic.fill_pattern(Q)
    assert np.array_equal(L2, np.tril(Q))
    par = symbolic.etree(L2)
    assert list(par) == [n - 1] * (n - 1) + [-1]


def test_matches_numeric_cholesky_pattern():
    rng = np.random.default_rng(3)
    n = 30
    for trial in range(5):
        P = rng.uniform(size=(n, n)) < 0.08
        P = P | P.T | np.eye(n, dtype=bool)
        colptr, rows = _lower_csc(P)
        P2 = symbolic.dense_pattern_from_lower_csc(n, colptr, rows)
        assert np.array_equal(P, P2)
        A = np.where(P, rng.uniform(-1, 1, (n, n)), 0.0)
        A = 0.5 * (A + A.T)
        A += np.eye(n) * (np.abs(A).sum(axis=1).max() + 1.0)
        Lnum = sla.cholesky(A, lower=True)
        nz = np.abs(Lnum) > 1e-300
        L = symbolic.fill_pattern(P)
        assert np.array_equal(L, nz)
        par = symbolic.etree(L)
        for j in range(n):
            below = [i for i in range(j + 1, n) if L[i, j]]
            assert par[j] == (below[0] if below else -1)


def test_permute_is_the_permutation_similarity():
    """permute(P, perm) = Q^T P Q with Q the permutation matrix whose column
    `new` is e_perm[new] (an integer matrix product, not the oracle's
    indexing)."""
    rng = np.random.default_rng(11)
    n = 9
    P = rng.uniform(size=(n, n)) < 0.3
    P = P | P.T
    perm = rng.permutation(n)
    Q = np.zeros((n, n), dtype=np.int64)
    Q[perm, np.arange(n)] = 1
    want = (Q.T @ P.astype(np.int64) @ Q) != 0
    assert np.array_equal(symbolic.permute(P, perm), want)
    # the inverse permutation undoes it
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    assert np.array_equal(symbolic.permute(symbolic.permute(P, perm), inv), P)


def test_permute_reversed_arrow_fills_completely():
    """A bottom arrow (full last row and column) has no fill in natural
    order; reversed (perm[new] = n - 1 - new) it is a top arrow, whose first
    elimination step connects every pair, so L is completely full."""
    n = 8
    P = np.eye(n, dtype=bool)
    P[-1, :] = True
    P[:, -1] = True
    L0 = symbolic.fill_pattern(P)
    assert np.array_equal(L0, np.tril(P))
    R = symbolic.permute(P, np.arange(n)[::-1])
    assert R[0].all() and R[:, 0].all() and R[1:, 1:].sum() == n - 1
    assert np.array_equal(symbolic.fill_pattern(R), np.tril(np.ones((n, n), dtype=bool)))
