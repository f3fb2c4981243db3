"""Single columns of the inverse for systems too large for dense routines
(oracle; test infrastructure only).

Selected inversion returns entries of Z = A^{-1}, A = H - w S (Sec. II.A,
II.B).  Column j of Z solves A x = e_j; for a shift well off the real axis
A is well conditioned (every eigenvalue of the pencil is at distance at
least Im w from w), so a Krylov solve (scipy's GMRES, no preconditioner)
reaches the entries to near machine precision without any factorization.
The residual is checked before the column is returned.
"""
import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla


def matrix(n, colptr, rowind, hval, sval, w):
    """A = H - w S as a full CSR matrix from the lower triangle in CSC
    (upper entries mirrored, conjugated for complex values)."""
    cols = np.repeat(np.arange(n), np.diff(colptr))
    rows = np.asarray(rowind, dtype=np.int64)
    a = np.asarray(hval, dtype=np.complex128) - w * np.asarray(sval, dtype=np.complex128)
    at = np.conj(np.asarray(hval, dtype=np.complex128)) - w * np.conj(np.asarray(sval, dtype=np.complex128))
    off = rows != cols
    r = np.concatenate([rows, cols[off]])
    c = np.concatenate([cols, rows[off]])
    v = np.concatenate([a, at[off]])
    return sps.csr_matrix((v, (r, c)), shape=(n, n))


def inverse_column(A, j, rtol=1e-14, restart=200, maxiter=20):
    """x = A^{-1} e_j; raises if the relative residual exceeds 100 rtol."""
    n = A.shape[0]
    b = np.zeros(n, dtype=np.complex128)
    b[j] = 1.0
    x, info = spla.gmres(A, b, rtol=rtol, atol=0.0, restart=restart, maxiter=maxiter)
    res = float(np.linalg.norm(A @ x - b))
    if not res <= 100.0 * rtol:
        raise RuntimeError(f"inverse_column: residual {res:.2e} (gmres info {info})")
    return x
