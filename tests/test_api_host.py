"""Host side of the high-level entry (paper_1405_0194_amd.api): conversion
of torch / scipy / dense inputs to the lower-triangle CSC union pattern, and
the Gershgorin bound used for Delta E."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sps
import torch

from paper_1405_0194_amd import api, lattice


def _system():
    return lattice.make_system("honeycomb", (3, 2), 5, 3.0, 21)


def _full(s):
    H, S = s.dense()
    return H, S


@pytest.mark.parametrize("layout", ["dense", "scipy_csc", "torch_coo", "torch_csr", "torch_csc"])
def test_lower_csc_recovers_the_system(layout):
    s = _system()
    H, S = _full(s)
    conv = {
        "dense": lambda M: M,
        "scipy_csc": lambda M: sps.csc_matrix(M),
        "torch_coo": lambda M: torch.from_numpy(M).to_sparse(),
        "torch_csr": lambda M: torch.from_numpy(M).to_sparse_csr(),
        "torch_csc": lambda M: torch.from_numpy(M).to_sparse_csc(),
    }[layout]
    n, colptr, rowind, hval, sval = api.lower_csc(conv(H), conv(S))
    assert n == s.n
    assert np.array_equal(colptr, s.colptr) and np.array_equal(rowind, s.rowind)
    assert np.array_equal(hval, s.hval) and np.array_equal(sval, s.sval)


def test_upper_only_entries_are_mirrored_and_patterns_united():
    n = 5
    H = np.zeros((n, n))
    H[0, 3] = 0.7                   # upper only
    H[2, 1] = H[1, 2] = -0.2        # both
    np.fill_diagonal(H, [0.1, 0.2, 0.3, 0.4, 0.5])
    S = np.eye(n)
    S[4, 0] = 0.05                  # only in S, lower
    n2, colptr, rowind, hval, sval = api.lower_csc(sps.coo_matrix(H), S)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    got = {(int(r), int(c)): (h, s_) for r, c, h, s_ in zip(rowind, cols, hval, sval)}
    assert got[(3, 0)] == (0.7, 0.0)
    assert got[(2, 1)] == (-0.2, 0.0)
    assert got[(4, 0)] == (0.0, 0.05)
    assert all(got[(i, i)][1] == 1.0 for i in range(n))
    assert np.all(rowind >= cols)
    for c in range(n):
        seg = rowind[colptr[c]:colptr[c + 1]]
        assert np.all(np.diff(seg) > 0) and seg[0] == c


def test_hermitian_upper_entries_are_conjugated():
    n = 3
    H = np.diag([0.1, 0.2, 0.3]).astype(np.complex128)
    H[0, 2] = 0.3 + 0.4j            # stored above the diagonal only
    S = np.eye(n, dtype=np.complex128)
    _, colptr, rowind, hval, _ = api.lower_csc(sps.csr_matrix(H), S)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    k = np.nonzero((rowind == 2) & (cols == 0))[0][0]
    assert hval[k] == 0.3 - 0.4j


def test_spectrum_bound_contains_the_pencil_spectrum():
    for seed in (1, 2):
        s = lattice.make_system("cubic", (3, 3, 2), 4, 2.0, seed)
        H, S = s.dense()
        ev = sla.eigh(H, S, eigvals_only=True)
        b = api.spectrum_bound(s.colptr, s.rowind, s.hval, s.sval)
        assert b is not None and np.max(np.abs(ev)) <= b
    # S without diagonal dominance: no bound
    n, colptr, rowind, hval, sval = api.lower_csc(np.eye(2), np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert api.spectrum_bound(colptr, rowind, hval, sval) is None


def test_rejects_bad_shapes_and_outputs():
    with pytest.raises(ValueError):
        api.lower_csc(np.eye(3), np.eye(4))
    with pytest.raises(ValueError):
        api.Solver().density_matrix(np.eye(2), np.eye(2), 0.0, 1000.0, 4, outputs=("rho", "X"))
