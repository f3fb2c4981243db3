"""The seeded input generator: deterministic per seed, the stated structure
(symmetric pattern with the diagonal, rows sorted), spectrum of the pencil
inside [-1, 1] with S diagonally dominant, and the configuration sizes."""
import numpy as np
import scipy.linalg as sla

from paper_1405_0194_amd import lattice


def test_same_seed_same_system_other_seed_other_values():
    a = lattice.make_system("honeycomb", (3, 3), 4, 3.0, 5)
    b = lattice.make_system("honeycomb", (3, 3), 4, 3.0, 5)
    c = lattice.make_system("honeycomb", (3, 3), 4, 3.0, 6)
    for f in ("colptr", "rowind", "hval", "sval", "blkptr", "coords"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.array_equal(a.rowind, c.rowind) and not np.array_equal(a.hval, c.hval)
    h1 = lattice.make_hermitian_system("cubic", (3, 3, 2), 4, 2.0, 9)
    h2 = lattice.make_hermitian_system("cubic", (3, 3, 2), 4, 2.0, 9)
    assert np.array_equal(h1.hval, h2.hval) and np.array_equal(h1.sval, h2.sval)


def test_structure_and_spectrum():
    for s in (lattice.make_system("chain", 20, 4, 2.0, 1), lattice.make_system("honeycomb", (4, 3), 5, 3.0, 2),
              lattice.make_system("cubic", (3, 3, 3), 3, 2.0, 3),
              lattice.make_hermitian_system("honeycomb", (3, 3), 4, 3.0, 4)):
        n = s.n
        cols = s.entry_cols()
        assert np.all(s.rowind >= cols)
        for c in range(n):
            seg = s.rowind[s.colptr[c]:s.colptr[c + 1]]
            assert seg[0] == c and np.all(np.diff(seg) > 0)
        H, S = s.dense()
        ev = sla.eigh(H, S, eigvals_only=True)
        assert ev[0] >= -1.0 and ev[-1] <= 1.0
        off = np.abs(S - np.diag(np.diag(S))).sum(axis=1)
        assert np.all(np.real(np.diag(S)) - off >= 1.0 - 1e-12)


def test_configuration_sizes():
    s = lattice.config_system(0)
    assert s.n == 256 and 2 * s.nnz_lower - s.n == 5024
