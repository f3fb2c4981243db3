"""Seeded synthetic H/S pencils on atom lattices.

This module only builds inputs: atom positions, neighbour lists and the
values of H and S on their sparsity pattern.  It holds none of the method's
arithmetic and imports neither the oracle nor the compiled library, so both
sides of every parity test consume exactly the same arrays.

The paper's own systems (DNA, C-BN, water, Al, SiH; Sec. III, Tables
"tab:system" and "tab:exampleFeatures") need SIESTA and DZP basis sets,
which are not available.  These lattices stand in for them: a 1D open chain
(quasi-1D like DNA), a periodic honeycomb sheet (quasi-2D like C-BN) and a
periodic simple-cubic bulk (3D like water/Al), each atom carrying ``orb``
orbitals (13 as for the DZP basis of C/N/B/O/P).

Recipe (one draw sequence per system, ``numpy.random.default_rng(seed)``):
  * pairs (I, J), I <= J, within the Euclidean cutoff (nearest-neighbour
    units, minimum image on periodic axes), in lexicographic order; for each
    pair an ``orb x orb`` standard-normal block for H, then one for S;
  * H block = G * exp(-d_IJ); on-site blocks (G + G^T)/2; H_JI = H_IJ^T;
    then H is divided by its largest absolute row sum, so spec(H) in [-1, 1];
  * S off-diagonal entries = 0.1 * G * exp(-d_IJ) (the on-site block keeps
    only its symmetrised off-diagonal part); S_ii = 1 + sum_{j != i} |S_ij|,
    so S is strictly diagonally dominant with lambda_min(S) >= 1;
  * hence every eigenvalue of the pencil (H, S) lies in [-1, 1] and
    Delta E = 1 + |mu| bounds the spectrum width about mu.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Boltzmann constant in Hartree per Kelvin (CODATA 2018).
KB_HARTREE_PER_K = 3.166811563e-6


def beta_for_temperature(T_kelvin: float) -> float:
    """Inverse temperature beta = 1/(k_B T) in 1/Hartree."""
    return 1.0 / (KB_HARTREE_PER_K * T_kelvin)


@dataclasses.dataclass
class System:
    """A sparse symmetric pencil (H, S) stored as its lower triangle in CSC.

    colptr (int64, n+1), rowind (int32, nnz): 0-based, rows sorted within a
    column, diagonal included, row >= column.  hval/sval (float64, nnz) are
    aligned with rowind.  blkptr (int32, natoms+1) gives the orbital range of
    each atom; coords (natoms, 3) the atom positions.
    """
    kind: str
    n: int
    colptr: np.ndarray
    rowind: np.ndarray
    hval: np.ndarray
    sval: np.ndarray
    blkptr: np.ndarray
    coords: np.ndarray
    orb: int
    seed: int
    meta: dict

    @property
    def nnz_lower(self) -> int:
        return int(self.rowind.shape[0])

    def dense(self):
        """Dense H and S (real symmetric, or complex Hermitian when the values
        are complex: the upper triangle is the conjugate of the lower), for
        small systems only."""
        n = self.n
        H = np.zeros((n, n), dtype=self.hval.dtype)
        S = np.zeros((n, n), dtype=self.sval.dtype)
        cols = np.repeat(np.arange(n), np.diff(self.colptr))
        H[cols, self.rowind] = np.conj(self.hval)
        S[cols, self.rowind] = np.conj(self.sval)
        H[self.rowind, cols] = self.hval
        S[self.rowind, cols] = self.sval
        return H, S

    @property
    def hermitian(self) -> bool:
        return np.iscomplexobj(self.hval)

    def entry_cols(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.colptr))


# --------------------------------------------------------------------------
# lattices
# --------------------------------------------------------------------------

def _chain(natoms):
    coords = np.zeros((natoms, 3))
    coords[:, 0] = np.arange(natoms, dtype=np.float64)
    return coords, np.zeros(3), np.array([False, False, False])


def _honeycomb(nx, ny):
    # nearest-neighbour distance 1; lattice vectors a1, a2 of length sqrt(3)
    a1 = np.array([math.sqrt(3.0), 0.0, 0.0])
    a2 = np.array([math.sqrt(3.0) / 2.0, 1.5, 0.0])
    basis = [np.zeros(3), np.array([0.0, 1.0, 0.0])]
    pts = []
    for j in range(ny):
        for i in range(nx):
            o = i * a1 + j * a2
            for b in basis:
                pts.append(o + b)
    return np.array(pts), (a1, a2), None


def _cubic(nx, ny, nz):
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij"), axis=-1).reshape(-1, 3)
    # order atoms x fastest
    g = g[np.lexsort((g[:, 0], g[:, 1], g[:, 2]))]
    return g.astype(np.float64), None, None


def _pairs_within(coords, cutoff, cell_vectors, periodic_flags):
    """All pairs (I <= J) with minimum-image distance <= cutoff.

    cell_vectors: list of supercell translation vectors for periodic axes.
    Returns (I, J, d) sorted lexicographically by (I, J).
    """
    nat = coords.shape[0]
    tol = 1e-9
    shifts = [np.zeros(3)]
    if cell_vectors:
        import itertools
        rng1 = (-1, 0, 1)
        shifts = []
        for c in itertools.product(rng1, repeat=len(cell_vectors)):
            s = np.zeros(3)
            for ci, v in zip(c, cell_vectors):
                s = s + ci * v
            shifts.append(s)
    # coarse spatial hashing with cell size = cutoff
    I_all, J_all, D_all = [], [], []
    block = 2048
    for i0 in range(0, nat, block):
        ci = coords[i0:i0 + block]
        best = np.full((ci.shape[0], nat), np.inf)
        for s in shifts:
            d = np.linalg.norm(ci[:, None, :] - (coords[None, :, :] + s[None, None, :]), axis=-1)
            best = np.minimum(best, d)
        ii, jj = np.nonzero(best <= cutoff + tol)
        ii = ii + i0
        keep = ii <= jj
        I_all.append(ii[keep])
        J_all.append(jj[keep])
        D_all.append(best[ii[keep] - i0, jj[keep]])
    I = np.concatenate(I_all)
    J = np.concatenate(J_all)
    D = np.concatenate(D_all)
    order = np.lexsort((J, I))
    return I[order], J[order], D[order]


def make_system(kind: str, dims, orb: int, cutoff: float, seed: int,
                periodic: bool = True, dilute: float = 0.0) -> System:
    """Build one synthetic pencil.

    kind: "chain" (dims = natoms, open ends), "honeycomb" (dims = (nx, ny)
    cells of 2 atoms) or "cubic" (dims = (nx, ny, nz)).  ``periodic`` applies
    to honeycomb/cubic; an axis with fewer than 5 cells is left open.
    ``dilute`` removes that fraction of the off-site pairs (drawn after the
    blocks, so the other draws do not change), which gives systems of the
    same size distinct sparsity patterns.
    """
    if kind == "chain":
        nat = int(dims)
        coords, _, _ = _chain(nat)
        cellv = []
    elif kind == "honeycomb":
        nx, ny = dims
        coords, (a1, a2), _ = _honeycomb(nx, ny)
        cellv = []
        if periodic and nx >= 5:
            cellv.append(nx * a1)
        if periodic and ny >= 5:
            cellv.append(ny * a2)
    elif kind == "cubic":
        nx, ny, nz = dims
        coords, _, _ = _cubic(nx, ny, nz)
        cellv = []
        for k, m in enumerate((nx, ny, nz)):
            if periodic and m >= 5:
                v = np.zeros(3)
                v[k] = m
                cellv.append(v)
    else:
        raise ValueError(f"unknown lattice kind {kind!r}")

    nat = coords.shape[0]
    I, J, D = _pairs_within(coords, cutoff, cellv, None)
    npair = I.shape[0]
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((npair, 2, orb, orb))
    scale = np.exp(-D)[:, None, None]
    Hb = G[:, 0] * scale
    Sb = 0.1 * G[:, 1] * scale
    onsite = I == J
    if dilute > 0.0:
        keep = onsite | (rng.uniform(size=npair) >= dilute)
        I, J, D, Hb, Sb, onsite = I[keep], J[keep], D[keep], Hb[keep], Sb[keep], onsite[keep]
        npair = I.shape[0]
    Hb[onsite] = 0.5 * (Hb[onsite] + np.transpose(Hb[onsite], (0, 2, 1)))
    So = 0.5 * (Sb[onsite] + np.transpose(Sb[onsite], (0, 2, 1)))
    idx = np.arange(orb)
    So[:, idx, idx] = 0.0
    Sb[onsite] = So

    n = nat * orb
    # lower-triangle entries.  For a pair I < J the block (J, I) of the lower
    # triangle holds H_JI = (H_IJ)^T, i.e. entry (J*o + b, I*o + a) = Hb[a, b].
    a_idx, b_idx = np.meshgrid(idx, idx, indexing="ij")  # a row of block, b col
    rows_list, cols_list, hv_list, sv_list = [], [], [], []
    off = ~onsite
    if off.any():
        Io, Jo = I[off], J[off]
        r = Jo[:, None, None] * orb + b_idx[None]
        c = Io[:, None, None] * orb + a_idx[None]
        rows_list.append(r.ravel())
        cols_list.append(c.ravel())
        hv_list.append(Hb[off].ravel())
        sv_list.append(Sb[off].ravel())
    if onsite.any():
        Io = I[onsite]
        tri = a_idx >= b_idx  # lower part of the on-site block (row a >= col b)
        r = Io[:, None] * orb + a_idx[tri][None]
        c = Io[:, None] * orb + b_idx[tri][None]
        rows_list.append(r.ravel())
        cols_list.append(c.ravel())
        hv_list.append(Hb[onsite][:, tri].ravel())
        sv_list.append(Sb[onsite][:, tri].ravel())
    rows = np.concatenate(rows_list).astype(np.int64)
    cols = np.concatenate(cols_list).astype(np.int64)
    hv = np.concatenate(hv_list)
    sv = np.concatenate(sv_list)
    order = np.lexsort((rows, cols))
    rows, cols, hv, sv = rows[order], cols[order], hv[order], sv[order]
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr)

    # Gershgorin normalisation of H (absolute row sums of the full matrix)
    absrow = np.zeros(n)
    np.add.at(absrow, rows, np.abs(hv))
    offd = rows != cols
    np.add.at(absrow, cols[offd], np.abs(hv[offd]))
    hv = hv / absrow.max()
    # diagonal dominance of S
    srow = np.zeros(n)
    np.add.at(srow, rows[offd], np.abs(sv[offd]))
    np.add.at(srow, cols[offd], np.abs(sv[offd]))
    diag = ~offd
    sv = sv.copy()
    sv[diag] = 1.0 + srow[rows[diag]]

    blkptr = (np.arange(nat + 1) * orb).astype(np.int32)
    return System(kind=kind, n=n, colptr=colptr, rowind=rows.astype(np.int32),
                  hval=hv, sval=sv, blkptr=blkptr, coords=coords, orb=orb,
                  seed=seed, meta=dict(dims=dims, cutoff=cutoff, npairs=int(npair),
                                       periodic_axes=len(cellv)))


def make_hermitian_system(kind: str, dims, orb: int, cutoff: float, seed: int,
                          periodic: bool = True, dilute: float = 0.0, imag_scale: float = 0.5) -> System:
    """A complex Hermitian pencil on the same lattice and pattern as
    make_system: every stored (lower) entry gets an imaginary part
    imag_scale * N(0,1) * |real part| (diagonal entries stay real), drawn from
    a second stream seeded with seed + 1; then H is rescaled by its largest
    absolute row sum and S is made diagonally dominant again, so the pencil's
    spectrum stays inside [-1, 1] and S is Hermitian positive definite.
    Stands in for k-point Hamiltonians (Bloch phases make H complex)."""
    base = make_system(kind, dims, orb, cutoff, seed, periodic=periodic, dilute=dilute)
    rng = np.random.default_rng(seed + 1)
    rows = base.rowind.astype(np.int64)
    cols = base.entry_cols()
    offd = rows != cols
    hv = base.hval.astype(np.complex128)
    sv = base.sval.astype(np.complex128)
    g = rng.standard_normal((2, rows.shape[0]))
    hv[offd] += 1j * imag_scale * g[0][offd] * np.abs(base.hval[offd])
    sv[offd] += 1j * imag_scale * g[1][offd] * np.abs(base.sval[offd])
    n = base.n
    absrow = np.zeros(n)
    np.add.at(absrow, rows, np.abs(hv))
    np.add.at(absrow, cols[offd], np.abs(hv[offd]))
    hv = hv / absrow.max()
    srow = np.zeros(n)
    np.add.at(srow, rows[offd], np.abs(sv[offd]))
    np.add.at(srow, cols[offd], np.abs(sv[offd]))
    diag = ~offd
    sv[diag] = 1.0 + srow[rows[diag]]
    meta = dict(base.meta, hermitian=True, imag_scale=imag_scale)
    return dataclasses.replace(base, hval=hv, sval=sv, meta=meta)


def _abs_row_sum_max(colptr, rowind, v):
    """Largest absolute row sum of the symmetric matrix whose lower triangle
    (CSC) holds v."""
    n = colptr.shape[0] - 1
    cols = np.repeat(np.arange(n), np.diff(colptr))
    rows = rowind.astype(np.int64)
    absrow = np.zeros(n)
    np.add.at(absrow, rows, np.abs(v))
    offd = rows != cols
    np.add.at(absrow, cols[offd], np.abs(v[offd]))
    return float(absrow.max())


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

BETA_300K = beta_for_temperature(300.0)
CONFIG_SEED_BASE = 14050194


def config_system(k: int) -> System:
    """The single-system workloads (0: 1D chain N=256; 1: honeycomb
    N=26,624; 2: simple cubic N=22,464)."""
    seed = CONFIG_SEED_BASE + k
    if k == 0:
        return make_system("chain", 64, 4, 2.0, seed)
    if k == 1:
        return make_system("honeycomb", (32, 32), 13, 3.0, seed)
    if k == 2:
        return make_system("cubic", (12, 12, 12), 13, 2.0, seed)
    raise ValueError(k)


CONFIG_POLES = {0: 40, 1: 60, 2: 80}


def _dims_for(kind, n_target):
    if kind == "chain":
        return max(4, int(round(n_target / 4))), 4, 2.0
    if kind == "honeycomb":
        cells = max(1, int(round(n_target / 26.0)))
        nx = max(2, int(round(math.sqrt(cells))))
        ny = max(2, int(round(cells / nx)))
        return (nx, ny), 13, 3.0
    side = max(2, int(round((n_target / 13.0) ** (1.0 / 3.0))))
    nz = max(2, int(round(n_target / 13.0 / side / side)))
    return (side, side, nz), 13, 2.0


def batch_systems(count: int = 64, seed: int = CONFIG_SEED_BASE + 3,
                  n_lo: float = 500.0, n_hi: float = 8000.0, only=None):
    """The uneven batch: kind = s mod 3 (chain / honeycomb / cubic), target
    size log-uniform in [n_lo, n_hi], pole count uniform in [40, 80] (even).
    only: indices of the systems to build (the others are drawn but not
    built, so a subset equals the same systems of the whole batch)."""
    rng = np.random.default_rng(seed)
    out = []
    kinds = ("chain", "honeycomb", "cubic")
    for s in range(count):
        kind = kinds[s % 3]
        n_t = math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))
        P = 2 * int(rng.integers(20, 41))
        if only is not None and s not in only:
            continue
        dims, orb, cut = _dims_for(kind, n_t)
        out.append((make_system(kind, dims, orb, cut, seed * 1000 + s), P))
    return out


def serving_requests(count: int, seed: int = CONFIG_SEED_BASE + 4,
                     kmax: int = 40, zipf_a: float = 1.2, repeat_frac: float = 0.3,
                     size_unit: float = 1000.0):
    """Request stream: size class k in 1..kmax with P(k) ~ k^-a, N ~ unit*k,
    kind uniform; a fraction repeats one of the last 8 patterns with H
    perturbed by 1e-3 same-pattern noise (an SCF-like repeat).  Yields dicts
    with the system, mu, a repeat flag and, for new patterns, 16 real shifts
    for an inertia count in [mu - 0.1, mu + 0.1]."""
    rng = np.random.default_rng(seed)
    ks = np.arange(1, kmax + 1, dtype=np.float64)
    pk = ks ** (-zipf_a)
    pk /= pk.sum()
    kinds = ("chain", "honeycomb", "cubic")
    recent = []
    reqs = []
    for r in range(count):
        mu = float(rng.uniform(-0.05, 0.05))
        if recent and rng.uniform() < repeat_frac:
            base = recent[int(rng.integers(0, len(recent)))]
            noise = rng.standard_normal(base.hval.shape[0]) * 1e-3
            hv = base.hval + noise * np.abs(base.hval).max()
            hv = hv / _abs_row_sum_max(base.colptr, base.rowind, hv)
            sys_r = dataclasses.replace(base, hval=hv)
            reqs.append(dict(system=sys_r, mu=mu, repeat=True, eps=None))
        else:
            k = int(rng.choice(len(ks), p=pk)) + 1
            kind = kinds[int(rng.integers(0, 3))]
            dims, orb, cut = _dims_for(kind, size_unit * k)
            s = make_system(kind, dims, orb, cut, seed * 100000 + r, dilute=0.02)
            recent.append(s)
            recent = recent[-8:]
            eps = np.sort(rng.uniform(mu - 0.1, mu + 0.1, size=16))
            reqs.append(dict(system=s, mu=mu, repeat=False, eps=eps))
    return reqs
