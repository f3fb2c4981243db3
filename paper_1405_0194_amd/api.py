"""Density matrices of sparse pencils given as ordinary sparse matrices.

    G, GE, tr = density_matrix(H, S, mu, beta, P, outputs=("rho", "E"))

H and S are torch sparse tensors (COO, CSR or CSC, on any device), scipy
sparse matrices or dense arrays; real symmetric, or complex Hermitian (then
the path is the L D U factorization and two-sided selected inversion and the
results are complex).  Only their lower triangles are read: an entry given in
one triangle only is mirrored (conjugated for complex input).  The union of
the two patterns is the pattern of the problem (Sec. II.B: the selected
elements are those of H and S).

This module marshals data: it converts the input once per call to the lower
triangle in CSC, keeps one symbolic analysis per pattern (the analysis is
reused across SCF steps, Sec. II.B) with its factor and workspace buffers,
and returns the pole-expanded matrices (eqs. gammapole, gammaF) as torch
sparse CSC tensors of the lower triangle on the device, with the traces
Tr(G S), Tr(G H) (eq. Nmu and the band energy), Tr(G^E S), the free energy
Tr(G^F S) + mu N and N'(mu) = Tr(G^d S) (Sec. II.C) for the sets asked for.
Every numerical step runs in the HIP library.
"""
import contextlib
import hashlib

import numpy as np

from . import binding as B

SETS = ("rho", "E", "F", "d")


def _as_coo(M):
    """(n, rows, cols, values) of a square matrix on the host."""
    import scipy.sparse as sp
    try:
        import torch
    except ImportError:          # pragma: no cover
        torch = None
    if torch is not None and isinstance(M, torch.Tensor):
        if M.layout in (torch.sparse_csr, torch.sparse_csc, torch.sparse_bsr, torch.sparse_bsc):
            M = M.to_sparse_coo()
        if M.layout == torch.sparse_coo:
            M = M.coalesce()
            idx = M.indices().cpu().numpy()
            vals = M.values().cpu().numpy()
            return int(M.shape[0]), idx[0].astype(np.int64), idx[1].astype(np.int64), vals, tuple(M.shape)
        M = M.cpu().numpy()
    if sp.issparse(M):
        c = M.tocoo()
        c.sum_duplicates()
        return int(c.shape[0]), c.row.astype(np.int64), c.col.astype(np.int64), c.data, c.shape
    a = np.asarray(M)
    r, c = np.nonzero(a)
    return int(a.shape[0]), r.astype(np.int64), c.astype(np.int64), a[r, c], a.shape


def lower_csc(H, S):
    """(n, colptr int64, rowind int32, hval, sval): the lower triangle of
    pattern(H) U pattern(S) in CSC (rows sorted, diagonal included), values
    aligned with it (zero where a matrix has no entry).  Lower entries win;
    an entry present only above the diagonal is mirrored, conjugated when the
    values are complex."""
    nh, rh, ch, vh, shape_h = _as_coo(H)
    ns, rs, cs, vs, shape_s = _as_coo(S)
    if shape_h[0] != shape_h[1] or tuple(shape_h) != tuple(shape_s):
        raise ValueError(f"H and S must be square of one size, got {shape_h} and {shape_s}")
    n = nh
    cplx = np.iscomplexobj(vh) or np.iscomplexobj(vs)
    dt = np.complex128 if cplx else np.float64

    def lower_keyed(r, c, v):
        v = np.asarray(v, dtype=dt)
        lo = r >= c
        key_lo = c[lo] * n + r[lo]                       # column-major key of (r, c), r >= c
        up = ~lo
        key_up = r[up] * n + c[up]                       # (c, r) mirrored below
        v_up = np.conj(v[up]) if cplx else v[up]
        # lower entries first: np.unique keeps the first occurrence
        keys = np.concatenate([key_lo, key_up])
        vals = np.concatenate([v[lo], v_up])
        k, first = np.unique(keys, return_index=True)
        return k, vals[first]

    kh, vh2 = lower_keyed(rh, ch, vh)
    ks, vs2 = lower_keyed(rs, cs, vs)
    keys = np.union1d(kh, ks)
    diag = np.arange(n, dtype=np.int64) * (n + 1)
    keys = np.union1d(keys, diag)                        # the diagonal is always stored
    hval = np.zeros(keys.shape[0], dtype=dt)
    sval = np.zeros(keys.shape[0], dtype=dt)
    hval[np.searchsorted(keys, kh)] = vh2
    sval[np.searchsorted(keys, ks)] = vs2
    cols = keys // n
    rows = keys % n
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr)
    return n, colptr, rows.astype(np.int32), hval, sval


def spectrum_bound(colptr, rowind, hval, sval):
    """A bound on max |eps| over the pencil's eigenvalues, from Gershgorin:
    ||H||_2 <= max_i sum_j |H_ij| and lambda_min(S) >= min_i (S_ii - sum_{j != i} |S_ij|).
    None when S is not strictly diagonally dominant."""
    n = colptr.shape[0] - 1
    cols = np.repeat(np.arange(n), np.diff(colptr))
    rows = rowind.astype(np.int64)
    off = rows != cols
    ah, as_ = np.abs(hval), np.abs(sval)
    hrow = np.bincount(rows, ah, minlength=n) + np.bincount(cols[off], ah[off], minlength=n)
    srow = np.bincount(rows[off], as_[off], minlength=n) + np.bincount(cols[off], as_[off], minlength=n)
    sdiag = np.zeros(n)
    sdiag[rows[~off]] = np.real(sval[~off])
    lo = float(np.min(sdiag - srow))
    if lo <= 0.0:
        return None
    return float(np.max(hrow)) / lo


def pencil_dE(colptr, rowind, hval, sval, mu):
    """Delta E of the pole table for a pencil given on its lower triangle:
    the Gershgorin bound on max |eps| plus |mu|, which bounds max |eps - mu|
    over the spectrum.  Raises ValueError when S is not strictly diagonally
    dominant (then the caller must give Delta E)."""
    bound = spectrum_bound(colptr, rowind, hval, sval)
    if bound is None:
        raise ValueError("S is not strictly diagonally dominant: pass dE, a bound on max |eps - mu|")
    return bound + abs(mu)


def _on(stream):
    """Makes stream torch's current stream for the block (None: unchanged),
    so uploads, allocations and the library's launches share one stream."""
    if stream is None:
        return contextlib.nullcontext()
    import torch
    return torch.cuda.stream(stream)


class Solver:
    """Keeps one symbolic analysis per sparsity pattern (bound to the
    device) and the last factor/workspace buffers of each; analysis options
    (leaf_cols, panel_width, ...) apply to every pattern."""

    def __init__(self, device="cuda", **analysis_options):
        self.device = device
        self.options = analysis_options
        self._cache = {}

    def _entry(self, n, colptr, rowind, blocks, coords):
        h = hashlib.sha1()
        h.update(np.int64(n).tobytes())
        h.update(colptr.tobytes())
        h.update(rowind.tobytes())
        key = h.hexdigest()
        e = self._cache.get(key)
        if e is None:
            a = B.Analysis(n, colptr, rowind, blkptr=blocks, coords=coords, **self.options)
            a.bind(self.device)
            import torch
            e = {"analysis": a, "buffers": {},
                 "colptr": torch.from_numpy(colptr).to(self.device),
                 "rowind": torch.from_numpy(rowind.astype(np.int64)).to(self.device)}
            self._cache[key] = e
        return e

    def _buffers(self, e, kind, P):
        import torch
        a = e["analysis"]
        b = e["buffers"].get(kind)
        if b is None or b[0] != P:
            e["buffers"].pop(kind, None)
            if kind == "herm":
                lb, wb = B.hermitian_sizes(a, P)
                L = torch.empty(lb, dtype=torch.uint8, device=self.device)
                W = torch.empty(wb, dtype=torch.uint8, device=self.device)
            else:
                L, W = a.buffers(P, device=self.device)
            b = (P, L, W)
            e["buffers"][kind] = b
        return b[1], b[2]

    def check_overlap(self, H, S, blocks=None, coords=None, stream=None):
        """Whether S is positive definite, as the pencil needs (Sec. II.A),
        checked on the device on the pattern of (H, S): real S by the
        inertia of S (Sylvester: the number of negative pivots of its
        L D L^T), complex Hermitian S by the pivots of its L D U, which are
        real and all positive exactly when S is.  Returns (ok, number of
        non-positive pivots, tiny-pivot column or 0)."""
        n, colptr, rowind, hval, sval = lower_csc(H, S)
        with _on(stream):
            import torch
            e = self._entry(n, colptr, rowind, blocks, coords)
            a = e["analysis"]
            Sd = torch.from_numpy(sval).to(self.device)
            Z = torch.zeros_like(Sd)
            if np.iscomplexobj(sval):
                f = B.HermitianFactorization(a, Sd, Z, np.array([0j]))
                info = int(f.info[0])
                d = f.diag(0).cpu().numpy()
                bad = int(np.sum(d.real <= 0.0))
            else:
                neg, inf = B.inertia(a, Sd, Z, np.array([0.0]))
                info, bad = int(inf[0]), int(neg[0])
        return info == 0 and bad == 0, bad, info

    def density_matrix(self, H, S, mu, beta, P, outputs=("rho", "E"), dE=None, blocks=None, coords=None,
                       stream=None, check_overlap=False):
        """Returns (*matrices in the order of `outputs`, traces dict).  Each
        matrix is a torch sparse CSC tensor of the lower triangle of the
        union pattern on the device (float64, complex128 for Hermitian
        input).  traces: N = Tr(G S), Eband = Tr(G H), and with the sets
        asked for TrES = Tr(G^E S), free_energy = Tr(G^F S) + mu N,
        dN_dmu = Tr(G^d S); info = per-shift tiny-pivot columns (0 = none).
        check_overlap runs check_overlap first and raises ValueError when S
        is not positive definite.  stream: a torch.cuda.Stream for every
        upload, allocation and launch of the call (default: the current
        stream)."""
        with _on(stream):
            return self._density_matrix(H, S, mu, beta, P, outputs, dE, blocks, coords, check_overlap)

    def _density_matrix(self, H, S, mu, beta, P, outputs, dE, blocks, coords, check_overlap):
        import torch
        outputs = tuple(outputs)
        if not outputs or any(o not in SETS for o in outputs):
            raise ValueError(f"outputs must be a non-empty subset of {SETS}")
        if check_overlap:
            ok, bad, info = self.check_overlap(H, S, blocks=blocks, coords=coords)
            if not ok:
                raise ValueError(f"S is not positive definite: {bad} non-positive pivots, tiny pivot at {info}")
        nsets = 1 + max(SETS.index(o) for o in outputs)
        n, colptr, rowind, hval, sval = lower_csc(H, S)
        herm = np.iscomplexobj(hval)
        if dE is None:
            dE = pencil_dE(colptr, rowind, hval, sval, mu)
        e = self._entry(n, colptr, rowind, blocks, coords)
        a = e["analysis"]
        Hd = torch.from_numpy(hval).to(self.device)
        Sd = torch.from_numpy(sval).to(self.device)
        if herm:
            L, W = self._buffers(e, "herm", P)
            sh, wt = B.poles(beta, dE, mu, P, nsets)
            f = B.HermitianFactorization(a, Hd, Sd, sh, L=L, work=W)
            info = f.info.copy()
            f.selinv()
            out, tr = f.pole_sum(wt)
            del f
        else:
            L, W = self._buffers(e, "real", P)
            out, tr, info, sh, wt = B.density_matrix(a, Hd, Sd, beta, dE, mu, P, nsets=nsets, L=L, work=W)
        mats = []
        for o in outputs:
            g = SETS.index(o)
            mats.append(torch.sparse_csc_tensor(e["colptr"], e["rowind"], out[g], size=(n, n)))
        N = float(tr[0, 0])
        traces = {"N": N, "Eband": float(tr[0, 1]), "dE": float(dE), "info": info}
        if nsets > 1:
            traces["TrES"] = float(tr[1, 0])
        if nsets > 2:
            traces["free_energy"] = float(tr[2, 0]) + mu * N
        if nsets > 3:
            traces["dN_dmu"] = float(tr[3, 0])
        return (*mats, traces)


_default = None


def density_matrix(H, S, mu, beta, P, outputs=("rho", "E"), dE=None, blocks=None, coords=None, stream=None,
                   check_overlap=False):
    """Solver.density_matrix on a module-level solver (device cuda)."""
    global _default
    if _default is None:
        _default = Solver()
    return _default.density_matrix(H, S, mu, beta, P, outputs=outputs, dE=dE, blocks=blocks, coords=coords,
                                   stream=stream, check_overlap=check_overlap)
