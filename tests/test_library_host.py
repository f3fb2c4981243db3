"""Host-side checks of the C-ABI library (no GPU): the library loads and
exports every declared entry point; its pole table matches the oracle's;
its symbolic analysis contains the exact pattern of L (brute-force oracle)
and obeys eq. parent at supernode level; malformed input is rejected."""
import os
import re

import numpy as np
import pytest

from oracle import poles as opoles
from oracle import symbolic as osym
from paper_1405_0194_amd import binding as B
from paper_1405_0194_amd import lattice

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pxs_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = B.load()
    names = _declared()
    assert len(names) >= 14
    for n in sorted(names):
        assert hasattr(lib, n), n


@pytest.mark.parametrize("beta,dE,mu,P", [(lattice.BETA_300K, 2.0, 0.1, 40),
                                          (lattice.BETA_300K, 1.05, -0.05, 80),
                                          (100.0, 3.0, 0.5, 20), (5000.0, 1.0, 0.0, 60)])
def test_pole_table_matches_oracle(beta, dE, mu, P):
    sh, wt = B.poles(beta, dE, mu, P, 4)
    osh, ow = opoles.pole_table(beta, dE, mu, P)
    scale = np.abs(osh - mu).max()
    assert np.abs(sh - osh).max() <= 1e-11 * scale
    for g, name in enumerate(opoles.SETS):
        assert np.abs(wt[g] - ow[name]).max() <= 1e-11 * np.abs(ow[name]).max(), name
    assert np.all(sh.imag > 0)


def test_pole_table_rejects_bad_arguments():
    with pytest.raises(B.PxsError):
        B.poles(1000.0, 1.0, 0.0, 41)
    with pytest.raises(B.PxsError):
        B.poles(-1.0, 1.0, 0.0, 40)
    with pytest.raises(B.PxsError):
        B.poles(1000.0, 1.0, 0.0, 40, nsets=5)


def _lower_csc_from_dense(P):
    n = P.shape[0]
    colptr = [0]
    rows = []
    for j in range(n):
        r = [i for i in range(j, n) if P[i, j]]
        rows += r
        colptr.append(len(rows))
    return np.array(colptr, dtype=np.int64), np.array(rows, dtype=np.int32)


def _check_symbolic(a, Pfull):
    ex = a.export()
    n = Pfull.shape[0]
    perm = ex["perm"]
    assert sorted(perm.tolist()) == list(range(n))
    Lx = osym.fill_pattern(osym.permute(Pfull, perm))       # exact pattern, new order
    sp, rp, rows, par = ex["super_ptr"], ex["row_ptr"], ex["rows"], ex["parent"]
    ns = sp.shape[0] - 1
    owner = np.zeros(n, dtype=np.int64)
    for J in range(ns):
        owner[sp[J]:sp[J + 1]] = J
    for J in range(ns):
        E = rows[rp[J]:rp[J + 1]]
        w = sp[J + 1] - sp[J]
        assert np.array_equal(E[:w], np.arange(sp[J], sp[J + 1]))
        assert np.all(np.diff(E) > 0)
        Eset = set(E.tolist())
        for j in range(sp[J], sp[J + 1]):
            need = np.nonzero(Lx[j:, j])[0] + j
            assert set(need.tolist()) <= Eset, (J, j)
        below = E[w:]
        # eq. parent at supernode level: the owner of the first row below
        assert par[J] == (owner[below[0]] if below.size else -1)
    return Lx


@pytest.mark.parametrize("ordering", [0, 1])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_symbolic_contains_exact_pattern_random(seed, ordering):
    rng = np.random.default_rng(seed)
    n = 60
    P = rng.uniform(size=(n, n)) < 0.05
    P = P | P.T | np.eye(n, dtype=bool)
    colptr, rows = _lower_csc_from_dense(P)
    a = B.Analysis(n, colptr, rows, ordering=ordering, leaf_cols=8, panel_width=5)
    Lx = _check_symbolic(a, P)
    # without blocks the exact counts are exact at column level
    ck = Lx.sum(axis=0) - 1
    assert a.info["nnz_L_exact"] == int(Lx.sum())
    assert a.info["flops_factor"] == pytest.approx(8.0 * np.sum(ck * (ck + 1) / 2.0))
    assert a.info["flops_selinv"] == pytest.approx(8.0 * np.sum(ck * ck + ck))


def test_symbolic_chain_with_blocks_and_coords():
    s = lattice.config_system(0)
    a = B.Analysis.from_system(s, leaf_cols=16)
    P = osym.dense_pattern_from_lower_csc(s.n, s.colptr, s.rowind)
    Lx = _check_symbolic(a, P)
    assert a.info["nnz_L_exact"] == int(Lx.sum())
    assert a.info["nsuper"] > 3


def test_symbolic_small_honeycomb_graph_ordering():
    s = lattice.make_system("honeycomb", (4, 3), 3, 3.0, 5, periodic=False)
    a = B.Analysis(s.n, s.colptr, s.rowind, blkptr=s.blkptr, leaf_cols=9)
    P = osym.dense_pattern_from_lower_csc(s.n, s.colptr, s.rowind)
    Lx = _check_symbolic(a, P)
    assert a.info["nnz_L_exact"] == int(Lx.sum())


@pytest.mark.parametrize("sep_cols", [4, 9, 30])
def test_separator_pieces_keep_exact_pattern(sep_cols):
    # wide separators cut into supernodes of at most sep_cols columns: still
    # a relaxed pattern that contains the exact one, the same exact counts,
    # and no more stored entries than one supernode per separator
    s = lattice.make_system("cubic", (5, 5, 4), 2, 2.0, 11, periodic=False)
    whole = B.Analysis.from_system(s, leaf_cols=16)
    cut = B.Analysis.from_system(s, leaf_cols=16, sep_cols=sep_cols)
    P = osym.dense_pattern_from_lower_csc(s.n, s.colptr, s.rowind)
    Lx = _check_symbolic(cut, P)
    assert cut.info["nnz_L_exact"] == int(Lx.sum())
    ex = cut.export()
    widths = np.diff(ex["super_ptr"])
    assert cut.info["nsuper"] > whole.info["nsuper"]
    # a piece is wider than sep_cols only when one atom block alone is
    assert np.all((widths <= max(sep_cols, s.orb)) | (widths <= 16))
    assert cut.info["nnz_L"] <= whole.info["nnz_L"]
    assert cut.info["bytes_per_shift"] <= whole.info["bytes_per_shift"]
    ck = Lx.sum(axis=0) - 1                 # exact counts of the cut ordering
    assert cut.info["flops_factor"] == pytest.approx(8.0 * np.sum(ck * (ck + 1) / 2.0))
    assert cut.info["flops_selinv"] == pytest.approx(8.0 * np.sum(ck * ck + ck))
    assert sum(cut.info["macs_exact"]) == pytest.approx(
        (cut.info["flops_factor"] + cut.info["flops_selinv"]) / 8.0, rel=1e-12)


def test_negative_separator_width_rejected():
    s = lattice.make_system("cubic", (3, 3, 3), 1, 1.0, 2, periodic=False)
    with pytest.raises(B.PxsError):
        B.Analysis.from_system(s, sep_cols=-1)


def test_nested_dissection_reduces_fill_on_grid():
    # 2D grid: nested dissection must beat the natural (banded) order
    s = lattice.make_system("cubic", (16, 16, 1), 1, 1.0, 9, periodic=False)
    nd = B.Analysis.from_system(s, leaf_cols=8)
    nat = B.Analysis.from_system(s, ordering=1)
    assert nd.info["nnz_L_exact"] < nat.info["nnz_L_exact"]
    assert nd.info["flops_factor"] < nat.info["flops_factor"]


def test_fill_growth_slopes_1d_2d_3d():
    # Sec. II.A: nnz(L) grows like N (1D), N^1.5 (2D), N^2 (3D) -- check
    # that the measured log-log slopes are ordered and near those values
    def slope(kind, dims_list, orb):
        xs, ys = [], []
        for d in dims_list:
            s = lattice.make_system(kind, d, orb, 1.0 if kind != "chain" else 1.0, 3, periodic=False)
            a = B.Analysis.from_system(s, leaf_cols=8)
            xs.append(np.log(s.n))
            ys.append(np.log(a.info["nnz_L_exact"]))
        return np.polyfit(xs, ys, 1)[0]
    s1 = slope("chain", [200, 400, 800, 1600], 1)
    s2 = slope("cubic", [(12, 12, 1), (24, 24, 1), (48, 48, 1)], 1)
    s3 = slope("cubic", [(6, 6, 6), (9, 9, 9), (12, 12, 12)], 1)
    assert 0.9 < s1 < 1.15
    assert 1.1 < s2 < 1.6
    assert 1.4 < s3 < 2.1
    assert s1 < s2 < s3


@pytest.mark.parametrize("bad", ["unsorted", "nodiag", "upper", "range"])
def test_analyze_rejects_malformed_csc(bad):
    colptr = np.array([0, 2, 4, 5], dtype=np.int64)
    rows = np.array([0, 2, 1, 2, 2], dtype=np.int32)
    if bad == "unsorted":
        rows = np.array([0, 2, 2, 1, 2], dtype=np.int32)
    elif bad == "nodiag":
        rows = np.array([1, 2, 1, 2, 2], dtype=np.int32)
    elif bad == "upper":
        rows = np.array([0, 2, 0, 1, 2], dtype=np.int32)
    elif bad == "range":
        rows = np.array([0, 3, 1, 2, 2], dtype=np.int32)
    with pytest.raises(B.PxsError) as ei:
        B.Analysis(3, colptr, rows)
    assert ei.value.code == B.PXS_EINVAL


def test_analyze_rejects_bad_blocks():
    colptr = np.array([0, 1, 2, 3], dtype=np.int64)
    rows = np.array([0, 1, 2], dtype=np.int32)
    with pytest.raises(B.PxsError):
        B.Analysis(3, colptr, rows, blkptr=np.array([0, 2, 2, 3]))
    with pytest.raises(B.PxsError):
        B.Analysis(3, colptr, rows, blkptr=np.array([0, 1, 4]))


def test_profile_rejects_bad_class_and_unopened_profile():
    lib = B.load()
    assert lib.pxs_profile_begin(0) == B.PXS_EINVAL
    assert lib.pxs_profile_begin(10) == B.PXS_EINVAL
    with pytest.raises(B.PxsError):
        B.profile_end()
    # an open profile with no launches closes cleanly (no device work)
    B.profile_begin("gather")
    ms, n, w, b = B.profile_end(with_bytes=True)
    assert (ms, n, w, b) == (0.0, 0, 0.0, 0.0)
    with pytest.raises(B.PxsError):
        B.profile_end()


def test_empty_and_oversized_inputs_rejected():
    lib = B.load()
    # an empty matrix
    with pytest.raises(B.PxsError) as ei:
        B.Analysis(0, np.array([0]), np.array([], dtype=np.int32))
    assert ei.value.code == B.PXS_EINVAL
    a = B.Analysis(3, np.array([0, 2, 3, 4]), np.array([0, 1, 1, 2], dtype=np.int32))
    # batch sizes outside 1..4096 shifts
    import ctypes as C
    b = C.c_int64()
    for nshift in (0, -1, 4097):
        assert lib.pxs_workspace_size(a._h, nshift, 0, C.byref(b)) == B.PXS_EINVAL
    assert lib.pxs_workspace_size(a._h, 4096, 0, C.byref(b)) == B.PXS_OK
    # the fused call checks the pole count before touching any buffer
    for P, nsets in ((4098, 2), (3, 2), (0, 2), (40, 0), (40, 5)):
        code = lib.pxs_density_matrix(a._h, None, None, 1000.0, 1.0, 0.0, P, nsets, None, None, None,
                                      None, None, None, None, None)
        assert code == B.PXS_EINVAL, (P, nsets)


def _exact_macs_by_class(a, Lx, pw):
    """Brute force: the multiply-adds of every column on the exact pattern
    (boolean elimination) split by the kernel that performs them, for
    panels of pw columns inside the exported supernodes."""
    ex = a.export()
    sp = ex["super_ptr"]
    n = Lx.shape[0]
    got = np.zeros(8)
    owner = np.zeros(n, dtype=np.int64)
    for J in range(sp.shape[0] - 1):
        owner[sp[J]:sp[J + 1]] = J
    for k in range(n):
        rows = np.nonzero(Lx[k + 1:, k])[0] + k + 1
        J = owner[k]
        s0, s1 = sp[J], sp[J + 1]
        fe = min(s0 + ((k - s0) // pw + 1) * pw, s1)
        a_ = np.sum(rows < fe)
        g = np.sum((rows >= fe) & (rows < s1))
        e = np.sum(rows >= s1)
        b = g + e
        got[6] += a_ * (a_ + 1) / 2      # diagonal block
        got[3] += a_ * b                 # TRSM
        got[1] += g * (g + 1) / 2 + g * e + e * (e + 1) / 2   # updates
        got[2] += b * b                  # SelInv Z_BB L-hat
        got[4] += 2 * a_ * b             # SelInv diagonal partials
        got[0] += a_ * a_ + a_ + b       # SelInv diagonal block in LDS
    return got


@pytest.mark.parametrize("seed,pw", [(1, 5), (2, 3), (4, 64)])
def test_exact_macs_per_kernel_class_random(seed, pw):
    """The per-kernel-class exact counts (the roofline numerators) equal a
    brute-force count on the boolean elimination pattern and partition the
    factor and SelInv flop formulas."""
    rng = np.random.default_rng(seed)
    n = 70
    P = rng.uniform(size=(n, n)) < 0.05
    P = P | P.T | np.eye(n, dtype=bool)
    colptr, rows = _lower_csc_from_dense(P)
    a = B.Analysis(n, colptr, rows, leaf_cols=12, panel_width=pw)
    ex = a.export()
    Lx = osym.fill_pattern(osym.permute(P, ex["perm"]))
    want = _exact_macs_by_class(a, Lx, pw)
    got = np.array(a.info["macs_exact"])
    assert np.allclose(got, want, rtol=1e-12, atol=0), (got, want)
    assert got[5] == 0.0 and got[7] == 0.0
    i = a.info
    assert 8.0 * (got[1] + got[3] + got[6]) == pytest.approx(i["flops_factor"], rel=1e-12)
    assert 8.0 * (got[0] + got[2] + got[4]) == pytest.approx(i["flops_selinv"], rel=1e-12)


def test_exact_macs_per_kernel_class_atom_blocks():
    s = lattice.make_system("honeycomb", (4, 3), 3, 3.0, 5, periodic=False)
    a = B.Analysis.from_system(s, leaf_cols=9, panel_width=4)
    Pd = osym.dense_pattern_from_lower_csc(s.n, s.colptr, s.rowind)
    Lx = osym.fill_pattern(osym.permute(Pd, a.export()["perm"]))
    want = _exact_macs_by_class(a, Lx, 4)
    assert np.allclose(np.array(a.info["macs_exact"]), want, rtol=1e-12, atol=0)


def test_fused_lanes_option_values():
    """fused_lanes takes -1, 0 or 1; it leaves the structure, the sizes and
    the workspace of the analysis unchanged (fused lanes use the regions of
    the subtree streams).  By default (0) the lanes are fused for trees of
    small supernodes (a 1D chain) and not for large ones (a 13-orbital
    sheet); -1 and 1 force either."""
    s = lattice.make_system("honeycomb", (6, 6), 13, 3.0, 3)
    a0 = B.Analysis.from_system(s)
    a1 = B.Analysis.from_system(s, fused_lanes=1)
    for k in ("nnz_L", "nsuper", "npanel", "bytes_per_shift", "work_bytes", "gather_per_shift", "sel_lanes"):
        assert a0.info[k] == a1.info[k], k
    assert a0.workspace_size(20) == a1.workspace_size(20)
    assert a0.info["fused_lanes"] == 0 and a1.info["fused_lanes"] == 1
    assert a0.info["sel_lanes"] > 1
    c = lattice.config_system(0)
    assert B.Analysis.from_system(c).info["fused_lanes"] == 1
    assert B.Analysis.from_system(c, fused_lanes=-1).info["fused_lanes"] == 0
    for bad in (-2, 2):
        with pytest.raises(B.PxsError):
            B.Analysis.from_system(s, fused_lanes=bad)


def test_lane_fusion_rule_over_the_batch_mix():
    """The structural default fuses the subtree lanes of every 1D chain of
    the 64-system mix (many supernodes of a few hundred columns, latency
    bound) and of no 2D sheet or 3D bulk system (a few large supernodes)."""
    for s, P in lattice.batch_systems():
        a = B.Analysis.from_system(s)
        per = (a.info["flops_factor"] + a.info["flops_selinv"]) / a.info["nsuper"]
        assert a.info["fused_lanes"] == (1 if s.kind == "chain" else 0), (s.kind, s.n, per)
