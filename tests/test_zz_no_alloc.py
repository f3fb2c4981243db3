"""The allocation-free entry point (pxs_density_matrix_noalloc): its
workspace is the library's device scratch array.  Checked through the C ABI
against the entry point it varies (pxs_density_matrix with a caller
workspace) and against the oracle, on two calls in a row, the second with a
smaller system, so stale scratch contents from the first call would show."""
import sys

import numpy as np
import pytest

from oracle import dense as odense
from oracle import poles as opoles
from paper_1405_0194_amd import binding as B
from paper_1405_0194_amd import lattice

BETA = lattice.BETA_300K


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_rejects_oversized_before_device_work():
    """Host-side size check: a batch whose workspace exceeds the scratch
    array is refused with PXS_EINVAL before any pointer is used (no GPU)."""
    lib = B.load()
    s = lattice.config_system(0)
    a = B.Analysis.from_system(s)
    code = lib.pxs_density_matrix_noalloc(a._h, None, None, BETA, 1.0, 0.0, 4096, 2, None, None, None, None,
                                          None, None, None)
    assert code == B.PXS_EINVAL
    assert "scratch" in lib.pxs_last_error().decode()
    # bad pole counts are refused as by pxs_density_matrix
    for P, nsets in ((3, 2), (0, 2), (40, 0), (40, 5)):
        assert lib.pxs_density_matrix_noalloc(a._h, None, None, BETA, 1.0, 0.0, P, nsets, None, None, None,
                                              None, None, None, None) == B.PXS_EINVAL


def _oracle_gamma(s, mu, dE, P):
    Hd, Sd = s.dense()
    ow, oom = opoles.pole_table(BETA, dE, mu, P, sets=("rho", "E"))
    G = odense.gamma_route_b(Hd, Sd, ow, oom)
    cols = s.entry_cols()
    return [G[n][s.rowind, cols] for n in ("rho", "E")], [odense.traces(G[n], Hd, Sd) for n in ("rho", "E")]


@pytest.mark.gpu
def test_noalloc_equals_workspace_entry_point_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cases = [(lattice.config_system(0), 40, 0.02),                                  # N = 256
             (lattice.make_system("chain", 30, 4, 2.0, 1405), 20, -0.03)]          # N = 120: smaller
    for s, P, mu in cases:
        dE = 1.0 + abs(mu)
        a = B.Analysis.from_system(s)
        H = torch.from_numpy(s.hval).cuda()
        S = torch.from_numpy(s.sval).cuda()
        say(f"case: noalloc N={s.n} P={P}")
        out_n, tr_n, info_n, sh_n, wt_n = B.density_matrix_noalloc(a, H, S, BETA, dE, mu, P, nsets=2)
        out_n = out_n.cpu().numpy().copy()
        say(f"case: workspace entry point N={s.n} P={P}")
        out_w, tr_w, info_w, sh_w, wt_w = B.density_matrix(a, H, S, BETA, dE, mu, P, nsets=2)
        torch.cuda.synchronize()
        out_w = out_w.cpu().numpy()
        assert np.all(info_n == 0) and np.all(info_w == 0)
        assert np.array_equal(sh_n, sh_w) and np.array_equal(wt_n, wt_w)
        # same kernels in the same issue order: the same bits
        assert np.array_equal(out_n, out_w)
        assert np.array_equal(tr_n, tr_w)
        want, wtr = _oracle_gamma(s, mu, dE, P)
        for g in range(2):
            e = float(np.max(odense.entry_error(out_n[g], want[g])))
            say("entry error", e)
            assert e <= 1e-10
            assert abs(tr_n[g, 0] - wtr[g][0]) <= 1e-10 * max(1.0, abs(wtr[g][0]))
            assert abs(tr_n[g, 1] - wtr[g][1]) <= 1e-10 * max(1.0, abs(wtr[g][1]))
