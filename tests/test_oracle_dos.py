"""Pins of the DOS/LDOS oracle (Sec. II.D): bin averages integrate to the
electron count; the dense-inverse and eigen-decomposition routes of the LDOS
agree; its trace against S is the Lorentzian-broadened DOS; a diagonal pencil
has the closed form; the broadened DOS integrates to 2N as eta -> 0 and its
bin integrals approach the exact bin counts."""
import numpy as np
import pytest

from oracle import dense as od
from oracle import dos as odos


def _pencil(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    H = (A + A.T) / (2 * np.sqrt(n))
    B = 0.1 * rng.standard_normal((n, n))
    S = (B + B.T) / 2
    np.fill_diagonal(S, 1.0 + np.abs(S).sum(axis=1))
    return H, S


def test_bins_integrate_to_electron_count():
    H, S = _pencil(40, 1)
    ev = od.gen_eigh(H, S)[0]
    edges = np.linspace(ev[0] - 0.1, ev[-1] + 0.1, 57)
    g = odos.dos_bins(ev, edges)
    assert np.all(g >= 0)
    assert abs((g * np.diff(edges)).sum() - 2 * len(ev)) < 1e-9
    # a bin holding exactly one eigenvalue
    e = ev[10]
    gap = min(ev[10] - ev[9], ev[11] - ev[10]) / 2
    one = odos.dos_bins(ev, np.array([e - gap, e + gap]))
    assert abs(one[0] * 2 * gap - 2.0) < 1e-12


@pytest.mark.parametrize("eps,eta", [(0.0, 1e-2), (0.13, 1e-3), (-0.4, 5e-2)])
def test_ldos_routes_agree_and_trace_is_broadened_dos(eps, eta):
    H, S = _pencil(30, 2)
    eig = od.gen_eigh(H, S)
    G1 = odos.ldos_dense(H, S, eps, eta)
    G2 = odos.ldos_eig(H, S, eps, eta, eig)
    assert np.abs(G1 - G2).max() <= 1e-10 * np.abs(G2).max()
    assert np.abs(G1 - G1.T).max() <= 1e-12 * np.abs(G1).max()
    tr = float(np.sum(G1 * S))
    assert abs(tr - odos.broadened_dos(eig[0], eps, eta)[0]) <= 1e-10 * max(1.0, abs(tr))


def test_ldos_diagonal_pencil_closed_form():
    h = np.array([-0.5, -0.1, 0.2, 0.7])
    s = np.array([1.0, 2.0, 1.5, 3.0])
    eps, eta = 0.05, 0.02
    G = odos.ldos_dense(np.diag(h), np.diag(s), eps, eta)
    z = h - (eps + 1j * eta) * s
    assert np.allclose(np.diag(G), (2 / np.pi) * np.imag(1 / z), rtol=1e-13, atol=0)
    assert np.abs(G - np.diag(np.diag(G))).max() == 0.0


def test_broadened_dos_tends_to_bin_counts():
    H, S = _pencil(25, 3)
    ev = od.gen_eigh(H, S)[0]
    lo, hi = ev[0] - 1.0, ev[-1] + 1.0
    x = np.linspace(lo, hi, 400001)
    for eta in (1e-2, 1e-3):
        g = odos.broadened_dos(ev, x, eta)
        total = np.trapezoid(g, x)
        # the Lorentzian tails beyond [lo, hi] carry (2/pi) eta / distance per state
        assert abs(total - 2 * len(ev)) < 2 * len(ev) * (2 / np.pi) * eta / 1.0 * 1.05
    # bin integral around one isolated eigenvalue -> 2 as eta -> 0
    i = 12
    a, b = (ev[i - 1] + ev[i]) / 2, (ev[i] + ev[i + 1]) / 2
    xs = np.linspace(a, b, 200001)
    got = np.trapezoid(odos.broadened_dos(ev, xs, 1e-5), xs)
    assert abs(got - 2.0) < 1e-2
