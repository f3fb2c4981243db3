"""GPU parity of the DOS / LDOS of Sec. II.D against the oracle: cumulative
counts and bin averages bit-exact against the eigenvalue counts; LDOS entries
against the dense inverse within 1e-10 per entry; Tr[G S] against the
Lorentzian-broadened DOS."""
import sys

import numpy as np
import pytest

from oracle import dense as odense
from oracle import dos as odos
from paper_1405_0194_amd import lattice

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


SYSTEMS = {"chain": lambda: lattice.config_system(0),
           "honeycomb": lambda: lattice.make_system("honeycomb", (4, 3), 13, 3.0, 78)}


@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_dos_bins_bit_exact(torch_cuda, name):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import dos as pdos
    s = SYSTEMS[name]()
    Hd, Sd = s.dense()
    ev = odense.gen_eigh(Hd, Sd)[0]
    edges = np.linspace(-1.0137, 1.0213, 57)
    gap = np.min(np.abs(edges[:, None] - ev[None, :]))
    assert gap > 1e-9, "an edge sits on an eigenvalue"
    say(f"case: dos {name} N={s.n} bins={len(edges) - 1}")
    a = B.Analysis.from_system(s).bind()
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    centres, g, c = pdos.dos(a, H, S, edges, batch=16)
    oc = 2 * np.searchsorted(ev, edges, side="left")
    assert np.array_equal(c, oc)
    assert np.array_equal(g, odos.dos_bins(ev, edges))
    assert c[0] == 0 and c[-1] == 2 * s.n


@pytest.mark.parametrize("name,eta", [("chain", 1e-2), ("honeycomb", 3e-3)])
def test_ldos_matches_oracle(torch_cuda, name, eta):
    torch = torch_cuda
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import dos as pdos
    s = SYSTEMS[name]()
    Hd, Sd = s.dense()
    eig = odense.gen_eigh(Hd, Sd)
    energies = np.array([-0.31, 0.0, 0.047, 0.21, 0.5])
    say(f"case: ldos {name} N={s.n} energies={len(energies)} eta={eta}")
    a = B.Analysis.from_system(s).bind()
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    out, tr, info = pdos.ldos(a, H, S, energies, eta)
    assert np.all(info == 0)
    out = out.cpu().numpy()
    cols = s.entry_cols()
    worst = 0.0
    for j, e in enumerate(energies):
        G = odos.ldos_dense(Hd, Sd, e, eta)
        worst = max(worst, float(np.max(odense.entry_error(out[j], G[s.rowind, cols]))))
        ref = odos.broadened_dos(eig[0], e, eta)[0]
        assert abs(tr[j, 0] - ref) <= TOL * max(1.0, abs(ref)), (e, tr[j, 0], ref)
        trH = float(np.sum(G * Hd))
        assert abs(tr[j, 1] - trH) <= TOL * max(1.0, abs(trH))
    say("ldos worst entry error", worst)
    assert worst <= TOL


def test_hermitian_dos_and_ldos(torch_cuda):
    """A complex Hermitian pencil: DOS bins bit-exact from the signs of the
    L D U pivots; LDOS (2/pi)(M - M^H)/2i, M = [H - (eps + i eta) S]^{-1},
    against the oracle's Hermitian inverse route; Tr[G S] against the
    broadened DOS."""
    torch = torch_cuda
    from oracle import hermitian as oherm
    from paper_1405_0194_amd import binding as B
    from paper_1405_0194_amd import dos as pdos
    s = lattice.make_hermitian_system("honeycomb", (4, 3), 13, 3.0, 80)
    Hd, Sd = s.dense()
    ev = oherm.gen_eigh(Hd, Sd)[0]
    edges = np.linspace(-1.0137, 1.0213, 41)
    assert np.min(np.abs(edges[:, None] - ev[None, :])) > 1e-9
    say(f"case: hermitian dos/ldos N={s.n}")
    a = B.Analysis.from_system(s).bind()
    H = torch.from_numpy(s.hval).cuda()
    S = torch.from_numpy(s.sval).cuda()
    centres, g, c = pdos.dos(a, H, S, edges, batch=16)
    assert np.array_equal(c, 2 * np.searchsorted(ev, edges, side="left"))
    assert np.array_equal(g, odos.dos_bins(ev, edges))
    energies = np.array([-0.2, 0.013, 0.3])
    eta = 3e-3
    out, tr, info = pdos.ldos(a, H, S, energies, eta)
    assert np.all(info == 0) and out.dtype == torch.complex128
    out = out.cpu().numpy()
    cols = s.entry_cols()
    worst = 0.0
    for j, e in enumerate(energies):
        G = oherm.gamma_route_a(Hd, Sd, np.array([e + 1j * eta]), {"g": np.array([2.0 / np.pi])})["g"]
        worst = max(worst, float(np.max(odense.entry_error(out[j], G[s.rowind, cols]))))
        ref = odos.broadened_dos(ev, e, eta)[0]
        assert abs(tr[j, 0] - ref) <= TOL * max(1.0, abs(ref)), (e, tr[j, 0], ref)
    say("hermitian ldos worst entry error", worst)
    assert worst <= TOL
