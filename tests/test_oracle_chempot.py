"""Pins of the oracle's chemical-potential search (Sec. II.C) against what
the mathematics fixes: the zero-temperature limit of the integration by
parts is linear interpolation; densely sampled N_inf reproduces the exact
smeared electron count; a gapped spectrum gives band-edge estimates within
one sample spacing; the exact Newton root satisfies N_P(mu*) = N_e and sits
within the expansion error of the Fermi-Dirac root; Tr[Gamma^d S] is the
mu-derivative of N_P."""
import numpy as np
import pytest

from oracle import chempot as oc
from oracle import dense as od
from oracle import fermi as of
from oracle import poles as op

BETA = 1052.58


def test_zero_temperature_limit_is_linear_interpolation():
    rng = np.random.default_rng(1)
    eps = np.sort(rng.uniform(-1, 1, 12))
    ninf = 2.0 * np.cumsum(rng.integers(0, 4, 12))
    for mu in np.linspace(-1.2, 1.2, 37):
        got = oc.n_beta_from_samples(eps, ninf, mu, 1e12)
        assert abs(got - np.interp(mu, eps, ninf)) <= 1e-6, mu


def test_dense_samples_reproduce_smeared_count():
    rng = np.random.default_rng(2)
    ev = np.sort(rng.uniform(-0.9, 0.9, 60))
    beta = 40.0
    eps = np.linspace(-1.2, 1.2, 24001)
    ninf = 2.0 * oc.counts_from_eigenvalues(ev)(eps)
    for mu in (-0.5, -0.1, 0.0, 0.33, 0.7):
        exact = od.electron_number(ev, mu, beta)
        got = oc.n_beta_from_samples(eps, ninf, mu, beta)
        assert abs(got - exact) <= 2e-3, (mu, got, exact)


def test_bracket_finds_band_edges_of_gapped_spectrum():
    rng = np.random.default_rng(3)
    lower = np.sort(rng.uniform(-0.9, -0.2, 20))
    upper = np.sort(rng.uniform(0.3, 0.9, 20))
    lower[-1], upper[0] = -0.2, 0.3
    ev = np.concatenate([lower, upper])
    Ne = 40.0
    lo, hi, mu, samples = oc.bracket(oc.counts_from_eigenvalues(ev), Ne, -1.0, 1.0, BETA, Q=16, dN=0.1,
                                     rounds=3)
    h = samples[-1][0][1] - samples[-1][0][0]
    assert -0.2 < mu < 0.3
    assert abs(mu - 0.05) <= h + 10.0 / BETA
    assert lo <= -0.2 and hi >= 0.3
    assert hi - lo <= 0.5 + 4 * h + 20.0 / BETA


def test_bracket_widens_when_start_interval_misses():
    ev = np.linspace(-0.9, 0.9, 50)
    Ne = 2.0 * 40
    lo, hi, mu, samples = oc.bracket(oc.counts_from_eigenvalues(ev), Ne, -0.9, -0.5, BETA, Q=8, rounds=2)
    assert len(samples) > 2
    assert ev[39] - 0.05 <= mu <= ev[40] + 0.05


@pytest.mark.parametrize("Ne_frac", [0.37, 0.5, 0.81])
def test_newton_root_matches_fermi_dirac_within_expansion_error(Ne_frac):
    rng = np.random.default_rng(4)
    ev = np.sort(rng.uniform(-1, 1, 80))
    Ne = 2.0 * 80 * Ne_frac + 0.3
    P = 80
    spec = (-1.0, 1.0)
    mu = oc.mu_exact(ev, Ne, BETA, P, spec, -0.99, 0.99)
    Np, dNp = oc.n_pole(ev, mu, BETA, P, spec)
    assert abs(Np - Ne) <= 1e-9
    dE = max(abs(spec[0] - mu), abs(spec[1] - mu))
    eP = op.expansion_error(BETA, dE, mu, P, extra=ev)
    assert abs(od.electron_number(ev, mu, BETA) - Ne) <= len(ev) * eP + 1e-12
    # Tr[Gamma^d S] against the closed form sum_i -f'(eps_i - mu) and a
    # central difference of N_P
    eP_d = op.expansion_error(BETA, dE, mu, P, g="d", extra=ev)
    exact_d = float(of.dfermi_dmu(ev - mu, BETA).sum())
    assert abs(dNp - exact_d) <= len(ev) * eP_d + 1e-9
    d = 1e-6
    fd = (oc.n_pole(ev, mu + d, BETA, P, spec)[0] - oc.n_pole(ev, mu - d, BETA, P, spec)[0]) / (2 * d)
    assert abs(fd - dNp) <= 1e-4 * max(1.0, abs(dNp))
