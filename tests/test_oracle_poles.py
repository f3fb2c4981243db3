"""Pins of the oracle's pole table (Sec. II.A, eq. polerho; Sec. II.C).

Nothing here compares the oracle with itself: the Jacobi functions are
checked against their identities and the imaginary transformation, and the
expansion against the closed-form occupation functions on a fine grid.
"""
import numpy as np
import pytest
import scipy.special as sp

from oracle import fermi, poles

BETA = 1.0 / (3.166811563e-6 * 300.0)


@pytest.mark.parametrize("m", [0.3, 0.9, 0.98817])
def test_jacobi_complex_identities(m):
    m1 = 1.0 - m
    a = np.linspace(-1.5, 1.5, 7)
    b = np.linspace(0.1, 1.2, 7)
    A, B = np.meshgrid(a, b)
    sn, cn, dn = poles.jacobi_complex(A.ravel(), B.ravel(), m, m1)
    assert np.allclose(sn ** 2 + cn ** 2, 1.0, atol=1e-13)
    assert np.allclose(dn ** 2 + m * sn ** 2, 1.0, atol=1e-13)
    # complex derivative d sn / dt = cn dn, along the real and imaginary axes
    h = 1e-6
    snr, _, _ = poles.jacobi_complex(A.ravel() + h, B.ravel(), m, m1)
    snl, _, _ = poles.jacobi_complex(A.ravel() - h, B.ravel(), m, m1)
    snu, _, _ = poles.jacobi_complex(A.ravel(), B.ravel() + h, m, m1)
    snd, _, _ = poles.jacobi_complex(A.ravel(), B.ravel() - h, m, m1)
    d_re = (snr - snl) / (2 * h)
    d_im = (snu - snd) / (2j * h)
    assert np.allclose(d_re, cn * dn, rtol=1e-7, atol=1e-7)
    assert np.allclose(d_im, cn * dn, rtol=1e-7, atol=1e-7)


def test_jacobi_imaginary_transformation():
    # sn(iy|m) = i sc(y|1-m)   (Jacobi's imaginary transformation)
    m = 0.7
    y = np.linspace(0.05, 1.0, 9)
    sn, cn, dn = poles.jacobi_complex(np.zeros_like(y), y, m, 1 - m)
    s1, c1, d1, _ = sp.ellipj(y, 1 - m)
    assert np.allclose(sn, 1j * s1 / c1, atol=1e-14)
    assert np.allclose(cn, 1.0 / c1, atol=1e-14)
    assert np.allclose(dn, d1 / c1, atol=1e-14)


def test_shifts_upper_half_plane_and_count():
    for P in (2, 10, 40, 80):
        w, om = poles.pole_table(BETA, 1.5, 0.2, P)
        assert w.shape == (P,)
        assert np.all(w.imag > 0)
        for g in poles.SETS:
            assert om[g].shape == (P,)
    with pytest.raises(ValueError):
        poles.pole_table(BETA, 1.5, 0.2, 41)


@pytest.mark.parametrize("g", ["rho", "E", "F", "d"])
def test_expansion_error_decays_geometrically(g):
    # Sec. II.A: O(log(beta dE)) poles suffice, i.e. the error falls
    # geometrically in P.  Reference: the closed-form occupation on a grid.
    dE, mu = 2.0, 0.1
    errs = [poles.expansion_error(BETA, dE, mu, P, g, npts=4001) for P in (40, 50, 60, 70, 80)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 8.0, errs
    scale = {"rho": 1.0, "E": 1.0, "F": 1.0, "d": BETA}[g]
    assert errs[0] < 2e-3 * scale
    assert errs[-1] < 2e-8 * scale


def test_rho_expansion_absolute_levels():
    # P = 40..80 at 300 K with Delta E = 2 Ha
    assert poles.expansion_error(BETA, 2.0, 0.0, 40) < 1e-4
    assert poles.expansion_error(BETA, 2.0, 0.0, 60) < 1e-6
    assert poles.expansion_error(BETA, 2.0, 0.0, 80) < 1e-9


def test_special_values_and_particle_hole_symmetry():
    P, mu, dE = 60, -0.07, 1.07
    w, om = poles.pole_table(BETA, dE, mu, P)
    e_p = poles.expansion_error(BETA, dE, mu, P)
    r_mu = poles.rational([mu], w, om["rho"])[0]
    assert abs(r_mu - 1.0) <= 2 * e_p + 1e-14          # f(0) = 1
    x = np.linspace(0.0, 1.0, 301)
    rp = poles.rational(mu + x, w, om["rho"])
    rm = poles.rational(mu - x, w, om["rho"])
    assert np.max(np.abs(rp + rm - 2.0)) <= 2 * e_p + 1e-14   # f(x) + f(-x) = 2
    # low/high limits of the occupation
    assert abs(poles.rational([mu - 0.9], w, om["rho"])[0] - 2.0) < 1e-6
    assert abs(poles.rational([mu + 0.9], w, om["rho"])[0]) < 1e-6


def test_energy_and_derivative_sets_match_closed_forms():
    P, mu, dE = 80, 0.05, 1.05
    w, om = poles.pole_table(BETA, dE, mu, P)
    eps = mu + np.linspace(-dE, dE, 2001)
    f = fermi.fermi(eps - mu, BETA)
    rE = poles.rational(eps, w, om["E"])
    assert np.max(np.abs(rE - eps * f)) < 1e-8
    # d/dmu of f by a centred difference of the closed form
    h = 1e-7
    fd = (fermi.fermi(eps - mu - h, BETA) - fermi.fermi(eps - mu + h, BETA)) / (2 * h)
    rd = poles.rational(eps, w, om["d"])
    assert np.max(np.abs(rd - fd)) < 1e-4 * BETA
    rF = poles.rational(eps, w, om["F"])
    x = eps - mu
    Fx = -(2.0 / BETA) * np.logaddexp(0.0, -BETA * x)
    assert np.max(np.abs(rF - Fx)) < 1e-8


def test_fermi_closed_forms():
    x = np.linspace(-0.5, 0.5, 101)
    f = fermi.fermi(x, BETA)
    assert np.allclose(f + fermi.fermi(-x, BETA), 2.0, atol=1e-15)
    assert fermi.fermi(np.array([0.0]), BETA)[0] == 1.0
    # complex continuation agrees with the defining formula where it is safe
    z = np.array([0.001 + 0.001j, -0.002 + 0.0005j])
    assert np.allclose(fermi.fermi(z, BETA), 2.0 / (1.0 + np.exp(BETA * z)), rtol=1e-13)
    zf = np.array([0.001 + 0.001j, -0.002 + 0.0005j])
    assert np.allclose(fermi.free_occ(zf, BETA), -(2.0 / BETA) * np.log(1.0 + np.exp(-BETA * zf)),
                       rtol=1e-12)
