"""Pole table {z_l, omega_l^g} of the pole expansion (oracle; test
infrastructure).

The paper (Sec. II.A, eq. polerho) states that f_beta(eps - mu) is
approximated by Im sum_{l=1}^P omega_l / (eps - (z_l + mu)), that z_l and
omega_l depend only on beta, Delta E and P, that O(log(beta Delta E)) terms
suffice, and that the energy/free-energy (eq. gammaF) and derivative (Sec.
II.C) expansions reuse the same z_l with other weights.  It defers the
construction to other work.  The reading implemented here (and, separately,
in the library's host code) is the contour-quadrature construction:

1.  For g analytic off the imaginary-axis Matsubara points +-(2k+1) i pi/beta
    and x in [-Delta E, Delta E],
        g(x) = (1/2 pi i) oint g(z) / (z - x) dz
    around a contour that encloses [-Delta E, Delta E] and passes between
    +- i pi/beta.
2.  Substitute xi = z^2 + pi^2/beta^2.  The interval maps to [m, M] with
    m = pi^2/beta^2, M = Delta E^2 + pi^2/beta^2, and every singularity to
    (-inf, 0].  Summing the two branches z = +-sqrt(xi - m) gives the
    single-valued integrand
        h(xi) = (1/(2z)) [ g(z)/(z - x) + g(-z)/(z + x) ],
    so g(x) = (1/2 pi i) oint h(xi) dxi around [m, M].
3.  Map the rectangle [-K, K] x [0, K'] onto the upper half xi-plane with
    xi = sqrt(mM) (1/k + sn(t|k)) / (1/k - sn(t|k)),
    k = (sqrt(M/m) - 1)/(sqrt(M/m) + 1), and integrate along Im t = K'/2 with
    the midpoint rule at t_j = -K + i K'/2 + (j - 1/2) 2K/Q, j = 1..Q.
    The lower half follows by conjugate symmetry, so
        g(x) ~= -(2K/(pi Q)) Im sum_j xi'(t_j) h(xi_j),
    xi'(t) = sqrt(mM) (2/k) cn(t) dn(t) / (1/k - sn(t))^2.
4.  Each node gives a pole z_j = sqrt(xi_j - m) (first quadrant) and a pole
    -z_j (third quadrant).  For real x, Im[a/(x - b)] = -Im[conj(a)/(x -
    conj(b))], so the third-quadrant pole is folded onto -conj(z_j) in the
    second quadrant.  Hence P = 2Q poles, all with Im z_l > 0.

The Jacobi functions at complex argument use the addition formulas of
Abramowitz & Stegun 16.21.2-4 on scipy's real-argument sn, cn, dn.
"""
import numpy as np
import scipy.special as sp

from . import fermi

SETS = ("rho", "E", "F", "d")


def jacobi_complex(a, b, m, m1):
    """sn, cn, dn of t = a + i b (real a, b) for parameter m = k^2, with
    complementary parameter m1 = 1 - m passed separately for accuracy.
    A&S 16.21.2-4."""
    s, c, d, _ = sp.ellipj(a, m)
    s1, c1, d1, _ = sp.ellipj(b, m1)
    den = c1 * c1 + m * s * s * s1 * s1
    sn = (s * d1 + 1j * c * d * s1 * c1) / den
    cn = (c * c1 - 1j * s * d * s1 * d1) / den
    dn = (d * c1 * d1 - 1j * m * s * c * s1) / den
    return sn, cn, dn


def quadrature_nodes(beta, dE, Q):
    """Nodes z_j (first quadrant) and coefficients c_j such that
    g(x) ~= Im sum_j [ c_j g(z_j)/(z_j - x) + c_j g(-z_j)/(z_j + x) ]."""
    mshift = (np.pi / beta) ** 2
    m = mshift
    M = dE * dE + mshift
    r = np.sqrt(M / m)
    k = (r - 1.0) / (r + 1.0)
    kp2 = 4.0 * r / (r + 1.0) ** 2          # k'^2 = 1 - k^2 without cancellation
    K = sp.ellipkm1(kp2)                    # K(k) with parameter 1 - kp2 = k^2
    Kp = sp.ellipk(kp2)                     # K'(k) = K(k')
    j = np.arange(1, Q + 1)
    a = -K + (j - 0.5) * 2.0 * K / Q
    b = np.full(Q, 0.5 * Kp)
    sn, cn, dn = jacobi_complex(a, b, k * k, kp2)
    sq = np.sqrt(m * M)
    xi = sq * (1.0 / k + sn) / (1.0 / k - sn)
    dxi = sq * (2.0 / k) * cn * dn / (1.0 / k - sn) ** 2
    z = np.sqrt(xi - mshift)                # principal branch: Im z > 0
    coef = -(2.0 * K / (np.pi * Q)) * dxi / (2.0 * z)
    return z, coef


def pole_table(beta, dE, mu, P, sets=SETS):
    """Shifts w_l = z_l + mu (complex, Im > 0) and weights omega_l^g for the
    requested occupation sets, such that
        g(eps - mu) ~= Im sum_l omega_l^g / (eps - w_l).
    P must be even (P/2 quadrature nodes, two poles each)."""
    if P < 2 or P % 2:
        raise ValueError("P must be a positive even number")
    Q = P // 2
    z, coef = quadrature_nodes(beta, dE, Q)
    zl = np.concatenate([z, -np.conj(z)])
    weights = {}
    for g in sets:
        gp = fermi.occupation(g, z, beta, mu)
        gm = fermi.occupation(g, -z, beta, mu)
        # Im[c g(z)/(z - x)] = Im[-c g(z)/(x - z)]
        w1 = -coef * gp
        # Im[c g(-z)/(z + x)] = Im[c g(-z)/(x - (-z))] = Im[-conj(c g(-z))/(x - (-conj z))]
        w2 = -np.conj(coef * gm)
        weights[g] = np.concatenate([w1, w2])
    return zl + mu, weights


def rational(eps, shifts, weight):
    """r(eps) = Im sum_l omega_l / (eps - w_l), eps real (array)."""
    eps = np.asarray(eps, dtype=np.float64)
    return np.imag((weight[None, :] / (eps[:, None] - shifts[None, :])).sum(axis=1))


def expansion_error(beta, dE, mu, P, g="rho", npts=20001, extra=None):
    """e_P^g = max over a grid of [mu - dE, mu + dE] (plus optional extra
    points) of |g(eps - mu) - r^g(eps)|."""
    shifts, w = pole_table(beta, dE, mu, P, sets=(g,))
    eps = mu + np.linspace(-dE, dE, npts)
    if extra is not None:
        eps = np.concatenate([eps, np.asarray(extra, dtype=np.float64)])
    exact = np.real(fermi.occupation(g, eps - mu, beta, mu))
    return float(np.max(np.abs(exact - rational(eps, shifts, w[g]))))
