// Pole table of the Fermi-Dirac expansion (host).
//
// The paper (Sec. II.A, eq. polerho) fixes the form
//   f_beta(eps - mu) ~= Im sum_l omega_l / (eps - (z_l + mu)),
// states that z_l, omega_l depend only on beta, Delta E and P with
// O(log(beta Delta E)) terms, and that the energy / free-energy (eq. gammaF)
// and mu-derivative (Sec. II.C) expansions share the same z_l.  The
// construction used here is contour quadrature of the Cauchy integral:
//   * xi = x^2 + (pi/beta)^2 maps [-dE, dE] to [m, M] = [(pi/beta)^2,
//     dE^2 + (pi/beta)^2] and every Matsubara pole onto (-inf, 0];
//   * the two branches z = +-sqrt(xi - m) give the single-valued integrand
//     h(xi) = (g(z)/(z - x) + g(-z)/(z + x)) / (2z);
//   * the rectangle [-K, K] x [0, K'] maps onto the upper half xi-plane by
//     xi = sqrt(mM) (1/k + sn t)/(1/k - sn t), k = (sqrt(M/m) - 1)/(sqrt(M/m) + 1);
//     the midpoint rule on Im t = K'/2 with Q = P/2 nodes, plus conjugate
//     symmetry, gives g(x) ~= -(2K/(pi Q)) Im sum_j xi'(t_j) h(xi_j);
//   * node j yields the poles z_j (first quadrant) and -conj(z_j) (the
//     third-quadrant pole -z_j folded into the upper half plane).
// Elliptic functions: the arithmetic-geometric mean for K and for the
// real-argument sn, cn, dn (Abramowitz & Stegun 16.4, 17.6) and the
// addition formulas A&S 16.21.2-4 for the complex argument.
#include <cmath>
#include <complex>
#include <vector>

#include "pxs_internal.h"

namespace pxs {
namespace {

using cd = std::complex<double>;

// Complete elliptic integral of the first kind for modulus k, given the
// complementary modulus kp = sqrt(1 - k^2) (passed separately so that k
// close to 1 loses no digits): K(k) = pi / (2 AGM(1, kp)).
double ellip_K_from_kp(double kp) {
  double a = 1.0, b = kp;
  for (int it = 0; it < 64 && std::fabs(a - b) > 1e-16 * a; ++it) {
    double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return M_PI / (2.0 * a);
}

// sn, cn, dn of real u for modulus k (complementary modulus kp) by the
// descending AGM sequence: phi_N = 2^N a_N u, then
// phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2.
void jacobi_real(double u, double k, double kp, double* sn, double* cn, double* dn) {
  if (k == 0.0) {
    *sn = std::sin(u); *cn = std::cos(u); *dn = 1.0;
    return;
  }
  double a[64], c[64];
  a[0] = 1.0;
  double b = kp;
  c[0] = k;
  int N = 0;
  while (N < 62 && std::fabs(c[N]) > 1e-17) {
    double an = 0.5 * (a[N] + b);
    double cn_ = 0.5 * (a[N] - b);
    b = std::sqrt(a[N] * b);
    ++N;
    a[N] = an;
    c[N] = cn_;
  }
  double phi = std::ldexp(a[N] * u, N);
  double phi_prev = phi;
  for (int n = N; n >= 1; --n) {
    phi_prev = phi;
    phi = 0.5 * (phi + std::asin(c[n] * std::sin(phi) / a[n]));
  }
  *sn = std::sin(phi);
  *cn = std::cos(phi);
  *dn = (N >= 1) ? std::cos(phi) / std::cos(phi_prev - phi) : 1.0;
}

// A&S 16.21.2-4: sn, cn, dn at x + i y for modulus k, complementary kp.
void jacobi_complex(double x, double y, double k, double kp, cd* sn, cd* cn, cd* dn) {
  double s, c, d, s1, c1, d1;
  jacobi_real(x, k, kp, &s, &c, &d);
  jacobi_real(y, kp, k, &s1, &c1, &d1);
  double m = k * k;
  double den = c1 * c1 + m * s * s * s1 * s1;
  *sn = cd(s * d1, c * d * s1 * c1) / den;
  *cn = cd(c * c1, -s * d * s1 * d1) / den;
  *dn = cd(d * c1 * d1, -m * s * c * s1) / den;
}

// Occupation functions continued to complex x = z (Sec. II.A eq. fermidirac
// with spin factor 2; eq. gammaF; Sec. II.C for d/dmu).
cd occ_rho(cd z, double beta) {
  cd bz = beta * z;
  if (bz.real() > 0) {
    cd e = std::exp(-bz);
    return 2.0 * e / (1.0 + e);
  }
  return 2.0 / (1.0 + std::exp(bz));
}
cd occ(int set, cd z, double beta, double mu) {
  switch (set) {
    case 0: return occ_rho(z, beta);
    case 1: return (z + mu) * occ_rho(z, beta);
    case 2: {
      cd bz = beta * z;
      if (bz.real() > 0) return -(2.0 / beta) * std::log(1.0 + std::exp(-bz));
      return 2.0 * z - (2.0 / beta) * std::log(1.0 + std::exp(bz));
    }
    default: {
      cd f = occ_rho(z, beta);
      return 0.5 * beta * f * (2.0 - f);
    }
  }
}

}  // namespace

int pole_table(double beta, double dE, double mu, int P, int nsets, double* shifts_ri,
               double* weights_ri) {
  if (!(beta > 0) || !(dE > 0) || P < 2 || (P & 1) || nsets < 1 || nsets > 4) return -1;
  const int Q = P / 2;
  const double mshift = (M_PI / beta) * (M_PI / beta);
  const double m = mshift, M = dE * dE + mshift;
  const double r = std::sqrt(M / m);
  const double k = (r - 1.0) / (r + 1.0);
  const double kp = 2.0 * std::sqrt(r) / (r + 1.0);   // sqrt(1 - k^2), no cancellation
  const double K = ellip_K_from_kp(kp);
  const double Kp = ellip_K_from_kp(k);
  const double sq = std::sqrt(m * M);
  for (int j = 0; j < Q; ++j) {
    double x = -K + (j + 0.5) * 2.0 * K / Q;
    cd sn, cn, dn;
    jacobi_complex(x, 0.5 * Kp, k, kp, &sn, &cn, &dn);
    cd xi = sq * (1.0 / k + sn) / (1.0 / k - sn);
    cd dxi = sq * (2.0 / k) * cn * dn / ((1.0 / k - sn) * (1.0 / k - sn));
    cd z = std::sqrt(xi - mshift);   // principal branch, Im z > 0
    cd coef = -(2.0 * K / (M_PI * Q)) * dxi / (2.0 * z);
    cd z2 = -std::conj(z);
    shifts_ri[2 * j] = z.real() + mu;
    shifts_ri[2 * j + 1] = z.imag();
    shifts_ri[2 * (j + Q)] = z2.real() + mu;
    shifts_ri[2 * (j + Q) + 1] = z2.imag();
    for (int g = 0; g < nsets; ++g) {
      cd w1 = -coef * occ(g, z, beta, mu);
      cd w2 = -std::conj(coef * occ(g, -z, beta, mu));
      weights_ri[2 * (g * P + j)] = w1.real();
      weights_ri[2 * (g * P + j) + 1] = w1.imag();
      weights_ri[2 * (g * P + j + Q)] = w2.real();
      weights_ri[2 * (g * P + j + Q) + 1] = w2.imag();
    }
  }
  return 0;
}

}  // namespace pxs
