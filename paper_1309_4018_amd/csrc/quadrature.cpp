// Quadrature tables of libpbtc (host side).
//
// Triangle rules: the symmetric Gauss rules of Dunavant (1985), the family
// behind "K Gauss points per triangular element" and "K_fine points in the
// near-singular region" (sec. 3, parameter tables).  Angular rule of the
// semi-analytic self integral: Gauss-Legendre, N_k points per sub-triangle
// (sec. 3, lysozyme parameter table).
#include <cmath>

#include "internal.h"

namespace pbtc {

namespace {

int put3(double* b, double* w, int at, double a, double wt) {
  const double c = 0.5 * (1.0 - a);
  const double pts[3][3] = {{a, c, c}, {c, a, c}, {c, c, a}};
  for (int i = 0; i < 3; ++i) {
    b[3 * (at + i) + 0] = pts[i][0];
    b[3 * (at + i) + 1] = pts[i][1];
    b[3 * (at + i) + 2] = pts[i][2];
    w[at + i] = wt;
  }
  return at + 3;
}

int put6(double* b, double* w, int at, double a, double c, double wt) {
  const double d = 1.0 - a - c;
  const double pts[6][3] = {{a, c, d}, {a, d, c}, {c, a, d}, {c, d, a}, {d, a, c}, {d, c, a}};
  for (int i = 0; i < 6; ++i) {
    for (int k = 0; k < 3; ++k) b[3 * (at + i) + k] = pts[i][k];
    w[at + i] = wt;
  }
  return at + 6;
}

int put1(double* b, double* w, int at, double wt) {
  b[3 * at + 0] = b[3 * at + 1] = b[3 * at + 2] = 1.0 / 3.0;
  w[at] = wt;
  return at + 1;
}

}  // namespace

// Fills bary (K x 3) and weights (K); returns false for an unknown K.
bool triangle_rule(int k, double* bary, double* w) {
  int at = 0;
  switch (k) {
    case 1:
      at = put1(bary, w, at, 1.0);
      break;
    case 3:  // degree 2
      at = put3(bary, w, at, 2.0 / 3.0, 1.0 / 3.0);
      break;
    case 4:  // degree 3, negative centre weight
      at = put1(bary, w, at, -27.0 / 48.0);
      at = put3(bary, w, at, 0.6, 25.0 / 48.0);
      break;
    case 7: {  // degree 5
      const double r = std::sqrt(15.0);
      at = put1(bary, w, at, 9.0 / 40.0);
      at = put3(bary, w, at, (9.0 - 2.0 * r) / 21.0, (155.0 + r) / 1200.0);
      at = put3(bary, w, at, (9.0 + 2.0 * r) / 21.0, (155.0 - r) / 1200.0);
      break;
    }
    case 19:  // degree 9
      at = put1(bary, w, at, 0.097135796282799);
      at = put3(bary, w, at, 0.020634961602525, 0.031334700227139);
      at = put3(bary, w, at, 0.125820817014127, 0.077827541004774);
      at = put3(bary, w, at, 0.623592928761935, 0.079647738927210);
      at = put3(bary, w, at, 0.910540973211095, 0.025577675658698);
      at = put6(bary, w, at, 0.036838412054736, 0.221962989160766, 0.043283539377289);
      break;
    default:
      return false;
  }
  return at == k;
}

// n-point Gauss-Legendre on [-1, 1] by Newton's method on P_n, started from
// the Chebyshev-like guesses cos(pi (i - 1/4) / (n + 1/2)).
bool gauss_legendre(int n, double* x, double* w) {
  if (n < 1 || n > kMaxNk) return false;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1.0;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = (n == 1) ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
    const double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = wt;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
  return true;
}

}  // namespace pbtc
