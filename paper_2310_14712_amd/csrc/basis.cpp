// 1D ingredients of the spectral basis (Section "Spatial Discretization"):
// GLL points (the ends plus the roots of the Lobatto polynomial of order
// p-1), Gauss-Legendre rules, Lagrange polynomials on the GLL points, and the
// consistent 1D reference mass and stiffness matrices on [-1, 1].
#include <cmath>
#include <stdexcept>

#include "internal.h"

namespace imex {

namespace {
// Legendre P_0..P_m and derivatives P'_0..P'_m at x by the recurrences
// (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1},  P'_{k+1} = P'_{k-1} + (2k+1) P_k.
void legendre_table(int m, double x, double* P, double* dP) {
  P[0] = 1.0;
  dP[0] = 0.0;
  if (m == 0) return;
  P[1] = x;
  dP[1] = 1.0;
  for (int k = 1; k < m; ++k) {
    P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
    dP[k + 1] = dP[k - 1] + (2 * k + 1) * P[k];
  }
}
}  // namespace

// GLL nodes are the roots of (1 - x^2) P_p'(x), which is proportional to
// P_{p-1}(x) - P_{p+1}(x); Newton's method on that difference from a
// Chebyshev-Lobatto start.  Weights 2 / (p (p + 1) P_p(x_j)^2).
void gll_rule(int p, std::vector<double>& x, std::vector<double>& w) {
  if (p < 1) throw std::invalid_argument("p >= 1");
  x.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  double P[kMaxN + 2], dP[kMaxN + 2];
  for (int j = 0; j <= p; ++j) {
    double t = -std::cos(M_PI * j / p);
    if (j > 0 && j < p) {
      for (int it = 0; it < 100; ++it) {
        legendre_table(p + 1, t, P, dP);
        double q = P[p - 1] - P[p + 1];
        double dq = dP[p - 1] - dP[p + 1];
        double step = q / dq;
        t -= step;
        if (std::fabs(step) < 1e-17) break;
      }
    }
    x[j] = t;
  }
  x[0] = -1.0;
  x[p] = 1.0;
  for (int j = 0; j <= p; ++j) {
    legendre_table(p, x[j], P, dP);
    w[j] = 2.0 / (p * (p + 1.0) * P[p] * P[p]);
  }
}

// n-point Gauss-Legendre rule: Newton's method on P_n from the classical
// start cos(pi (i + 3/4) / (n + 1/2)); weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  double P[kMaxN + 4], dP[kMaxN + 4];
  for (int i = 0; i < n; ++i) {
    double t = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre_table(n, t, P, dP);
      double step = P[n] / dP[n];
      t -= step;
      if (std::fabs(step) < 1e-17) break;
    }
    legendre_table(n, t, P, dP);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dP[n] * dP[n]);
  }
}

// Lagrange polynomials l_i(xi) = prod_{j != i} (xi - x_j) / (x_i - x_j) and
// their derivatives l_i'(xi) = l_i(xi) * sum_{k != i} 1 / (xi - x_k), the
// latter evaluated by the product rule so it stays exact at the nodes.
void lagrange_eval(const std::vector<double>& nodes, double xi, double* val, double* der) {
  const int n = (int)nodes.size();
  for (int i = 0; i < n; ++i) {
    double v = 1.0, d = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const double inv = 1.0 / (nodes[i] - nodes[j]);
      // d(v * (xi - x_j) inv) = d * (xi - x_j) inv + v * inv
      d = d * (xi - nodes[j]) * inv + v * inv;
      v = v * (xi - nodes[j]) * inv;
    }
    val[i] = v;
    if (der) der[i] = d;
  }
}

// Consistent reference matrices Mh_ij = int N_i N_j, Kh_ij = int N_i' N_j'
// on [-1, 1], exact with the (p+1)-point Gauss-Legendre rule (degree 2p).
Ref1D make_ref1d(int p) {
  Ref1D r;
  r.p = p;
  r.n = p + 1;
  gll_rule(p, r.x, r.w);
  std::vector<double> gx, gw;
  gauss_rule(p + 1, gx, gw);
  const int n = r.n;
  r.Mh.assign(n * n, 0.0);
  r.Kh.assign(n * n, 0.0);
  double v[kMaxN], d[kMaxN];
  for (int q = 0; q < n; ++q) {
    lagrange_eval(r.x, gx[q], v, d);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        r.Mh[i * n + j] += gw[q] * v[i] * v[j];
        r.Kh[i * n + j] += gw[q] * d[i] * d[j];
      }
  }
  return r;
}

}  // namespace imex
