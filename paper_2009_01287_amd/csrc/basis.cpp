// 1D Gauss-Lobatto nodal basis (Sec. 2.2) and exact 1D matrices.
//
// The nodes of degree p on [0,1] are the endpoints and the p-1 roots of the
// derivative of the Legendre polynomial P_p (mapped from [-1,1]); they are
// found by Newton's method on the three-term Legendre recurrence. Mass and
// stiffness matrices are integrated exactly with a (p+1)-point Gauss rule.
#include <cmath>
#include <mutex>

#include "internal.hpp"

namespace hpdg {

static void legendre(int n, double x, double& P, double& dP, double& d2P) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1; dP = 0; d2P = 0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // (1-x^2) P'' - 2x P' + n(n+1) P = 0 ; P' = n (x P_n - P_{n-1}) / (x^2 - 1)
  dP = n * (x * p1 - p0) / (x * x - 1.0);
  d2P = (2.0 * x * dP - n * (n + 1.0) * P) / (1.0 - x * x);
}

static void gauss_rule_compute(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int j = 0; j < q; ++j) {
    double t = -std::cos(M_PI * (j + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP, d2P;
      legendre(q, t, P, dP, d2P);
      double dt = P / dP;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    double P, dP, d2P;
    legendre(q, t, P, dP, d2P);
    x[j] = 0.5 * (t + 1.0);
    w[j] = 1.0 / ((1.0 - t * t) * dP * dP);   // 2/((1-t^2)P'^2) scaled by 1/2
  }
  for (int j = 0; j < q / 2; ++j) {           // exact symmetry
    double a = 0.5 * (x[j] + (1.0 - x[q - 1 - j]));
    x[j] = a;
    x[q - 1 - j] = 1.0 - a;
    double b = 0.5 * (w[j] + w[q - 1 - j]);
    w[j] = w[q - 1 - j] = b;
  }
  if (q % 2 == 1) x[q / 2] = 0.5;
}

// rules up to 32 points are computed once and copied
void gauss_rule(int q, std::vector<double>& x, std::vector<double>& w) {
  constexpr int kCache = 32;
  static std::once_flag once;
  static std::vector<std::vector<double>> cx, cw;
  std::call_once(once, [] {
    cx.resize(kCache + 1);
    cw.resize(kCache + 1);
    for (int k = 1; k <= kCache; ++k) gauss_rule_compute(k, cx[k], cw[k]);
  });
  if (q >= 1 && q <= kCache) {
    x = cx[q];
    w = cw[q];
    return;
  }
  gauss_rule_compute(q, x, w);
}

void lagrange_eval(const std::vector<double>& nodes, double t, double* out) {
  int n = (int)nodes.size();
  for (int i = 0; i < n; ++i) {
    double v = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != i) v *= (t - nodes[j]) / (nodes[i] - nodes[j]);
    out[i] = v;
  }
}

void lagrange_deriv(const std::vector<double>& nodes, double t, double* out) {
  int n = (int)nodes.size();
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int m = 0; m < n; ++m) {
      if (m == i) continue;
      double v = 1.0 / (nodes[i] - nodes[m]);
      for (int j = 0; j < n; ++j)
        if (j != i && j != m) v *= (t - nodes[j]) / (nodes[i] - nodes[j]);
      s += v;
    }
    out[i] = s;
  }
}

static void invert(std::vector<double> A, int n, std::vector<double>& inv) {
  inv.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    for (int j = 0; j < n; ++j) {
      std::swap(A[c * n + j], A[piv * n + j]);
      std::swap(inv[c * n + j], inv[piv * n + j]);
    }
    double d = 1.0 / A[c * n + c];
    for (int j = 0; j < n; ++j) { A[c * n + j] *= d; inv[c * n + j] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) { A[r * n + j] -= f * A[c * n + j]; inv[r * n + j] -= f * inv[c * n + j]; }
    }
  }
}

static Basis1D make_basis(int p) {
  Basis1D b;
  b.p = p;
  int n = p + 1;
  b.x.assign(n, 0.0);
  b.x[0] = 0.0;
  b.x[p] = 1.0;
  for (int j = 1; j < p; ++j) {
    double t = -std::cos(M_PI * j / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP, d2P;
      legendre(p, t, P, dP, d2P);
      double dt = dP / d2P;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    b.x[j] = 0.5 * (t + 1.0);
  }
  for (int j = 1; j < (p + 1) / 2; ++j) {
    double a = 0.5 * (b.x[j] + (1.0 - b.x[p - j]));
    b.x[j] = a;
    b.x[p - j] = 1.0 - a;
  }
  if (p % 2 == 0) b.x[p / 2] = 0.5;
  std::vector<double> gx, gw;
  gauss_rule(p + 1, gx, gw);
  b.M.assign(n * n, 0.0);
  b.K.assign(n * n, 0.0);
  std::vector<double> L(n), D(n);
  for (int g = 0; g < p + 1; ++g) {
    lagrange_eval(b.x, gx[g], L.data());
    lagrange_deriv(b.x, gx[g], D.data());
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        b.M[i * n + j] += gw[g] * L[i] * L[j];
        b.K[i * n + j] += gw[g] * D[i] * D[j];
      }
  }
  invert(b.M, n, b.Minv);
  b.D0.assign(n, 0.0);
  b.D1.assign(n, 0.0);
  lagrange_deriv(b.x, 0.0, b.D0.data());
  lagrange_deriv(b.x, 1.0, b.D1.data());
  return b;
}

const Basis1D& basis(int p) {
  static std::once_flag once;
  static std::vector<Basis1D> table;
  std::call_once(once, [] {
    table.resize(kMaxP + 1);
    for (int q = 1; q <= kMaxP; ++q) table[q] = make_basis(q);
  });
  if (p < 1 || p > kMaxP) throw Error(-1, "degree out of range");
  return table[p];
}

}  // namespace hpdg
