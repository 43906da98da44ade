// 1D tables of the nodal tensor-product basis (host code).
//
// Basis: Lagrange polynomials through the Legendre-Gauss-Lobatto nodes of
// degree k (Sec. 3.1); quadrature: Gauss-Legendre with nq points (Sec. 5).
// Nodes and points come from Newton's method on the Legendre three-term
// recurrence in long double; Lagrange values and derivatives from the
// barycentric form (Berrut & Trefethen, SIAM Review 46, 2004).
#include <cmath>

#include "internal.h"

namespace dgmf {

namespace {
using ld = long double;
const ld kPi = 3.141592653589793238462643383279502884L;

// P_n(x) and P_n'(x) by the recurrence (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}.
void legendre(int n, ld x, ld& p, ld& dp) {
  ld p0 = 1, p1 = x;
  if (n == 0) { p = 1; dp = 0; return; }
  for (int m = 1; m < n; ++m) {
    ld p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // derivative from (x^2 - 1) P_n' = n (x P_n - P_{n-1}); callers avoid |x| = 1
  dp = n * (x * p1 - p0) / (x * x - 1);
}
}  // namespace

void gauss_legendre01(int nq, std::vector<double>& x, std::vector<double>& w) {
  x.assign(nq, 0.0);
  w.assign(nq, 0.0);
  for (int i = 0; i < nq; ++i) {
    ld t = std::cos(kPi * (i + 0.75L) / (nq + 0.5L));
    ld p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(nq, t, p, dp);
      ld dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-22L) break;
    }
    legendre(nq, t, p, dp);
    ld wt = 2 / ((1 - t * t) * dp * dp);
    // t runs from +1 down to -1; map to [0,1] ascending
    x[nq - 1 - i] = static_cast<double>((t + 1) / 2);
    w[nq - 1 - i] = static_cast<double>(wt / 2);
  }
}

void gll_nodes01(int k, std::vector<double>& x) {
  x.assign(k + 1, 0.0);
  x[0] = 0.0;
  x[k] = 1.0;
  for (int i = 1; i < k; ++i) {
    ld t = -std::cos(kPi * i / k);
    for (int it = 0; it < 100; ++it) {
      ld p, dp;
      legendre(k, t, p, dp);
      // P_k'' from Legendre's equation (1 - t^2) P'' = 2 t P' - k (k+1) P
      ld ddp = (2 * t * dp - k * (k + 1) * p) / (1 - t * t);
      ld dt = dp / ddp;
      t -= dt;
      if (std::fabs(dt) < 1e-22L) break;
    }
    x[i] = static_cast<double>((t + 1) / 2);
  }
}

void lagrange_eval(const std::vector<double>& nodes, double xd, double* val, double* der) {
  const int n = static_cast<int>(nodes.size());
  std::vector<ld> bw(n, 1.0L);
  for (int j = 0; j < n; ++j)
    for (int m = 0; m < n; ++m)
      if (m != j) bw[j] /= (static_cast<ld>(nodes[j]) - nodes[m]);
  const ld x = xd;
  int at = -1;
  for (int j = 0; j < n; ++j)
    if (x == static_cast<ld>(nodes[j])) at = j;
  if (at >= 0) {
    // at a node: cardinal values; derivative matrix row of the barycentric form
    ld diag = 0;
    for (int j = 0; j < n; ++j) {
      if (val) val[j] = (j == at) ? 1.0 : 0.0;
      if (j != at) {
        ld dj = (bw[j] / bw[at]) / (x - static_cast<ld>(nodes[j]));
        if (der) der[j] = static_cast<double>(dj);
        diag -= dj;
      }
    }
    if (der) der[at] = static_cast<double>(diag);
    return;
  }
  ld L = 1;
  for (int m = 0; m < n; ++m) L *= (x - static_cast<ld>(nodes[m]));
  for (int j = 0; j < n; ++j) {
    ld lj = L * bw[j] / (x - static_cast<ld>(nodes[j]));
    ld s = 0;
    for (int m = 0; m < n; ++m)
      if (m != j) s += 1 / (x - static_cast<ld>(nodes[m]));
    if (val) val[j] = static_cast<double>(lj);
    if (der) der[j] = static_cast<double>(lj * s);
  }
}

void make_tables(int k, int nq, Tables1D& t) {
  t.k = k;
  t.n = k + 1;
  t.nq = nq;
  const int n = t.n;
  gll_nodes01(k, t.nodes);
  gauss_legendre01(nq, t.xq, t.wq);
  t.S.assign(nq * n, 0.0);
  t.D.assign(nq * n, 0.0);
  for (int q = 0; q < nq; ++q) lagrange_eval(t.nodes, t.xq[q], &t.S[q * n], &t.D[q * n]);
  t.Mhat.assign(n * n, 0.0);
  t.Khat.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      ld m = 0, kk = 0;
      for (int q = 0; q < nq; ++q) {
        m += static_cast<ld>(t.wq[q]) * t.S[q * n + i] * t.S[q * n + j];
        kk += static_cast<ld>(t.wq[q]) * t.D[q * n + i] * t.D[q * n + j];
      }
      t.Mhat[i * n + j] = static_cast<double>(m);
      t.Khat[i * n + j] = static_cast<double>(kk);
    }
  t.g0.assign(n, 0.0);
  t.g1.assign(n, 0.0);
  lagrange_eval(t.nodes, 0.0, nullptr, t.g0.data());
  lagrange_eval(t.nodes, 1.0, nullptr, t.g1.data());
  t.gll_w.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    ld s = 0;
    for (int q = 0; q < nq; ++q) s += static_cast<ld>(t.wq[q]) * t.S[q * n + j];
    t.gll_w[j] = static_cast<double>(s);
  }
}

}  // namespace dgmf
