// Small dense symmetric eigensolver for the projected problem (the paper's
// step "solve the projected eigenproblem", which it hands to LAPACK-class
// code).  m <= a few hundred, FP64, host.
//
// Method: Householder reduction to tridiagonal form with the reflections
// accumulated, then the QL iteration with implicit Wilkinson-type shifts on
// the tridiagonal matrix, rotating the accumulated basis along.
#include <cmath>
#include <cstring>
#include <vector>

#include "fe_internal.h"

namespace fe {

// a: n x n row-major symmetric (destroyed).  w: eigenvalues (unordered),
// z: n x n row-major, column j = eigenvector of w[j].  Returns false if the
// QL iteration did not converge.
bool sym_eig(int n, double* a, double* w, double* z) {
  auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };
  auto Z = [&](int i, int j) -> double& { return z[(size_t)i * n + j]; };
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Z(i, j) = (i == j) ? 1.0 : 0.0;
  std::vector<double> v(n), t(n);
  // --- Householder: zero A[k+2:, k] for k = 0..n-3
  for (int k = 0; k + 2 < n; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < n; ++i) xn += A(i, k) * A(i, k);
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double alpha = (A(k + 1, k) > 0.0) ? -xn : xn;
    for (int i = 0; i < n; ++i) v[i] = (i > k) ? A(i, k) : 0.0;
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
    if (vn == 0.0) continue;
    const double beta = 2.0 / vn;
    // A <- A H : t = A v ; A -= beta t v^T
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += A(i, j) * v[j];
      t[i] = s;
    }
    for (int i = 0; i < n; ++i)
      for (int j = k + 1; j < n; ++j) A(i, j) -= beta * t[i] * v[j];
    // A <- H A : t = v^T A ; A -= beta v t^T
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += v[i] * A(i, j);
      t[j] = s;
    }
    for (int i = k + 1; i < n; ++i)
      for (int j = 0; j < n; ++j) A(i, j) -= beta * v[i] * t[j];
    // Z <- Z H
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += Z(i, j) * v[j];
      t[i] = s;
    }
    for (int i = 0; i < n; ++i)
      for (int j = k + 1; j < n; ++j) Z(i, j) -= beta * t[i] * v[j];
  }
  // tridiagonal: d = diagonal, e[i] couples i and i+1
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = 0.5 * (A(i + 1, i) + A(i, i + 1));
  // --- QL with implicit shifts
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    int m;
    do {
      for (m = l; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m != l) {
        if (++iter > 60) return false;
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = std::hypot(g, 1.0);
        g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
        double s = 1.0, c = 1.0, p = 0.0;
        int i;
        bool early = false;
        for (i = m - 1; i >= l; --i) {
          double f = s * e[i], bb = c * e[i];
          r = std::hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) {
            d[i + 1] -= p;
            e[m] = 0.0;
            early = true;
            break;
          }
          s = f / r;
          c = g / r;
          g = d[i + 1] - p;
          r = (d[i] - g) * s + 2.0 * c * bb;
          p = s * r;
          d[i + 1] = g + p;
          g = c * r - bb;
          for (int k = 0; k < n; ++k) {
            f = Z(k, i + 1);
            Z(k, i + 1) = s * Z(k, i) + c * f;
            Z(k, i) = c * Z(k, i) - s * f;
          }
        }
        if (early) continue;
        d[l] -= p;
        e[l] = g;
        e[m] = 0.0;
      }
    } while (m != l);
  }
  for (int i = 0; i < n; ++i) w[i] = d[i];
  return true;
}

}  // namespace fe

extern "C" fe_status fe_dense_symeig(int32_t n, const double* a, double* w, double* z) {
  if (n < 1 || !a || !w || !z) return fe::fail(FE_EINVAL, "fe_dense_symeig: bad arguments");
  std::vector<double> tmp(a, a + (size_t)n * n);
  if (!fe::sym_eig(n, tmp.data(), w, z)) return fe::fail(FE_ENOCONV, "fe_dense_symeig: QL did not converge");
  return FE_OK;
}
