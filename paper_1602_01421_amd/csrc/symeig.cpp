// Small dense symmetric eigensolver for the projected problem (the paper's
// step "solve the projected eigenproblem", which it hands to LAPACK-class
// code).  m <= a few hundred, FP64, host.
//
// Method: Householder reduction to tridiagonal form with the reflections
// accumulated, then the symmetric QR algorithm on the tridiagonal matrix:
// implicit steps with the Wilkinson shift, each a chain of Givens rotations
// that chases the bulge down the diagonal, with deflation of negligible
// off-diagonal entries (Francis' implicit shifted QR; Golub and Van Loan,
// Matrix Computations, the symmetric QR algorithm section), the rotations
// accumulated into the eigenvector basis.
#include <cmath>
#include <cstring>
#include <vector>

#include "fe_internal.h"

namespace fe {

// a: n x n row-major symmetric (destroyed).  w: eigenvalues (unordered),
// z: n x n row-major, column j = eigenvector of w[j].  Returns false if the
// QR iteration did not converge.
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
  // --- symmetric QR on the tridiagonal (d, e)
  const double eps = 2.220446049250313e-16;
  const int max_steps = 60 * n + 60;
  int steps = 0;
  for (;;) {
    // deflate: off-diagonal entries below rounding relative to their
    // neighbours are set to zero
    for (int i = 0; i + 1 < n; ++i)
      if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    // the last unreduced block [lo, hi]: hi is the largest index with a
    // nonzero coupling to its predecessor, lo the start of that run
    int hi = n - 1;
    while (hi > 0 && e[hi - 1] == 0.0) --hi;
    if (hi == 0) break;  // diagonal
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++steps > max_steps) return false;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer to
    // its last diagonal entry
    const double half = 0.5 * (d[hi - 1] - d[hi]);
    const double off2 = e[hi - 1] * e[hi - 1];
    const double den = half + (half >= 0.0 ? 1.0 : -1.0) * std::hypot(half, e[hi - 1]);
    const double mu = d[hi] - (den != 0.0 ? off2 / den : 0.0);
    // implicit step: the first rotation is that of the first column of
    // T - mu I; each later one removes the bulge the previous one created
    double x = d[lo] - mu, y = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, y);
      const double c = r != 0.0 ? x / r : 1.0, sn = r != 0.0 ? y / r : 0.0;
      if (k > lo) e[k - 1] = r;
      // rows/columns k, k+1 of the 2 x 2 block [[a, b], [b, q]] <- R M R^T
      const double a = d[k], b = e[k], q = d[k + 1];
      const double cs = c * sn;
      d[k] = c * c * a + 2.0 * cs * b + sn * sn * q;
      d[k + 1] = sn * sn * a - 2.0 * cs * b + c * c * q;
      e[k] = cs * (q - a) + (c * c - sn * sn) * b;
      if (k + 1 < hi) {  // the new bulge sits at (k, k + 2)
        y = sn * e[k + 1];
        e[k + 1] *= c;
        x = e[k];
      }
      for (int row = 0; row < n; ++row) {  // Z <- Z R^T on columns k, k+1
        const double zk = Z(row, k), zk1 = Z(row, k + 1);
        Z(row, k) = c * zk + sn * zk1;
        Z(row, k + 1) = c * zk1 - sn * zk;
      }
    }
  }
  for (int i = 0; i < n; ++i) w[i] = d[i];
  return true;
}

}  // namespace fe

extern "C" fe_status fe_dense_symeig(int32_t n, const double* a, double* w, double* z) {
  if (n < 1 || !a || !w || !z) return fe::fail(FE_EINVAL, "fe_dense_symeig: bad arguments");
  std::vector<double> tmp(a, a + (size_t)n * n);
  if (!fe::sym_eig(n, tmp.data(), w, z)) return fe::fail(FE_ENOCONV, "fe_dense_symeig: QR iteration did not converge");
  return FE_OK;
}
