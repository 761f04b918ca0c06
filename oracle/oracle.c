/*
 * CPU oracle, compiled part.  TEST INFRASTRUCTURE ONLY: nothing in the GPU
 * library links, includes or calls this file.  It exists so that tests, the
 * smoke check and the CPU baseline leg of the benchmark can compare the GPU
 * results against a plain, obviously correct FP64 computation.
 *
 *   oracle_spmm    -- Y = A*X for a 0/1 pattern matrix in CSR: each nonzero
 *                     (i, j) adds row j of X into row i of Y (the sparse matrix
 *                     multiplication section; its execution subsection states
 *                     the per-nonzero row add).  Summation in ascending j, FP64.
 *                     threads > 1 only splits rows between OpenMP threads; the
 *                     per-row summation order is unchanged, so the result is
 *                     bitwise identical for every thread count.
 *   oracle_csr_build -- the pattern CSR of an edge stream by its definition
 *                     (the sparse matrix format section: no values; symmetric
 *                     for an undirected graph): every pair (u, v) gives (u, v)
 *                     and (v, u), self-loops are dropped, each row's columns are
 *                     sorted ascending and repeats merged.  OpenMP splits the
 *                     counting and the per-row sorting; the result does not
 *                     depend on the thread count.
 *   oracle_jacobi  -- cyclic-by-row Jacobi eigenvalue algorithm for a dense
 *                     symmetric matrix (Golub & Van Loan, Matrix Computations,
 *                     the symmetric Jacobi section): the brute-force check of
 *                     spectra for small graphs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void oracle_spmm(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *X,
                 int32_t b, double *Y, int32_t threads) {
#ifdef _OPENMP
  if (threads < 1) threads = 1;
#pragma omp parallel for schedule(dynamic, 1024) num_threads(threads)
#endif
  for (int64_t i = 0; i < n; ++i) {
    double *y = Y + i * (int64_t)b;
    for (int32_t c = 0; c < b; ++c) y[c] = 0.0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const double *x = X + (int64_t)col[e] * b;
      for (int32_t c = 0; c < b; ++c) y[c] += x[c];
    }
  }
}

static int cmp_i32(const void *a, const void *b) {
  const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* row_ptr: n+1 entries; col: room for 2*m entries.  Returns nnz, or -1 when
 * the scratch allocation fails. */
int64_t oracle_csr_build(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                         int64_t *row_ptr, int32_t *col, int32_t threads) {
  if (threads < 1) threads = 1;
  int64_t *cnt = calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *raw = malloc(sizeof(int32_t) * (size_t)(2 * m > 0 ? 2 * m : 1));
  int64_t *cur = malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!cnt || !raw || !cur) {
    free(cnt);
    free(raw);
    free(cur);
    return -1;
  }
#pragma omp parallel for schedule(static) num_threads(threads)
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] == dst[e]) continue;
#pragma omp atomic
    cnt[src[e]]++;
#pragma omp atomic
    cnt[dst[e]]++;
  }
  int64_t acc = 0;
  for (int64_t i = 0; i < n; ++i) {
    cur[i] = acc;
    acc += cnt[i];
  }
  cur[n] = acc;
  for (int64_t i = 0; i <= n; ++i) cnt[i] = cur[i]; /* cnt = raw row starts */
#pragma omp parallel for schedule(static) num_threads(threads)
  for (int64_t e = 0; e < m; ++e) {
    const int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    int64_t p, q;
#pragma omp atomic capture
    p = cur[u]++;
#pragma omp atomic capture
    q = cur[v]++;
    raw[p] = v;
    raw[q] = u;
  }
  /* sort each row, merge repeats; cur[i] = distinct count of row i */
#pragma omp parallel for schedule(dynamic, 4096) num_threads(threads)
  for (int64_t i = 0; i < n; ++i) {
    int32_t *r = raw + cnt[i];
    const int64_t len = cnt[i + 1] - cnt[i];
    qsort(r, (size_t)len, sizeof(int32_t), cmp_i32);
    int64_t k = 0;
    for (int64_t t = 0; t < len; ++t)
      if (k == 0 || r[t] != r[k - 1]) r[k++] = r[t];
    cur[i] = k;
  }
  row_ptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cur[i];
#pragma omp parallel for schedule(dynamic, 4096) num_threads(threads)
  for (int64_t i = 0; i < n; ++i)
    memcpy(col + row_ptr[i], raw + cnt[i], sizeof(int32_t) * (size_t)cur[i]);
  free(cnt);
  free(raw);
  free(cur);
  return row_ptr[n];
}

int32_t oracle_max_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* off(A)^2: sum of squares of the off-diagonal entries. */
static double off2(const double *A, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (i != j) s += A[i * n + j] * A[i * n + j];
  return s;
}

/*
 * A (n x n, row-major, symmetric) is overwritten; on return its diagonal holds
 * the eigenvalues and V (n x n, row-major) the eigenvectors as columns.
 * Sweeps visit (p, q), p < q, in row order; each step zeroes A[p][q] with the
 * rotation whose tangent is the smaller root of t^2 + 2*tau*t - 1 = 0,
 * tau = (A[q][q] - A[p][p]) / (2 A[p][q]).  Stops when
 * off(A) <= tol * ||A||_F or after max_sweeps.  Returns the number of sweeps.
 */
int32_t oracle_jacobi(int32_t n, double *A, double *V, double tol, int32_t max_sweeps) {
  double fro2 = 0.0;
  for (int64_t i = 0; i < (int64_t)n * n; ++i) fro2 += A[i] * A[i];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  int sweep = 0;
  while (sweep < max_sweeps && off2(A, n) > tol * tol * fro2) {
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                : -1.0 / (-tau + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        /* A <- J^T A J with J the identity except J[p][p]=J[q][q]=c, J[p][q]=s, J[q][p]=-s */
        for (int k = 0; k < n; ++k) { /* columns p, q: A <- A J */
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) { /* rows p, q: A <- J^T A */
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) { /* V <- V J */
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
    }
    ++sweep;
  }
  return sweep;
}
