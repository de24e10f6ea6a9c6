/* Plain float64 CSR kernels for the CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * y = A x with A in CSR, accumulated in float64 in column order, one row at
 * a time (the plain definition of y = Ax, eq. 1), and the transposed product
 * y = A^T g accumulated row by row.  The row loop of the forward product is
 * split across OpenMP threads; each row's sum is independent of the thread
 * count.  Nothing here is tuned: it is the reference and the CPU baseline.
 */
#include <stdint.h>
#include <omp.h>

void oracle_csr_spmv(int64_t n, const int64_t *rowptr, const int32_t *col,
                     const double *val, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double t = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) t += val[e] * x[col[e]];
    y[i] = t;
  }
}

void oracle_csr_spmv_t(int64_t n, int64_t m, const int64_t *rowptr,
                       const int32_t *col, const double *val, const double *g,
                       double *y) {
  for (int64_t j = 0; j < m; ++j) y[j] = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) y[col[e]] += val[e] * g[i];
}

void oracle_set_num_threads(int t) { omp_set_num_threads(t); }

int oracle_num_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    t = omp_get_num_threads();
  }
  return t;
}
