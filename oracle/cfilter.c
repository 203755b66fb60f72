/*
 * FP64 Chebyshev filter in plain C with OpenMP (Sec. 2.2, Step 1; Sec. 3.2).
 *
 * TEST INFRASTRUCTURE ONLY: the multi-core twin of chebyshev.filter_recurrence, used to time
 * the oracle on all host cores and to compute expected values of large cases.  It shares no
 * code with the HIP library.
 *
 * Given a sparse matrix M (the scaled Laplacian L~ = (2 / lmax) L - I, built by the Python
 * oracle) in CSR form and an n x w row-major block X, it computes
 *     Y = sum_{j=0..m} a_j T_j(M) X
 * by the three-term recurrence Z_0 = X, Z_1 = M X, Z_{j+1} = 2 M Z_j - Z_{j-1}, with the
 * same FP64 operations in the same order as the Python oracle: each row of a product is a
 * sum over the row's stored entries in storage order, starting from zero.  Rows are split
 * among threads; a row's arithmetic does not depend on the split, so the result is the same
 * for any number of threads.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* out[i, :] = sum_e val[e] z[col[e], :] over the entries e of row i */
static void spmm(int64_t n, int w, const int64_t *rowptr, const int32_t *col, const double *val,
                 const double *z, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double *o = out + i * w;
    for (int c = 0; c < w; ++c) o[c] = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const double v = val[e];
      const double *zr = z + (int64_t)col[e] * w;
      for (int c = 0; c < w; ++c) o[c] += v * zr[c];
    }
  }
}

/* Returns the number of threads used, or -1 when memory runs out.  threads <= 0: OpenMP's
 * default (all cores unless OMP_NUM_THREADS says otherwise). */
int oracle_cheb_filter(int64_t n, int w, const int64_t *rowptr, const int32_t *col,
                       const double *val, int m, const double *a, const double *X, double *Y,
                       int threads) {
  if (threads > 0) omp_set_num_threads(threads);
  const int used = omp_get_max_threads();
  const int64_t sz = n * (int64_t)w;
  double *zp = malloc(sizeof(double) * (size_t)(sz > 0 ? sz : 1));
  double *zc = malloc(sizeof(double) * (size_t)(sz > 0 ? sz : 1));
  double *zn = malloc(sizeof(double) * (size_t)(sz > 0 ? sz : 1));
  if (!zp || !zc || !zn) {
    free(zp);
    free(zc);
    free(zn);
    return -1;
  }
  memcpy(zp, X, sizeof(double) * (size_t)sz);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < sz; ++i) Y[i] = a[0] * zp[i];
  if (m >= 1) {
    spmm(n, w, rowptr, col, val, zp, zc);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < sz; ++i) Y[i] = Y[i] + a[1] * zc[i];
    for (int j = 1; j < m; ++j) {
      spmm(n, w, rowptr, col, val, zc, zn);
      const double aj = a[j + 1];
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < sz; ++i) {
        zn[i] = 2.0 * zn[i] - zp[i];
        Y[i] = Y[i] + aj * zn[i];
      }
      double *t = zp;
      zp = zc;
      zc = zn;
      zn = t;
    }
  }
  free(zp);
  free(zc);
  free(zn);
  return used;
}
