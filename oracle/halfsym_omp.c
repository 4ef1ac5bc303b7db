/*
 * Plain FP64 product with a half-stored symmetric matrix, on all host threads.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Nothing here is shared
 * with the GPU library.
 *
 * H = U + U^T - diag(U), U the upper triangle including the diagonal, given as
 * CSR (int64 row pointers, int32 column indices, FP32 values, which are
 * promoted exactly to FP64).  Section 3.1 of the paper stores its matrices by
 * half and Section 2.3 makes H W the only product of a LOBPCG iteration.
 *
 * Written out from the definition
 *     y_i = sum_{j >= i} u_ij x_j  +  sum_{k < i} u_ki x_k,
 * with the second sum read from L, the strictly lower triangle (the transpose
 * of U without its diagonal), stored as CSR by half_lower().  Every output row
 * is then an independent sum, so rows are shared out among OpenMP threads and
 * no two threads write the same element.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* L = strict lower triangle of H: entry (k, i) of U with k < i becomes entry
 * (i, k) of L.  lrowptr[n+1], lcol[nnz_l], lval[nnz_l] allocated by the caller
 * (nnz_l = nnz(U) minus the stored diagonal entries, at most nnz(U)).  Columns
 * of each row of L come out ascending (U is walked row by row). */
int64_t half_lower(int64_t n, const int64_t* rowptr, const int32_t* colidx, const float* vals, int64_t* lrowptr,
                   int32_t* lcol, float* lval) {
  memset(lrowptr, 0, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t k = 0; k < n; ++k)
    for (int64_t p = rowptr[k]; p < rowptr[k + 1]; ++p)
      if ((int64_t)colidx[p] != k) lrowptr[colidx[p] + 1]++;
  for (int64_t i = 0; i < n; ++i) lrowptr[i + 1] += lrowptr[i];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!fill) return -1;
  memcpy(fill, lrowptr, sizeof(int64_t) * (size_t)n);
  for (int64_t k = 0; k < n; ++k)
    for (int64_t p = rowptr[k]; p < rowptr[k + 1]; ++p) {
      const int64_t i = colidx[p];
      if (i == k) continue;
      const int64_t q = fill[i]++;
      lcol[q] = (int32_t)k;
      lval[q] = vals[p];
    }
  free(fill);
  return lrowptr[n];
}

/* Y = H X: X and Y row-major n x m (leading dimensions ldx, ldy), FP64.
 * nthreads <= 0: OpenMP's default. */
void half_matmul(int64_t n, const int64_t* rowptr, const int32_t* colidx, const float* vals, const int64_t* lrowptr,
                 const int32_t* lcol, const float* lval, int m, const double* X, int64_t ldx, double* Y,
                 int64_t ldy, int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
  {
    double* acc = (double*)malloc(sizeof(double) * (size_t)m);
#pragma omp for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
      for (int j = 0; j < m; ++j) acc[j] = 0.0;
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const double u = (double)vals[p];
        const double* x = X + (int64_t)colidx[p] * ldx;
        for (int j = 0; j < m; ++j) acc[j] += u * x[j];
      }
      for (int64_t p = lrowptr[i]; p < lrowptr[i + 1]; ++p) {
        const double u = (double)lval[p];
        const double* x = X + (int64_t)lcol[p] * ldx;
        for (int j = 0; j < m; ++j) acc[j] += u * x[j];
      }
      double* y = Y + i * ldy;
      for (int j = 0; j < m; ++j) y[j] = acc[j];
    }
    free(acc);
  }
}

/* threads an OpenMP parallel region gets by default */
int half_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    t = omp_get_num_threads();
  }
  return t;
}
