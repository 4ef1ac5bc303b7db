/* The C-ABI used from C alone (no Python, no torch).  The matrix is the
 * tridiagonal Toeplitz matrix T = tridiag(-1, 2, -1) of order n = 200, given
 * by its upper triangle; its eigenvalues are 2 - 2 cos(j pi / (n + 1)).
 *   1. hyeig_spmm_sym on an n x 8 FP64 block, against the product formed here
 *      on the host (2 x_i - x_{i-1} - x_{i+1});
 *   2. hyeig_solve_lowest_k (LOBPCG, plain FP64 form) for the 4 lowest pairs,
 *      against the closed form.
 * Exit status 0 when both hold. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "hyeig.h"

#define CHECK_HIP(x)                                                  \
  do {                                                                \
    if ((x) != hipSuccess) {                                          \
      fprintf(stderr, "HIP error at %s:%d\n", __FILE__, __LINE__);   \
      return 2;                                                       \
    }                                                                 \
  } while (0)
#define CHECK_HY(ctx, x)                                                              \
  do {                                                                                \
    hyeig_status s_ = (x);                                                            \
    if (s_ != HYEIG_OK) {                                                             \
      fprintf(stderr, "hyeig status %d at line %d: %s\n", (int)s_, __LINE__,         \
              hyeig_last_error(ctx));                                                 \
      return 3;                                                                       \
    }                                                                                 \
  } while (0)

int main(void) {
  const int64_t n = 200;
  const int m = 8, k = 4, nb = 8;
  const double pi = 3.14159265358979323846;
  /* upper-triangle CSR: diagonal first, then the superdiagonal */
  const int64_t nnz = 2 * n - 1;
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
  int32_t* ci = (int32_t*)malloc(sizeof(int32_t) * nnz);
  float* va = (float*)malloc(sizeof(float) * nnz);
  int64_t e = 0;
  for (int64_t i = 0; i < n; ++i) {
    rp[i] = e;
    ci[e] = (int32_t)i;
    va[e++] = 2.0f;
    if (i + 1 < n) {
      ci[e] = (int32_t)(i + 1);
      va[e++] = -1.0f;
    }
  }
  rp[n] = e;

  hyeig_ctx* ctx = NULL;
  if (hyeig_ctx_create(0, NULL, &ctx) != HYEIG_OK) {
    fprintf(stderr, "no context\n");
    return 2;
  }
  int64_t* d_rp;
  int32_t* d_ci;
  float* d_va;
  CHECK_HIP(hipMalloc((void**)&d_rp, sizeof(int64_t) * (n + 1)));
  CHECK_HIP(hipMalloc((void**)&d_ci, sizeof(int32_t) * nnz));
  CHECK_HIP(hipMalloc((void**)&d_va, sizeof(float) * nnz));
  CHECK_HIP(hipMemcpy(d_rp, rp, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(d_ci, ci, sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(d_va, va, sizeof(float) * nnz, hipMemcpyHostToDevice));
  hyeig_mat* H = NULL;
  CHECK_HY(ctx, hyeig_mat_create(ctx, n, nnz, d_rp, d_ci, d_va, HYEIG_F32, HYEIG_MAT_VALIDATE, &H));

  /* 1. the product */
  double* X = (double*)malloc(sizeof(double) * n * m);
  double* Y = (double*)malloc(sizeof(double) * n * m);
  uint64_t s = 12345u;
  for (int64_t i = 0; i < n * m; ++i) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    X[i] = (double)(s >> 11) / 9007199254740992.0 - 0.5;
  }
  double *d_X, *d_Y;
  CHECK_HIP(hipMalloc((void**)&d_X, sizeof(double) * n * m));
  CHECK_HIP(hipMalloc((void**)&d_Y, sizeof(double) * n * m));
  CHECK_HIP(hipMemcpy(d_X, X, sizeof(double) * n * m, hipMemcpyHostToDevice));
  CHECK_HY(ctx, hyeig_spmm_sym(ctx, H, m, d_X, m, HYEIG_F64, d_Y, m, HYEIG_F64, HYEIG_F64, HYEIG_F32));
  CHECK_HIP(hipMemcpy(Y, d_Y, sizeof(double) * n * m, hipMemcpyDeviceToHost));
  double perr = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) {
      double r = 2.0 * X[i * m + j] - (i > 0 ? X[(i - 1) * m + j] : 0.0) - (i + 1 < n ? X[(i + 1) * m + j] : 0.0);
      double d = fabs(Y[i * m + j] - r);
      if (d > perr) perr = d;
    }
  printf("product: max |error| %.3g\n", perr);

  /* 2. the lowest 4 pairs */
  float* X0 = (float*)malloc(sizeof(float) * n * nb);
  for (int64_t i = 0; i < n * nb; ++i) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    X0[i] = (float)((double)(s >> 11) / 9007199254740992.0 - 0.5);
  }
  float* d_X0;
  CHECK_HIP(hipMalloc((void**)&d_X0, sizeof(float) * n * nb));
  CHECK_HIP(hipMemcpy(d_X0, X0, sizeof(float) * n * nb, hipMemcpyHostToDevice));
  hyeig_params p;
  hyeig_params_default(&p);
  p.k = k;
  p.nb = nb;
  p.method = HYEIG_LOBPCG;
  p.tol = 1e-6;
  p.hnorm = 2.0 + 2.0 * cos(pi / (double)(n + 1));
  p.maxiter = 2000;
  p.precision = HYEIG_PREC_PLAIN_F64;
  double ev[4], rs[4];
  hyeig_report rep;
  rep.hist = NULL;
  rep.hist_t = NULL;
  rep.hist_cap = 0;
  CHECK_HY(ctx, hyeig_solve_lowest_k(ctx, H, &p, d_X0, nb, ev, rs, &rep));
  /* each Ritz value lies within ||r||^2 / gap of its eigenvalue (the gap to the
     neighbouring eigenvalues, known here in closed form) */
  int ok = 1;
  double eerr = 0.0;
  for (int j = 0; j < k; ++j) {
    double lam = 2.0 - 2.0 * cos((j + 1) * pi / (double)(n + 1));
    double up = 2.0 - 2.0 * cos((j + 2) * pi / (double)(n + 1));
    double gap = up - lam;
    if (j > 0) {
      double lo = 2.0 - 2.0 * cos(j * pi / (double)(n + 1));
      if (lam - lo < gap) gap = lam - lo;
    }
    double r = rs[j] * p.hnorm;
    double d = fabs(ev[j] - lam);
    printf("lambda_%d = %.15f (closed form %.15f), residual %.2e, error %.2e, bound %.2e\n", j + 1, ev[j], lam,
           rs[j], d, 2.0 * r * r / gap + 1e-15);
    if (d > 2.0 * r * r / gap + 1e-15 || rs[j] > 1e-6) ok = 0;
    if (d > eerr) eerr = d;
  }
  printf("solve: %d iterations, max |eigenvalue error| %.3g\n", rep.iters_front, eerr);

  hyeig_mat_destroy(H);
  hyeig_ctx_destroy(ctx);
  hipFree(d_rp);
  hipFree(d_ci);
  hipFree(d_va);
  hipFree(d_X);
  hipFree(d_Y);
  hipFree(d_X0);
  free(rp);
  free(ci);
  free(va);
  free(X);
  free(Y);
  free(X0);
  return (perr <= 1e-14 && ok) ? 0 : 1;
}
