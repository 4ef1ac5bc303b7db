// Host driver for the small dense FP64 solvers of libhyeig (csrc/smalldense.cpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_smalldense_sanitized.py.  Every routine runs on seeded random
// inputs and edge cases (order 1, clustered and repeated eigenvalues, a
// singular DIIS Gram matrix, a non-positive-definite Cholesky input, a band
// matrix at its width limits); each result is checked against its defining
// identity, and the program exits non-zero on the first failure.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2305_15552_amd/csrc/internal.h"

namespace {

int failures = 0;

void check(bool ok, const char* what, int k) {
  if (!ok) {
    std::printf("FAIL %s (order %d)\n", what, k);
    ++failures;
  }
}

std::vector<double> random_sym(int k, std::mt19937_64& rng, double diag_shift = 0.0) {
  std::normal_distribution<double> N(0.0, 1.0);
  std::vector<double> A((size_t)k * k);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i <= j; ++i) {
      const double v = N(rng);
      A[i + (size_t)j * k] = v;
      A[j + (size_t)i * k] = v;
    }
  for (int i = 0; i < k; ++i) A[i + (size_t)i * k] += diag_shift;
  return A;
}

// max |A V - V diag(w)| / ||A||_max and max |V^T V - I|
void eig_residuals(int k, const std::vector<double>& A, const double* w, const double* V, int want, double* res,
                   double* orth) {
  double amax = 1e-300;
  for (double a : A) amax = std::max(amax, std::fabs(a));
  *res = 0.0;
  *orth = 0.0;
  for (int c = 0; c < want; ++c) {
    for (int i = 0; i < k; ++i) {
      double t = -w[c] * V[i + (size_t)c * k];
      for (int j = 0; j < k; ++j) t += A[i + (size_t)j * k] * V[j + (size_t)c * k];
      *res = std::max(*res, std::fabs(t) / amax);
    }
    for (int d = 0; d < want; ++d) {
      double t = (c == d) ? -1.0 : 0.0;
      for (int i = 0; i < k; ++i) t += V[i + (size_t)c * k] * V[i + (size_t)d * k];
      *orth = std::max(*orth, std::fabs(t));
    }
  }
}

}  // namespace

int main() {
  std::mt19937_64 rng(20261203);
  std::normal_distribution<double> N(0.0, 1.0);

  // symmetric eigenproblem: random, order 1, repeated eigenvalues
  for (int k : {1, 2, 3, 7, 16, 48, 97}) {
    std::vector<double> A = random_sym(k, rng), w(k), V((size_t)k * k);
    check(sd::sym_eig(k, A.data(), w.data(), V.data()), "sym_eig returns", k);
    double res, orth;
    eig_residuals(k, A, w.data(), V.data(), k, &res, &orth);
    check(res < 1e-12 && orth < 1e-12, "sym_eig residual / orthogonality", k);
    for (int i = 1; i < k; ++i) check(w[i - 1] <= w[i], "sym_eig ascending", k);
  }
  {
    const int k = 12;  // identity plus a rank-one term: a 11-fold repeated eigenvalue
    std::vector<double> A((size_t)k * k, 0.0), u(k), w(k), V((size_t)k * k);
    for (int i = 0; i < k; ++i) u[i] = N(rng);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) A[i + (size_t)j * k] = (i == j ? 1.0 : 0.0) + u[i] * u[j];
    check(sd::sym_eig(k, A.data(), w.data(), V.data()), "sym_eig repeated", k);
    double res, orth;
    eig_residuals(k, A, w.data(), V.data(), k, &res, &orth);
    check(res < 1e-12 && orth < 1e-12, "sym_eig repeated residual", k);
  }

  // lowest eigenpairs of symmetric band matrices (block tridiagonal of block Lanczos)
  for (int nb : {1, 2, 8}) {
    for (int blocks : {1, 2, 5, 20}) {
      const int k = nb * blocks;
      std::vector<double> A((size_t)k * k, 0.0);
      for (int b = 0; b < blocks; ++b)
        for (int i = 0; i < nb; ++i)
          for (int j = 0; j <= i + nb && b * nb + j < k; ++j) {
            const int r = b * nb + i, c = b * nb + j;
            if (c < r || c - r > nb) continue;
            const double v = N(rng);
            A[r + (size_t)c * k] = v;
            A[c + (size_t)r * k] = v;
          }
      const int want = std::min(k, 6);
      std::vector<double> w(want), V((size_t)k * want);
      check(sd::sym_band_eig_lowest(k, A.data(), want, w.data(), V.data()), "band eig returns", k);
      double res, orth;
      eig_residuals(k, A, w.data(), V.data(), want, &res, &orth);
      check(res < 1e-10 && orth < 1e-10, "band eig residual / orthogonality", k);
      std::vector<double> wf(k), Vf((size_t)k * k);
      sd::sym_eig(k, A.data(), wf.data(), Vf.data());
      for (int i = 0; i < want; ++i) check(std::fabs(wf[i] - w[i]) < 1e-11 * (1.0 + std::fabs(wf[i])), "band eig values", k);
    }
  }

  // Cholesky, triangular inverse: SPD and not SPD
  for (int k : {1, 4, 16, 48}) {
    std::vector<double> B((size_t)k * k, 0.0), R((size_t)k * k), Ri((size_t)k * k);
    std::vector<double> M((size_t)k * k);
    for (double& m : M) m = N(rng);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        double t = (i == j) ? 0.5 : 0.0;
        for (int l = 0; l < k; ++l) t += M[l + (size_t)i * k] * M[l + (size_t)j * k];
        B[i + (size_t)j * k] = t;
      }
    check(sd::cholesky_upper(k, B.data(), R.data()), "cholesky SPD", k);
    double err = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        double t = -B[i + (size_t)j * k];
        for (int l = 0; l < k; ++l) t += R[l + (size_t)i * k] * R[l + (size_t)j * k];
        err = std::max(err, std::fabs(t));
      }
    check(err < 1e-10 * k, "cholesky R^T R = B", k);
    sd::tri_upper_inv(k, R.data(), Ri.data());
    err = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        double t = (i == j) ? -1.0 : 0.0;
        for (int l = 0; l < k; ++l) t += R[i + (size_t)l * k] * Ri[l + (size_t)j * k];
        err = std::max(err, std::fabs(t));
      }
    check(err < 1e-8, "triangular inverse", k);
    B[0] = -1.0;  // no longer positive definite
    check(!sd::cholesky_upper(k, B.data(), R.data()), "cholesky rejects non-SPD", k);
  }

  // generalised pencil of the Rayleigh-Ritz step
  for (int k : {1, 3, 24, 48}) {
    std::vector<double> A = random_sym(k, rng), B = random_sym(k, rng, 3.0 * k);
    const int want = std::max(1, k / 3);
    std::vector<double> th(want), C((size_t)k * want);
    double cond = 0.0;
    check(sd::gen_eig(k, A.data(), B.data(), want, th.data(), C.data(), &cond), "gen_eig returns", k);
    double res = 0.0, borth = 0.0;
    for (int c = 0; c < want; ++c) {
      for (int i = 0; i < k; ++i) {
        double t = 0.0;
        for (int j = 0; j < k; ++j) t += (A[i + (size_t)j * k] - th[c] * B[i + (size_t)j * k]) * C[j + (size_t)c * k];
        res = std::max(res, std::fabs(t));
      }
      for (int d = 0; d < want; ++d) {
        double t = (c == d) ? -1.0 : 0.0;
        for (int i = 0; i < k; ++i)
          for (int j = 0; j < k; ++j) t += C[i + (size_t)c * k] * B[i + (size_t)j * k] * C[j + (size_t)d * k];
        borth = std::max(borth, std::fabs(t));
      }
    }
    check(res < 1e-9 * k && borth < 1e-10 * k && cond >= 1.0, "gen_eig A C = B C theta, C^T B C = I", k);
    // the O(k^2) bound from the Cholesky factor is an upper bound on cond_2(B), and
    // the bisected cond_2(B) equals the ratio of B's extreme eigenvalues
    double cond2 = 0.0, bound = 0.0;
    check(sd::gen_eig(k, A.data(), B.data(), want, th.data(), C.data(), &cond2, &bound), "gen_eig with bound", k);
    std::vector<double> wb(k), Vb((size_t)k * k);
    sd::sym_eig(k, B.data(), wb.data(), Vb.data());
    const double ref = wb[k - 1] / wb[0];
    check(std::fabs(cond2 - ref) <= 1e-12 * ref * k && bound >= cond2 * (1.0 - 1e-12), "cond_2 and its bound", k);
  }
  {
    // an ill-conditioned SPD matrix: eigenvalues 1 ... 1e-11 in a random basis
    const int k = 24;
    std::vector<double> Qm((size_t)k * k), B((size_t)k * k, 0.0), wq(k), Vq((size_t)k * k);
    std::vector<double> S = random_sym(k, rng);
    sd::sym_eig(k, S.data(), wq.data(), Vq.data());
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        double t = 0.0;
        for (int l = 0; l < k; ++l) t += Vq[i + (size_t)l * k] * std::pow(10.0, -11.0 * l / (k - 1)) * Vq[j + (size_t)l * k];
        B[i + (size_t)j * k] = t;
      }
    const double c = sd::spd_cond(k, B.data());
    check(c > 1e10 && c < 1e12, "spd_cond of an ill-conditioned matrix", k);
    B[0] = -1.0;
    check(!(sd::spd_cond(k, B.data()) < 1e300), "spd_cond of an indefinite matrix is infinite", k);
  }

  // DIIS: well-posed, singular (two equal residual histories), single entry
  for (int s : {1, 2, 5, 10, 20}) {
    const int n = 40;
    std::vector<double> Rr((size_t)n * s), Bm((size_t)s * s), alpha(s);
    for (double& r : Rr) r = N(rng);
    if (s >= 3)
      for (int i = 0; i < n; ++i) Rr[i + (size_t)2 * n] = Rr[i + (size_t)1 * n];  // singular Gram
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += Rr[i + (size_t)a * n] * Rr[i + (size_t)b * n];
        Bm[a + (size_t)b * s] = t;
      }
    sd::diis(s, Bm.data(), alpha.data());
    double sum = 0.0;
    bool finite = true;
    for (double a : alpha) {
      sum += a;
      finite = finite && std::isfinite(a);
    }
    check(finite && std::fabs(sum - 1.0) < 1e-10, "diis coefficients finite, sum 1", s);
  }

  // 2x2 pencil: random, B = I, nearly singular B
  for (int t = 0; t < 50; ++t) {
    const double a00 = N(rng), a01 = N(rng), a11 = N(rng);
    const double x = N(rng), y = N(rng);
    const double b00 = 1.0 + x * x, b01 = x * y * 0.5, b11 = 1.0 + y * y * (t == 0 ? 1e-12 : 1.0);
    double th, g0, g1;
    if (!sd::rr2(a00, a01, a11, b00, b01, b11, &th, &g0, &g1)) continue;
    const double r0 = (a00 - th * b00) * g0 + (a01 - th * b01) * g1;
    const double r1 = (a01 - th * b01) * g0 + (a11 - th * b11) * g1;
    const double nb = g0 * (b00 * g0 + b01 * g1) + g1 * (b01 * g0 + b11 * g1);
    check(std::fabs(r0) + std::fabs(r1) < 1e-8 * (1.0 + std::fabs(th)) && std::fabs(nb - 1.0) < 1e-8, "rr2", 2);
  }

  std::printf("%s: %d failure(s)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
