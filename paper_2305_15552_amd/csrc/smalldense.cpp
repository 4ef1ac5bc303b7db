// Small dense FP64 problems of the block eigensolvers, on the host:
//   symmetric eigenproblem (Householder tridiagonalisation + implicit QR with
//   Wilkinson shifts, Golub & Van Loan ch. 8), Cholesky, triangular inverse,
//   the generalised pencil of the Rayleigh-Ritz step (eq. (rreig)), the DIIS
//   constrained least-squares problem (eq. (xsum)-(rmm)) and the 2x2 pencil of
//   RMM-DIIS (eq. (rr)).
// All matrices are column-major.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace sd {

namespace {

inline double& at(std::vector<double>& A, int n, int i, int j) { return A[(size_t)i + (size_t)j * n]; }

// Householder reduction of the symmetric A (n x n) to tridiagonal form:
// A = Q T Q^T; on return d (diagonal), e (sub-diagonal, e[i] = T[i+1][i]) and,
// when want_q, Q (left empty otherwise).
void tridiagonalize(int n, std::vector<double>& A, std::vector<double>& d, std::vector<double>& e,
                    std::vector<double>& Q, bool want_q = true) {
  Q.clear();
  if (want_q) {
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) at(Q, n, i, i) = 1.0;
  }
  std::vector<double> v(n), p(n), w(n), qv(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    // column norm, scaled by its largest entry (no overflow, no per-entry hypot)
    double amax = 0.0;
    for (int i = 0; i < m; ++i) amax = std::max(amax, std::fabs(at(A, n, k + 1 + i, k)));
    double nx = 0.0;
    if (amax > 0.0) {
      double ss = 0.0;
      for (int i = 0; i < m; ++i) {
        const double t = at(A, n, k + 1 + i, k) / amax;
        ss += t * t;
      }
      nx = amax * std::sqrt(ss);
    }
    if (nx == 0.0) continue;
    const double x0 = at(A, n, k + 1, k);
    const double alpha = x0 >= 0 ? -nx : nx;
    for (int i = 0; i < m; ++i) v[i] = at(A, n, k + 1 + i, k);
    v[0] -= alpha;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // p = beta * A22 v, accumulated column by column (for each i the terms are
    // added in ascending j, as a row-by-row dot product would, but the inner loop
    // runs down a column)
    for (int i = 0; i < m; ++i) p[i] = 0.0;
    for (int j = 0; j < m; ++j) {
      const double vj = v[j];
      const double* col = &at(A, n, k + 1, k + 1 + j);
      for (int i = 0; i < m; ++i) p[i] += col[i] * vj;
    }
    for (int i = 0; i < m; ++i) p[i] *= beta;
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double K = 0.5 * beta * pv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) at(A, n, k + 1 + i, k + 1 + j) -= v[i] * w[j] + w[i] * v[j];
    at(A, n, k + 1, k) = alpha;
    at(A, n, k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) {
      at(A, n, k + 1 + i, k) = 0.0;
      at(A, n, k, k + 1 + i) = 0.0;
    }
    // Q <- Q H,  H = I - beta v v^T acting on indices k+1..n-1
    if (!want_q) continue;
    for (int r = 0; r < n; ++r) qv[r] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double vi = v[i];
      const double* col = &at(Q, n, 0, k + 1 + i);
      for (int r = 0; r < n; ++r) qv[r] += col[r] * vi;
    }
    for (int r = 0; r < n; ++r) qv[r] *= beta;
    for (int i = 0; i < m; ++i)
      for (int r = 0; r < n; ++r) at(Q, n, r, k + 1 + i) -= qv[r] * v[i];
  }
  d.resize(n);
  e.assign(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = at(A, n, i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = at(A, n, i + 1, i);
}

// implicit symmetric tridiagonal QR with Wilkinson shifts; rotations accumulated
// into Q unless Q is empty (eigenvalues only)
bool tridiag_qr(int n, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Q) {
  const bool vecs = !Q.empty();
  const double eps = 2.220446049250313e-16;
  for (int h = n - 1; h > 0; --h) {
    int iter = 0;
    for (;;) {
      int l = h;
      while (l > 0 && std::fabs(e[l - 1]) > eps * (std::fabs(d[l - 1]) + std::fabs(d[l]))) --l;
      if (l == h) break;
      if (++iter > 60 * n) return false;
      // Wilkinson shift from the trailing 2x2 of the window [l, h]
      const double a = d[h - 1], b = e[h - 1], c = d[h];
      const double del = 0.5 * (a - c);
      const double den = del + (del >= 0 ? 1.0 : -1.0) * std::hypot(del, b);
      const double mu = (den != 0.0) ? c - b * b / den : c;
      double x = d[l] - mu, z = e[l];
      double bulge = 0.0;
      for (int k = l; k < h; ++k) {
        if (k > l) {
          x = e[k - 1];
          z = bulge;
        }
        const double r = std::sqrt(x * x + z * z);  // O(norm) entries: no overflow
        double cs = 1.0, sn = 0.0;
        if (r != 0.0) {
          cs = x / r;
          sn = -z / r;
        }
        if (k > l) e[k - 1] = r;
        const double dk = d[k], ek = e[k], dk1 = d[k + 1];
        d[k] = cs * cs * dk - 2.0 * cs * sn * ek + sn * sn * dk1;
        d[k + 1] = sn * sn * dk + 2.0 * cs * sn * ek + cs * cs * dk1;
        e[k] = cs * sn * (dk - dk1) + (cs * cs - sn * sn) * ek;
        if (k + 1 < h) {
          bulge = -sn * e[k + 1];
          e[k + 1] = cs * e[k + 1];
        }
        if (vecs)
          for (int q = 0; q < n; ++q) {
            const double qk = at(Q, n, q, k), qk1 = at(Q, n, q, k + 1);
            at(Q, n, q, k) = cs * qk - sn * qk1;
            at(Q, n, q, k + 1) = sn * qk + cs * qk1;
          }
      }
    }
  }
  return true;
}

// Symmetric band matrix (half-bandwidth b) to tridiagonal form by Givens
// rotations with bulge chasing (Schwarz's reduction; Golub & Van Loan 8.3):
// column j's entries below the first subdiagonal are annihilated from the
// bottom of the band up; each rotation of rows/columns (p, p+1) leaves one
// entry just outside the band b rows further down, which the next rotation
// moves on by b.  The lower band is kept in compact storage with room for the
// bulge: L[j (b + 2) + i - j] = A(i, j) for 0 <= i - j <= b + 1, so a rotation
// touches about 4 b + 3 nearby entries.
void band_to_tridiagonal(int n, int b, const std::vector<double>& A, std::vector<double>& d, std::vector<double>& e) {
  const int W = b + 2;
  std::vector<double> L((size_t)n * W, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = j; i <= std::min(n - 1, j + b); ++i) L[(size_t)j * W + (i - j)] = A[i + (size_t)j * n];
  auto el = [&](int i, int j) -> double& { return L[(size_t)j * W + (i - j)]; };  // i >= j, i - j <= b + 1
  // similarity with the rotation of rows/columns p, q = p + 1 chosen so that
  // entry (q, col), col < p, becomes zero
  auto rotate = [&](int p, int col) {
    const int q = p + 1;
    const double x = el(p, col), z = el(q, col);
    if (z == 0.0) return;
    const double r = std::sqrt(x * x + z * z), c = x / r, s = z / r;
    // entries left of p: rows p and q
    for (int k = std::max(0, q - b - 1); k < p; ++k) {
      const double ap = el(p, k), aq = el(q, k);
      el(p, k) = c * ap + s * aq;
      el(q, k) = -s * ap + c * aq;
    }
    el(q, col) = 0.0;
    // the 2 x 2 block
    const double app = el(p, p), apq = el(q, p), aqq = el(q, q);
    el(p, p) = c * c * app + 2.0 * c * s * apq + s * s * aqq;
    el(q, q) = s * s * app - 2.0 * c * s * apq + c * c * aqq;
    el(q, p) = c * s * (aqq - app) + (c * c - s * s) * apq;
    // entries below q: columns p and q
    for (int k = q + 1; k <= std::min(n - 1, p + b + 1); ++k) {
      const double ap = el(k, p), aq = (k - q <= b + 1) ? el(k, q) : 0.0;
      el(k, p) = c * ap + s * aq;
      el(k, q) = -s * ap + c * aq;
    }
  };
  if (b > 1)
    for (int j = 0; j + 2 < n; ++j)
      for (int i = std::min(j + b, n - 1); i >= j + 2; --i) {
        if (el(i, j) == 0.0) continue;
        rotate(i - 1, j);
        // the bulge at (i + b, i - 1) moves down the band
        for (int k = i + b; k < n; k += b) rotate(k - 1, k - b - 1);
      }
  d.resize(n);
  e.assign(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = el(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = el(i + 1, i);
}

// LU with partial pivoting of T - sigma I for a band T (half-bandwidth b),
// kept in compact storage: row i holds columns i - b .. i + 2b (the upper
// bandwidth grows to 2b with the row exchanges).  Zero pivots are replaced by
// a tiny multiple of the norm (inverse iteration only needs a direction).
struct BandLU {
  int n = 0, b = 0, w = 0;
  std::vector<double> a;
  std::vector<int> piv;
  double& el(int i, int j) { return a[(size_t)i * w + (j - i + b)]; }
  double el(int i, int j) const { return a[(size_t)i * w + (j - i + b)]; }
  void factor(int n_, int b_, const double* T, double sigma, double tiny) {
    n = n_;
    b = b_;
    w = 3 * b + 1;
    a.assign((size_t)n * w, 0.0);
    piv.assign(n, 0);
    for (int i = 0; i < n; ++i)
      for (int j = std::max(0, i - b); j <= std::min(n - 1, i + b); ++j)
        el(i, j) = T[(size_t)i + (size_t)j * n] - (i == j ? sigma : 0.0);
    for (int c = 0; c < n; ++c) {
      const int last = std::min(n - 1, c + b), right = std::min(n - 1, c + 2 * b);
      int p = c;
      for (int r = c + 1; r <= last; ++r)
        if (std::fabs(el(r, c)) > std::fabs(el(p, c))) p = r;
      piv[c] = p;
      if (p != c)
        for (int j = c; j <= right; ++j) std::swap(el(c, j), el(p, j));
      if (std::fabs(el(c, c)) < tiny) el(c, c) = el(c, c) < 0 ? -tiny : tiny;
      const double inv = 1.0 / el(c, c);
      for (int r = c + 1; r <= last; ++r) {
        const double l = el(r, c) * inv;
        el(r, c) = l;
        if (l != 0.0)
          for (int j = c + 1; j <= right; ++j) el(r, j) -= l * el(c, j);
      }
    }
  }
  void solve(double* x) const {
    for (int c = 0; c < n; ++c) {
      std::swap(x[c], x[piv[c]]);
      for (int r = c + 1; r <= std::min(n - 1, c + b); ++r) x[r] -= el(r, c) * x[c];
    }
    for (int c = n - 1; c >= 0; --c) {
      double s = x[c];
      for (int j = c + 1; j <= std::min(n - 1, c + 2 * b); ++j) s -= el(c, j) * x[j];
      x[c] = s / el(c, c);
    }
  }
};

// Eigenvectors of the `want` lowest eigenvalues d[0..want) (ascending, from
// the same matrix) of a symmetric band matrix T (dense n x n column-major,
// half-bandwidth b) by inverse iteration: LU of T - d_j I, four solves from a
// fixed start; within a cluster (gap below 1e-3 of the norm) each iterate is
// orthogonalised against the cluster's earlier vectors, and numerically equal
// eigenvalues are separated as LAPACK's inverse iteration does.
// number of eigenvalues of the symmetric tridiagonal (d, e) below x (Sturm
// sequence of the LDL^T pivots; a pivot that vanishes is taken as -pivmin)
int sturm_below(int n, const double* d, const double* e, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (std::fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

// the j-th smallest eigenvalue (0-based) of the symmetric tridiagonal (d, e) by
// bisection from the Gershgorin interval, to an absolute accuracy of about
// eps (|lambda| + ||T||), the accuracy of the QR iteration's eigenvalues
double bisect_eig(int n, const double* d, const double* e, int j) {
  const double eps = 2.220446049250313e-16;
  double lo = INFINITY, hi = -INFINITY, nrm = 0.0, emax2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
    nrm = std::max(nrm, std::fabs(d[i]) + r);
    if (i + 1 < n) emax2 = std::max(emax2, e[i] * e[i]);
  }
  const double pivmin = 1e-290 * std::max(1.0, emax2);
  lo -= eps * nrm;
  hi += eps * nrm;
  for (int it = 0; it < 256; ++it) {
    const double tol = eps * (std::max(std::fabs(lo), std::fabs(hi)) + nrm);
    if (hi - lo <= tol) break;
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(n, d, e, mid, pivmin) > j)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

bool inverse_vectors(int n, int b, const double* T, const std::vector<double>& d, double nrm, int want, double* V) {
  const double eps = 2.220446049250313e-16;
  const double tiny = eps * std::max(nrm, 1e-300) * n;
  const double ctol = 1e-3 * std::max(nrm, 1e-300);
  BandLU lu;
  std::vector<double> x(n);
  int cstart = 0;
  for (int j = 0; j < want; ++j) {
    if (j > 0 && d[j] - d[j - 1] > ctol) cstart = j;
    double sigma = d[j];
    if (j > 0 && sigma - d[j - 1] < 10.0 * eps * nrm * n) sigma = d[j - 1] + 10.0 * eps * nrm * n;
    lu.factor(n, std::max(b, 1), T, sigma, tiny);
    for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.5 * std::sin(0.7 * (i + 1) * (j + 1));
    for (int it = 0; it < 4; ++it) {
      lu.solve(x.data());
      for (int pass = 0; pass < 2; ++pass)
        for (int q = cstart; q < j; ++q) {
          double dot = 0.0;
          for (int i = 0; i < n; ++i) dot += V[i + (size_t)q * n] * x[i];
          for (int i = 0; i < n; ++i) x[i] -= dot * V[i + (size_t)q * n];
        }
      double s2 = 0.0;
      for (int i = 0; i < n; ++i) s2 += x[i] * x[i];
      s2 = std::sqrt(s2);
      if (!(s2 > 0.0) || !std::isfinite(s2)) return false;
      for (int i = 0; i < n; ++i) x[i] /= s2;
    }
    for (int i = 0; i < n; ++i) V[i + (size_t)j * n] = x[i];
  }
  return true;
}

}  // namespace

bool sym_band_eig_lowest(int n, const double* Tin, int want, double* w, double* V) {
  if (n <= 0 || want <= 0) return n >= 0;
  want = std::min(want, n);
  std::vector<double> A((size_t)n * n);
  int b = 0;
  double nrm = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const double v = 0.5 * (Tin[i + (size_t)j * n] + Tin[j + (size_t)i * n]);
      if (!std::isfinite(v)) return false;
      A[i + (size_t)j * n] = v;
      if (v != 0.0) b = std::max(b, std::abs(i - j));
      nrm = std::max(nrm, std::fabs(v));
    }
  // eigenvalues: band -> tridiagonal, then QR without vectors
  std::vector<double> d, e, none;
  band_to_tridiagonal(n, b, A, d, e);
  const std::vector<double>& Ts = A;  // the band matrix itself, for inverse iteration
  if (!tridiag_qr(n, d, e, none)) return false;
  std::sort(d.begin(), d.end());
  if (!inverse_vectors(n, b, Ts.data(), d, nrm, want, V)) return false;
  for (int j = 0; j < want; ++j) w[j] = d[j];
  return true;
}

bool sym_eig(int k, const double* Ain, double* w, double* V) {
  std::vector<double> A((size_t)k * k);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i) A[i + (size_t)j * k] = 0.5 * (Ain[i + (size_t)j * k] + Ain[j + (size_t)i * k]);
  for (double x : A)
    if (!std::isfinite(x)) return false;
  std::vector<double> d, e, Q;
  tridiagonalize(k, A, d, e, Q, V != nullptr);
  if (!tridiag_qr(k, d, e, Q)) return false;
  std::vector<int> idx(k);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  for (int j = 0; j < k; ++j) {
    w[j] = d[idx[j]];
    if (V)
      for (int i = 0; i < k; ++i) V[i + (size_t)j * k] = Q[i + (size_t)idx[j] * k];
  }
  return true;
}

bool cholesky_upper(int k, const double* G, double* R) {
  // R^T R = G, R upper; symmetrised input
  std::memset(R, 0, sizeof(double) * k * k);
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i <= j; ++i) {
      double s = 0.5 * (G[i + (size_t)j * k] + G[j + (size_t)i * k]);
      for (int q = 0; q < i; ++q) s -= R[q + (size_t)i * k] * R[q + (size_t)j * k];
      if (i == j) {
        // a pivot at rounding level of the diagonal entry means numerical rank deficiency
        const double gjj = std::fabs(G[j + (size_t)j * k]);
        if (!(s > 16.0 * k * 2.220446049250313e-16 * gjj) || !std::isfinite(s)) return false;
        R[j + (size_t)j * k] = std::sqrt(s);
      } else {
        R[i + (size_t)j * k] = s / R[i + (size_t)i * k];
      }
    }
  }
  return true;
}

void tri_upper_inv(int k, const double* R, double* Ri) {
  std::memset(Ri, 0, sizeof(double) * k * k);
  for (int j = 0; j < k; ++j) {
    Ri[j + (size_t)j * k] = 1.0 / R[j + (size_t)j * k];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int q = i + 1; q <= j; ++q) s += R[i + (size_t)q * k] * Ri[q + (size_t)j * k];
      Ri[i + (size_t)j * k] = -s / R[i + (size_t)i * k];
    }
  }
}

double spd_cond(int k, const double* B) {
  // the two extreme eigenvalues of B alone: tridiagonal form, then bisection
  std::vector<double> Bs((size_t)k * k), d, e, none;
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i) {
      const double v = 0.5 * (B[i + (size_t)j * k] + B[j + (size_t)i * k]);
      if (!std::isfinite(v)) return INFINITY;
      Bs[i + (size_t)j * k] = v;
    }
  tridiagonalize(k, Bs, d, e, none, false);
  const double lmin = bisect_eig(k, d.data(), e.data(), 0), lmax = bisect_eig(k, d.data(), e.data(), k - 1);
  return lmin > 0 ? lmax / lmin : INFINITY;
}

bool gen_eig(int k, const double* A, const double* B, int nwant, double* theta, double* C, double* condB,
             double* cond_bound) {
  std::vector<double> w(k), V((size_t)k * k);
  if (!B) {
    if (!sym_eig(k, A, w.data(), V.data())) return false;
    for (int j = 0; j < nwant; ++j) {
      theta[j] = w[j];
      for (int i = 0; i < k; ++i) C[i + (size_t)j * k] = V[i + (size_t)j * k];
    }
    if (condB) *condB = 1.0;
    if (cond_bound) *cond_bound = 1.0;
    return true;
  }
  if (condB) *condB = spd_cond(k, B);
  std::vector<double> R((size_t)k * k), Ri((size_t)k * k), M((size_t)k * k), T((size_t)k * k);
  if (!cholesky_upper(k, B, R.data())) return false;
  tri_upper_inv(k, R.data(), Ri.data());
  if (cond_bound) {
    // cond_2(B) <= ||B||_1 ||B^-1||_1 <= ||B||_1 ||R^-1||_1 ||R^-1||_inf (B symmetric, B^-1 = R^-1 R^-T)
    double b1 = 0.0, r1 = 0.0, rinf = 0.0;
    std::vector<double> rowsum(k, 0.0);
    for (int j = 0; j < k; ++j) {
      double cb = 0.0, cr = 0.0;
      for (int i = 0; i < k; ++i) {
        cb += std::fabs(B[i + (size_t)j * k]);
        const double r = std::fabs(Ri[i + (size_t)j * k]);
        cr += r;
        rowsum[i] += r;
      }
      b1 = std::max(b1, cb);
      r1 = std::max(r1, cr);
    }
    for (int i = 0; i < k; ++i) rinf = std::max(rinf, rowsum[i]);
    *cond_bound = b1 * r1 * rinf;
  }
  // M = Ri^T A Ri with A symmetrised once, both products as AXPYs down
  // contiguous columns (T = A Ri; M = Ri^T T through a transposed copy of Ri).
  // Every entry sums its terms in ascending q, as the dot products would.
  std::vector<double> As((size_t)k * k), RiT((size_t)k * k);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i) {
      As[i + (size_t)j * k] = 0.5 * (A[i + (size_t)j * k] + A[j + (size_t)i * k]);
      RiT[i + (size_t)j * k] = Ri[j + (size_t)i * k];
    }
  std::fill(T.begin(), T.end(), 0.0);
  for (int j = 0; j < k; ++j) {
    double* tj = &T[(size_t)j * k];
    for (int q = 0; q <= j; ++q) {
      const double r = Ri[q + (size_t)j * k];
      const double* aq = &As[(size_t)q * k];
      for (int i = 0; i < k; ++i) tj[i] += aq[i] * r;
    }
  }
  std::fill(M.begin(), M.end(), 0.0);
  for (int j = 0; j < k; ++j) {
    const double* tj = &T[(size_t)j * k];
    double* mj = &M[(size_t)j * k];
    for (int q = 0; q < k; ++q) {
      const double tq = tj[q];
      const double* rq = &RiT[(size_t)q * k];
      for (int i = q; i < k; ++i) mj[i] += rq[i] * tq;
    }
  }
  if (!sym_eig(k, M.data(), w.data(), V.data())) return false;
  // C = Ri V on the wanted columns, AXPYs down the columns of the upper-triangular Ri
  for (int j = 0; j < nwant; ++j) {
    theta[j] = w[j];
    double* cj = &C[(size_t)j * k];
    std::fill(cj, cj + k, 0.0);
    for (int q = 0; q < k; ++q) {
      const double v = V[q + (size_t)j * k];
      const double* rq = &Ri[(size_t)q * k];
      for (int i = 0; i <= q; ++i) cj[i] += rq[i] * v;
    }
  }
  return true;
}

void diis(int s, const double* Bm, double* alpha) {
  if (s == 1) {
    alpha[0] = 1.0;
    return;
  }
  double scale = 0.0;
  for (int i = 0; i < s; ++i) scale = std::max(scale, std::fabs(Bm[i + (size_t)i * s]));
  if (scale == 0.0) scale = 1.0;
  const int N = s + 1;
  std::vector<double> M((size_t)N * N, 0.0), rhs(N, 0.0);
  for (int j = 0; j < s; ++j)
    for (int i = 0; i < s; ++i) M[i + (size_t)j * N] = 0.5 * (Bm[i + (size_t)j * s] + Bm[j + (size_t)i * s]) / scale;
  for (int i = 0; i < s; ++i) {
    M[i + (size_t)s * N] = 1.0;
    M[s + (size_t)i * N] = 1.0;
  }
  rhs[s] = 1.0;
  // Gaussian elimination with partial pivoting
  std::vector<double> LU = M, b = rhs;
  bool singular = false;
  double maxabs = 0.0;
  for (double x : LU) maxabs = std::max(maxabs, std::fabs(x));
  for (int c = 0; c < N && !singular; ++c) {
    int piv = c;
    for (int r = c + 1; r < N; ++r)
      if (std::fabs(LU[r + (size_t)c * N]) > std::fabs(LU[piv + (size_t)c * N])) piv = r;
    if (std::fabs(LU[piv + (size_t)c * N]) <= 1e-14 * maxabs) {
      singular = true;
      break;
    }
    if (piv != c) {
      for (int q = 0; q < N; ++q) std::swap(LU[c + (size_t)q * N], LU[piv + (size_t)q * N]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < N; ++r) {
      double f = LU[r + (size_t)c * N] / LU[c + (size_t)c * N];
      if (f == 0.0) continue;
      for (int q = c; q < N; ++q) LU[r + (size_t)q * N] -= f * LU[c + (size_t)q * N];
      b[r] -= f * b[c];
    }
  }
  std::vector<double> x(N, 0.0);
  if (!singular) {
    for (int r = N - 1; r >= 0; --r) {
      double acc = b[r];
      for (int q = r + 1; q < N; ++q) acc -= LU[r + (size_t)q * N] * x[q];
      x[r] = acc / LU[r + (size_t)r * N];
    }
    for (double v : x)
      if (!std::isfinite(v)) singular = true;
  }
  if (singular) {
    // minimum-norm least squares through the symmetric eigendecomposition
    std::vector<double> w(N), V((size_t)N * N);
    if (!sym_eig(N, M.data(), w.data(), V.data())) {
      for (int i = 0; i < s; ++i) alpha[i] = (i == s - 1) ? 1.0 : 0.0;
      return;
    }
    double wmax = 0.0;
    for (double v : w) wmax = std::max(wmax, std::fabs(v));
    std::fill(x.begin(), x.end(), 0.0);
    for (int j = 0; j < N; ++j) {
      if (std::fabs(w[j]) <= 1e-14 * wmax) continue;
      double c = 0.0;
      for (int i = 0; i < N; ++i) c += V[i + (size_t)j * N] * rhs[i];
      c /= w[j];
      for (int i = 0; i < N; ++i) x[i] += c * V[i + (size_t)j * N];
    }
  }
  for (int i = 0; i < s; ++i) alpha[i] = x[i];
}

bool rr2(double a00, double a01, double a11, double b00, double b01, double b11, double* theta, double* g0,
         double* g1) {
  const double A[4] = {a00, a01, a01, a11};
  const double B[4] = {b00, b01, b01, b11};
  double th, C[4];
  if (!gen_eig(2, A, B, 1, &th, C, nullptr)) return false;
  double g[2] = {C[0], C[1]};
  double q = g[0] * (b00 * g[0] + b01 * g[1]) + g[1] * (b01 * g[0] + b11 * g[1]);
  if (!(q > 0)) return false;
  q = 1.0 / std::sqrt(q);
  // orientation: positive overlap with the first basis vector, (B g)_0 > 0
  if (b00 * g[0] + b01 * g[1] < 0) q = -q;
  *theta = th;
  *g0 = g[0] * q;
  *g1 = g[1] * q;
  return true;
}

}  // namespace sd
