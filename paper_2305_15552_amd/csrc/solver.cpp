// Host drivers of the block eigensolvers.  Every vector operation runs in the
// HIP kernels of this library; the host only solves the small FP64 problems
// (Rayleigh-Ritz pencils, DIIS least squares, 2x2 pencils, block tridiagonal
// eigenproblems) and takes the control decisions.
//   LOBPCG          Algorithm 2 with the H X / H P recurrences (eq. (upd1)-(upd2))
//   block Lanczos   Algorithm 1, two classical Gram-Schmidt passes, CholeskyQR2
//   RMM-DIIS        Algorithm 4, all columns batched into one product per sweep
//   hybrid          Section 2.7: front end, switch (eq. (switchtau)), RMM-DIIS
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <vector>

#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;
inline double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hyeig_status alloc(hyeig_ctx* ctx, size_t b) {
    release();
    hipError_t e = hipMalloc(&p, std::max<size_t>(b, 64));
    if (e != hipSuccess) {
      p = nullptr;
      return hip_err(ctx, e, "solver hipMalloc");
    }
    bytes = b;
    return HYEIG_OK;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  ~DBuf() { release(); }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};

size_t dsize(hyeig_dtype dt) { return dt == HYEIG_F64 ? 8 : 4; }

// algorithmic bytes of one product: stored entries (value + column index), the
// row pointer, X read once and Y written once
double spmm_bytes(const hyeig_mat* H, int m, hyeig_dtype xdt, hyeig_dtype ydt, hyeig_dtype vdt) {
  const double sv = vdt == HYEIG_BF16 ? 2.0 : 4.0;
  return (double)H->nnz * (sv + 4.0) + 8.0 * (double)(H->n + 1) +
         (double)H->n * m * (double)(dsize(xdt) + dsize(ydt));
}

// host <-> device small transfers through pinned staging.  The solvers read a
// few KB per iteration and have nothing else to do meanwhile, so the host polls
// an event recorded after the copy instead of sleeping in a stream
// synchronisation (the wake-up is on the iteration's critical path).
hyeig_status d2h(hyeig_ctx* ctx, void* h, const void* d, size_t bytes) {
  hyeig_status st;
  void* p = pin_get(ctx, bytes, &st);
  if (!p) return st;
  if (!ctx->d2h_ev) HY_HIP(ctx, hipEventCreateWithFlags(&ctx->d2h_ev, hipEventDisableTiming));
  HY_HIP(ctx, hipMemcpyAsync(p, d, bytes, hipMemcpyDeviceToHost, ctx->stream));
  HY_HIP(ctx, hipEventRecord(ctx->d2h_ev, ctx->stream));
  for (;;) {
    const hipError_t e = hipEventQuery(ctx->d2h_ev);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) return hip_err(ctx, e, "d2h: event query");
  }
  std::memcpy(h, p, bytes);
  return HYEIG_OK;
}

hyeig_status h2d(hyeig_ctx* ctx, void* d, const void* h, size_t bytes) { return h2d_queued(ctx, d, h, bytes); }

// accumulated kernel time of the products (HIP events, read at sync points)
struct SpmmClock {
  std::vector<hipEvent_t> ev;
  std::vector<char> mc;         // per timed product: ran on a matrix-core kernel
  std::vector<double> bytes;    // per timed product: its algorithmic bytes
  int used = 0;
  double ms = 0.0;
  double ms_mc = 0.0, bytes_mc = 0.0;  // the matrix-core products alone
  int n_mc = 0;
  hyeig_ctx* ctx = nullptr;
  ~SpmmClock() {
    for (auto e : ev) hipEventDestroy(e);
  }
  void start(hyeig_ctx* c) {
    ctx = c;
    if (used + 2 > (int)ev.size()) {
      hipEvent_t a, b;
      hipEventCreate(&a);
      hipEventCreate(&b);
      ev.push_back(a);
      ev.push_back(b);
    }
    hipEventRecord(ev[used], ctx->stream);
  }
  void stop(bool on_mc, double nbytes) {
    hipEventRecord(ev[used + 1], ctx->stream);
    const size_t q = (size_t)used / 2;
    if (mc.size() <= q) {
      mc.resize(q + 1);
      bytes.resize(q + 1);
    }
    mc[q] = on_mc;
    bytes[q] = nbytes;
    used += 2;
  }
  void collect() {
    for (int i = 0; i + 1 < used; i += 2) {
      float t = 0.f;
      hipEventSynchronize(ev[i + 1]);
      if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) == hipSuccess) {
        ms += t;
        if (mc[i / 2]) {
          ms_mc += t;
          bytes_mc += bytes[i / 2];
          ++n_mc;
        }
      }
    }
    used = 0;
  }
};

struct Run {
  hyeig_ctx* ctx;
  const hyeig_mat* H;
  const hyeig_params* p;
  hyeig_report* rep;
  SpmmClock clk;
  double hnorm = 1.0;
  int64_t n;
  hyeig_dtype dt;            // block data type
  hyeig_dtype vdt = HYEIG_F32;  // stored values used by the products
  hyeig_mma_mode gmode;      // Gram contraction mode
  int hist_row = 0;
  double t_small = 0.0;
  Clock::time_point t_start = Clock::now();
  double cond_now = 0.0;  // condition number of S^T S in the last LOBPCG Rayleigh-Ritz step

  hyeig_status spmm(int m, const void* X, int64_t ldx, void* Y, int64_t ldy) {
    // the product's column width for m, and the element size
    const int mp = m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : m <= 8 ? 8 : m <= 12 ? 12 : m <= 16 ? 16 : 32;
    const int es = dt == HYEIG_F64 ? 8 : 4;
    if (m > 1 && ldx != mp && (mp * es < 64 || (m * es) % 16 != 0)) {
      // columns inside wider rows (the active part of W in [X W P]): rows under
      // 64 bytes leave most of each memory line the x blocks touch unused, and
      // widths off a 16-byte boundary take the element-wise x loads; gather
      // them into whole, zero-padded rows first
      hyeig_status st;
      void* Xc = ws_get(ctx, WS_TMP, (size_t)n * mp * es, &st);
      if (!Xc) return st;
      HY_CHECK(launch_gather_pad(ctx, n, m, mp, X, ldx, Xc, dt));
      clk.start(ctx);
      HY_CHECK(launch_spmm(ctx, H, m, Xc, mp, dt, Y, ldy, dt, vdt, true));
    } else {
      // rows exactly the product's width are whole rows of one of the solver's
      // arrays (the blocks of [X W P]): the product may read them in pieces
      clk.start(ctx);
      HY_CHECK(launch_spmm(ctx, H, m, X, ldx, dt, Y, ldy, dt, vdt, ldx == mp));
    }
    const double b = spmm_bytes(H, m, dt, dt, vdt);
    clk.stop(spmm_on_matrix_cores(H, m, dt, dt, vdt), b);
    rep->spmm_count++;
    rep->spmv_count += m;
    rep->bytes_spmm += b;
    return HYEIG_OK;
  }
  double scale(double theta) const {
    return p->tol_norm == HYEIG_NORM_THETA ? std::max(std::fabs(theta), 1e-300) : hnorm;
  }
  void hist(const double* rel, int k) {
    if (rep->hist && hist_row < rep->hist_cap) {
      std::memcpy(rep->hist + (size_t)hist_row * k, rel, sizeof(double) * k);
      if (rep->hist_t) {
        rep->hist_t[4 * (size_t)hist_row] = ms_since(t_start);
        rep->hist_t[4 * (size_t)hist_row + 1] = clk.ms;
        rep->hist_t[4 * (size_t)hist_row + 2] = t_small;
        rep->hist_t[4 * (size_t)hist_row + 3] = cond_now;
      }
      rep->hist_len = ++hist_row;
    }
  }
};

// ---------------------------------------------------------------------------
// switch rule of the hybrids (Section 4.1)
// ---------------------------------------------------------------------------
struct Switch {
  const hyeig_params* p;
  std::vector<double> prev;
  bool enabled = false;
  double last_tau = INFINITY;
  // returns true when the front end should hand over
  bool fire(int it, const double* theta, const double* rel, int k) {
    if (!enabled) return false;
    if (p->switch_rule == HYEIG_SWITCH_ITERS) return it >= (int)p->switch_thr;
    if (p->switch_rule == HYEIG_SWITCH_RESID) {
      double mx = 0;
      for (int j = 0; j < k; ++j) mx = std::max(mx, rel[j]);
      return it >= 1 && mx < p->switch_thr;
    }
    bool out = false;
    if ((int)prev.size() == k) {
      double s = 0;  // eq. (switchtau): (1/n_ev) sqrt(sum ((t_k - t_{k-1}) / t_k)^2)
      for (int j = 0; j < k; ++j) {
        double q = (theta[j] - prev[j]) / theta[j];
        s += q * q;
      }
      last_tau = std::sqrt(s) / k;
      out = it >= p->min_front && last_tau < p->switch_thr;
    }
    prev.assign(theta, theta + k);
    return out;
  }
};

// ---------------------------------------------------------------------------
// LOBPCG (Algorithm 2).  S = [X | W | P] and HS = [HX | HW | HP] have 3 nb
// columns (ld), double buffered.  For n_b = 16 each of X, W, P (HX, HW, HP)
// is its own contiguous n x 16 array (lds = 16, block bs = 16 n elements
// after the previous one), so that every pass over one block streams whole
// memory lines; otherwise the three blocks share n x 3 nb rows (lds = ld).
// W holds the active columns compacted to the front, P all nb directions; the
// Rayleigh-Ritz step picks the rows of the active subspace.
// ---------------------------------------------------------------------------
struct Lobpcg {
  Run& R;
  int nb, k;
  int ld;          // columns of S
  bool planar;     // blocks stored apart
  int lds;         // leading dimension of one block
  int64_t bs;      // elements from the start of one block to the next
  // dC: the update coefficients [C1 C2] (2 ld x nb) and, behind them, the nb
  // Ritz values, so that one upload carries both
  DBuf S[2], HS[2], dG, dC, dnrm, dpos, dmlp;
  int cur = 0;
  bool haveP = false;
  int prank = 0;  // FP32 forms: P holds prank orthonormal directions (columns 0..prank-1)
  std::vector<double> theta, rel;
  std::vector<int> active;
  int it = 0;
  const float* d = nullptr;
  double floor_ = 0.0;
  // the column positions dpos holds on the device (empty: unknown), and whether
  // the residual pass at the top of this iteration already formed W with them
  std::vector<int> pos_dev;
  bool w_formed = false;
  // the last update also ran the next residual pass (W and the norms on the
  // device, with the positions pos_dev): the pass at the top of the iteration
  // only reads the norms
  bool resid_fused = false;
  // the iterate whose worst wanted residual was lowest once below 1e-4 or 100
  // times the tolerance (copied when that residual halves): an iteration that ends
  // unconverged, at its limit or by a breakdown (a tolerance below what the
  // arithmetic attains lets FP32 iterates drift from a good block), returns it
  // rather than the last block (the copy lives in the context's workspace)
  void* best = nullptr;
  double best_worst = INFINITY;

  // blocks stored apart for n_b = 16, except in the BF16 form, whose split-BF16
  // Gram products read the interleaved rows
  static bool use_planar(const Run& r, int nb_) { return nb_ == 16 && r.p->precision != HYEIG_PREC_BF16_SPMM; }
  explicit Lobpcg(Run& r, int nb_, int k_)
      : R(r), nb(nb_), k(k_), ld(3 * nb_), planar(use_planar(r, nb_)), lds(planar ? nb_ : 3 * nb_),
        bs(planar ? r.n * nb_ : nb_) {}

  // learned preconditioner on the compacted active residual columns (W holds R);
  // a non-finite output falls back to the shifted diagonal for this iteration.
  // The column scales come from the device-side norms and Ritz values, and the
  // fallback is decided on the device (a residual pass guarded by the flag),
  // so the iteration has no host round trip here; flags[1] counts fallbacks.
  hyeig_status mlp_precond(int na) {
    hyeig_ctx* ctx = R.ctx;
    int* flags = dmlp.as<int>();
    HY_CHECK(launch_mlp_precond(ctx, R.p->mlp, R.H, R.n, na, col(cur, false, nb), lds, R.dt, dth(),
                                dnrm.as<double>(), dpos.as<int>(), nb, R.hnorm, flags));
    HY_CHECK(launch_resid_precond(ctx, R.n, nb, col(cur, false, 0), lds, col(cur, true, 0), lds, dth(), d,
                                  floor_, na, dpos.as<int>(), col(cur, false, nb), lds, nb, R.dt, nullptr, flags));
    return launch_mlp_flag_count(ctx, flags);
  }
  // fallbacks counted on the device since the last call -> the report
  hyeig_status mlp_events() {
    if (R.p->precond != HYEIG_PRECOND_MLP || !dmlp.p) return HYEIG_OK;
    int flags[2] = {0, 0};
    HY_CHECK(d2h(R.ctx, flags, dmlp.p, sizeof(flags)));
    if (flags[1]) {
      R.rep->events_mlp_fallback += flags[1];
      const int zero[2] = {0, 0};
      HY_CHECK(h2d(R.ctx, dmlp.p, zero, sizeof(zero)));
    }
    return HYEIG_OK;
  }
  bool stable_basis() const { return R.p->basis == 1 || (R.p->basis < 0 && R.dt == HYEIG_F32); }
  double* dth() { return dC.as<double>() + 2 * ld * nb; }

  // column c of S (or HS): block c / nb, column c % nb of that block
  char* col(int buf, bool h, int c) {
    char* base = (char*)(h ? HS[buf].p : S[buf].p);
    return base + (size_t)((c / nb) * bs + c % nb) * dsize(R.dt);
  }

  hyeig_status alloc() {
    size_t blk = (size_t)R.n * ld * dsize(R.dt);
    for (int b = 0; b < 2; ++b) {
      HY_CHECK(S[b].alloc(R.ctx, blk));
      HY_CHECK(HS[b].alloc(R.ctx, blk));
      HY_CHECK(launch_fill(R.ctx, R.n, ld, S[b].p, ld, R.dt, 0.0));
      HY_CHECK(launch_fill(R.ctx, R.n, ld, HS[b].p, ld, R.dt, 0.0));
    }
    HY_CHECK(dG.alloc(R.ctx, sizeof(double) * 2 * ld * ld));
    HY_CHECK(dC.alloc(R.ctx, sizeof(double) * (2 * ld * nb + nb)));
    HY_CHECK(dnrm.alloc(R.ctx, sizeof(double) * nb));
    HY_CHECK(dpos.alloc(R.ctx, sizeof(int) * nb));
    HY_CHECK(dmlp.alloc(R.ctx, 64));
    HY_CHECK(launch_fill(R.ctx, 1, 2, dmlp.p, 2, HYEIG_F32, 0.0));  // two integer zeros (all bits clear)
    theta.assign(nb, 0.0);
    rel.assign(nb, INFINITY);
    active.assign(nb, 1);
    return HYEIG_OK;
  }

  // X0 (n x nb, FP32, ldx) -> orthonormal X, HX, Ritz pairs (the set-up of Algorithm 2)
  hyeig_status init(const float* X0, int64_t ldx, bool x0_is_internal = false) {
    hyeig_ctx* ctx = R.ctx;
    if (!x0_is_internal) HY_CHECK(launch_copy(ctx, R.n, nb, X0, ldx, HYEIG_F32, col(cur, false, 0), lds, R.dt));
    hyeig_status st = hyeig_cholqr(ctx, R.n, nb, col(cur, false, 0), lds, R.dt, 2, nullptr);
    if (st != HYEIG_OK) return st;
    HY_CHECK(R.spmm(nb, col(cur, false, 0), lds, col(cur, true, 0), lds));
    return rayleigh_ritz_block();
  }

  // Rayleigh-Ritz on span(X) alone: X <- X C, HX <- HX C
  hyeig_status rayleigh_ritz_block() {
    hyeig_ctx* ctx = R.ctx;
    double* G = dG.as<double>();
    // [X^T HX, X^T X] in one pass over X
    HY_CHECK(launch_gram2(ctx, R.n, nb, col(cur, false, 0), lds, nb, col(cur, true, 0), lds, nb, col(cur, false, 0), lds,
                          R.dt, R.gmode, G));
    std::vector<double> h(2 * nb * nb), C(nb * nb);
    HY_CHECK(d2h(ctx, h.data(), G, sizeof(double) * 2 * nb * nb));
    auto t0 = Clock::now();
    bool ok = sd::gen_eig(nb, h.data(), h.data() + nb * nb, nb, theta.data(), C.data(), nullptr);
    R.t_small += ms_since(t0);
    if (!ok) return set_err(ctx, HYEIG_ENOTSPD, "lobpcg: Rayleigh-Ritz on the start block failed");
    HY_CHECK(h2d(ctx, dC.p, C.data(), sizeof(double) * nb * nb));
    HY_CHECK(launch_block_update(ctx, R.n, nb, nb, col(cur, false, 0), lds, dC.as<double>(), 0.0, col(cur, false, 0),
                                 lds, R.dt));
    HY_CHECK(launch_block_update(ctx, R.n, nb, nb, col(cur, true, 0), lds, dC.as<double>(), 0.0, col(cur, true, 0), lds,
                                 R.dt));
    HY_CHECK(h2d(ctx, dth(), theta.data(), sizeof(double) * nb));
    haveP = false;
    return HYEIG_OK;
  }

  // The hand-back after RMM-DIIS (the paper has none): X <- the nb lowest Ritz
  // vectors of span[X Xr] (Xr: the kr refined vectors, ldr).  Xr's part outside
  // span[X] is taken by two classical Gram-Schmidt passes; columns whose
  // remainder is at rounding level (below 1e-10 of their norm in FP64, 1e-5 in
  // FP32) add no direction and are dropped; the rest is orthonormalised by
  // CholQR2 (Y) and multiplied by H (one product), and a Rayleigh-Ritz step on
  // [X Y] (eq. (rreig)) gives X and, by linearity, HX.  P, HP, the locking state
  // and the iteration count stay.  span[X] lies inside span[X Y], so no Ritz
  // value rises.  Nothing to merge leaves the state as it is (*merged false).
  hyeig_status merge_refined(const void* Xr, int64_t ldr, int kr, bool* merged) {
    hyeig_ctx* ctx = R.ctx;
    *merged = false;
    if (kr < 1 || nb + kr > 64) return HYEIG_OK;
    const size_t es = dsize(R.dt);
    char* X = col(cur, false, 0);
    char* HX = col(cur, true, 0);
    DBuf y, hy, g;
    HY_CHECK(y.alloc(ctx, (size_t)R.n * kr * es));
    HY_CHECK(hy.alloc(ctx, (size_t)R.n * kr * es));
    HY_CHECK(g.alloc(ctx, sizeof(double) * 7 * 64 * 64));
    double* gd = g.as<double>();
    HY_CHECK(launch_copy(ctx, R.n, kr, Xr, ldr, R.dt, y.p, kr, R.dt));
    std::vector<double> before(kr), after(kr);
    HY_CHECK(launch_col_dots(ctx, R.n, kr, y.p, kr, y.p, kr, R.dt, gd));
    HY_CHECK(d2h(ctx, before.data(), gd, sizeof(double) * kr));
    for (int pass = 0; pass < 2; ++pass) {
      HY_CHECK(launch_gram(ctx, R.n, nb, X, lds, kr, y.p, kr, R.dt, HYEIG_MMA_F64, gd));
      HY_CHECK(launch_block_update_a(ctx, R.n, nb, kr, X, lds, gd, -1.0, 1.0, y.p, kr, R.dt));
    }
    HY_CHECK(launch_col_dots(ctx, R.n, kr, y.p, kr, y.p, kr, R.dt, gd));
    HY_CHECK(d2h(ctx, after.data(), gd, sizeof(double) * kr));
    const double rtol = R.dt == HYEIG_F64 ? 1e-10 : 1e-5;
    int ky = 0;  // kept columns, moved to the front in order
    for (int c = 0; c < kr; ++c)
      if (std::sqrt(std::max(after[c], 0.0)) > rtol * std::sqrt(std::max(before[c], 0.0))) {
        if (ky != c) HY_CHECK(launch_copy(ctx, R.n, 1, (char*)y.p + c * es, kr, R.dt, (char*)y.p + ky * es, kr, R.dt));
        ++ky;
      }
    if (ky == 0) return HYEIG_OK;
    if (hyeig_cholqr(ctx, R.n, ky, y.p, kr, R.dt, 2, nullptr) != HYEIG_OK) return HYEIG_OK;
    HY_CHECK(R.spmm(ky, y.p, kr, hy.p, kr));
    const int q = nb + ky;
    // the seven blocks of [X Y]^T [X Y] and [X Y]^T [HX HY], with FP64 sums
    struct Blk {
      const void *a, *b;
      int64_t la, lb;
      int ka, kb, r0, c0;
      bool h;
    };
    const Blk blk[7] = {{X, X, lds, lds, nb, nb, 0, 0, false},         {X, y.p, lds, kr, nb, ky, 0, nb, false},
                        {y.p, y.p, kr, kr, ky, ky, nb, nb, false},     {X, HX, lds, lds, nb, nb, 0, 0, true},
                        {X, hy.p, lds, kr, nb, ky, 0, nb, true},       {y.p, HX, kr, lds, ky, nb, nb, 0, true},
                        {y.p, hy.p, kr, kr, ky, ky, nb, nb, true}};
    for (int b = 0; b < 7; ++b)
      HY_CHECK(launch_gram(ctx, R.n, blk[b].ka, blk[b].a, blk[b].la, blk[b].kb, blk[b].b, blk[b].lb, R.dt,
                           HYEIG_MMA_F64, gd + (size_t)b * 64 * 64));
    std::vector<double> h((size_t)7 * 64 * 64), A((size_t)q * q), B((size_t)q * q);
    HY_CHECK(d2h(ctx, h.data(), g.p, sizeof(double) * h.size()));
    for (int b = 0; b < 7; ++b) {
      const Blk& e = blk[b];
      std::vector<double>& M = e.h ? A : B;
      const double* gb = h.data() + (size_t)b * 64 * 64;
      for (int c = 0; c < e.kb; ++c)
        for (int r = 0; r < e.ka; ++r) {
          M[(e.r0 + r) + (size_t)(e.c0 + c) * q] = gb[r + (size_t)c * e.ka];
          if (!e.h) M[(e.c0 + c) + (size_t)(e.r0 + r) * q] = gb[r + (size_t)c * e.ka];  // B symmetric
        }
    }
    std::vector<double> th(nb), C((size_t)q * nb);
    auto t0 = Clock::now();
    const bool ok = sd::gen_eig(q, A.data(), B.data(), nb, th.data(), C.data(), nullptr);
    R.t_small += ms_since(t0);
    if (!ok) return HYEIG_OK;
    // X' = X C1 + Y C2 and HX' = HX C1 + HY C2 into the W columns, then back
    std::vector<double> c12((size_t)q * nb);
    for (int j = 0; j < nb; ++j)
      for (int r = 0; r < nb; ++r) c12[r + (size_t)j * nb] = C[r + (size_t)j * q];
    for (int j = 0; j < nb; ++j)
      for (int r = 0; r < ky; ++r) c12[(size_t)nb * nb + r + (size_t)j * ky] = C[(nb + r) + (size_t)j * q];
    HY_CHECK(h2d(ctx, dC.p, c12.data(), sizeof(double) * c12.size()));
    const double* C1 = dC.as<double>();
    const double* C2 = C1 + (size_t)nb * nb;
    char* Wc = col(cur, false, nb);
    char* HWc = col(cur, true, nb);
    HY_CHECK(launch_block_update_a(ctx, R.n, nb, nb, X, lds, C1, 1.0, 0.0, Wc, lds, R.dt));
    HY_CHECK(launch_block_update_a(ctx, R.n, ky, nb, y.p, kr, C2, 1.0, 1.0, Wc, lds, R.dt));
    HY_CHECK(launch_block_update_a(ctx, R.n, nb, nb, HX, lds, C1, 1.0, 0.0, HWc, lds, R.dt));
    HY_CHECK(launch_block_update_a(ctx, R.n, ky, nb, hy.p, kr, C2, 1.0, 1.0, HWc, lds, R.dt));
    HY_CHECK(launch_copy(ctx, R.n, nb, Wc, lds, R.dt, X, lds, R.dt));
    HY_CHECK(launch_copy(ctx, R.n, nb, HWc, lds, R.dt, HX, lds, R.dt));
    theta = th;
    HY_CHECK(h2d(ctx, dth(), theta.data(), sizeof(double) * nb));
    resid_fused = false;
    w_formed = false;
    *merged = true;
    return HYEIG_OK;
  }

  // Residual norms for the convergence test.  The same pass also forms W for
  // the columns that were active in the last iteration (the shifted-diagonal
  // apply, or W = R for the learned preconditioner, which then runs in place);
  // step() keeps it when the active set has not changed (the usual case), which
  // saves a second pass over X and HX.
  hyeig_status residual_norms(hyeig_precond_kind pk) {
    if (pos_dev.empty()) {
      pos_dev.resize(nb);
      for (int j = 0; j < nb; ++j) pos_dev[j] = j;
      HY_CHECK(h2d(R.ctx, dpos.p, pos_dev.data(), sizeof(int) * nb));
    }
    int na = 0;
    for (int j = 0; j < nb; ++j) na += pos_dev[j] >= 0;
    const float* dd = (pk == HYEIG_PRECOND_JACOBI) ? d : nullptr;
    if (!resid_fused)
      HY_CHECK(launch_resid_precond(R.ctx, R.n, nb, col(cur, false, 0), lds, col(cur, true, 0), lds,
                                    dth(), dd, floor_, na, dpos.as<int>(), col(cur, false, nb), lds, nb,
                                    R.dt, dnrm.as<double>()));
    resid_fused = false;
    w_formed = na > 0;
    std::vector<double> nr(nb);
    HY_CHECK(d2h(R.ctx, nr.data(), dnrm.p, sizeof(double) * nb));
    for (int j = 0; j < nb; ++j) {
      if (!std::isfinite(nr[j])) return set_err(R.ctx, HYEIG_ENUMERIC, "lobpcg: NaN/Inf residual");
      rel[j] = std::sqrt(nr[j]) / R.scale(theta[j]);
    }
    return HYEIG_OK;
  }

  // one iteration after the residual test (the body of Algorithm 2's loop)
  hyeig_status step(hyeig_precond_kind pk) {
    hyeig_ctx* ctx = R.ctx;
    const hyeig_params* p = R.p;
    ++it;
    if (p->lock) {
      // soft locking; with the stabilised basis a locked column whose residual
      // drifts back above the tolerance is re-activated
      const bool relock = stable_basis();
      for (int j = 0; j < nb; ++j) active[j] = (relock || active[j]) && (rel[j] > p->tol);
    }
    std::vector<int> idx;
    for (int j = 0; j < nb; ++j)
      if (active[j]) idx.push_back(j);
    const int na0 = (int)idx.size();
    if (na0 == 0) {
      // every column locked while the leading ones are not converged: unlock them
      for (int j = 0; j < nb; ++j) active[j] = rel[j] > p->tol || j < k;
      for (int j = 0; j < nb; ++j)
        if (active[j]) idx.push_back(j);
    }
    const int na2 = (int)idx.size();
    if (na2 == 0) return set_err(ctx, HYEIG_ENUMERIC, "lobpcg: no active column");
    const int na = na2;
    std::vector<int> pos(nb, -1);
    for (int a = 0; a < na; ++a) pos[idx[a]] = a;
    // W = K^{-1} R on the active columns (compacted), remaining W columns cleared;
    // already formed by the residual pass when the active set is the last one
    if (!(w_formed && pos == pos_dev)) {
      HY_CHECK(h2d(ctx, dpos.p, pos.data(), sizeof(int) * nb));
      pos_dev = pos;
      const float* dd = (pk == HYEIG_PRECOND_JACOBI) ? d : nullptr;
      HY_CHECK(launch_resid_precond(ctx, R.n, nb, col(cur, false, 0), lds, col(cur, true, 0), lds, dth(),
                                    dd, floor_, na, dpos.as<int>(), col(cur, false, nb), lds, nb, R.dt,
                                    dnrm.as<double>()));
    }
    w_formed = false;
    if (pk == HYEIG_PRECOND_MLP) HY_CHECK(mlp_precond(na));
    // FP32 forms: W <- orthonormal basis of (I - X X^T) W.  Same subspace, so the
    // same Ritz pairs; it bounds the update coefficients, whose growth would
    // otherwise amplify FP32 rounding in the H X / H P recurrences.
    // One Gram pass over A = [X W] (FP64 sums) gives X^T X, X^T W and W^T W; with
    // G = X^T W the projected block W - X G has the Gram W^T W - 2 G^T G + G^T (X^T X) G
    // (exact for the stored X, W), whose Cholesky factor R gives the new W in one
    // pass: W <- [X W] [-G R^-1; R^-1].
    if (stable_basis()) {
      const int ka = planar ? 2 * nb : nb + na;  // A: the X block and the W block (planar: all its columns)
      double* Gd = dG.as<double>();
      double* Kd = Gd + (size_t)ka * (nb + ka);
      HY_CHECK(launch_gram2(ctx, R.n, ka, col(cur, false, 0), lds, nb, col(cur, false, 0), lds, ka, col(cur, false, 0),
                            lds, R.dt, HYEIG_MMA_F64, Gd, planar ? bs : 0));
      std::vector<double> g((size_t)ka * (nb + ka));
      HY_CHECK(d2h(ctx, g.data(), Gd, sizeof(double) * g.size()));
      auto t1 = Clock::now();
      const double* AA = g.data() + (size_t)ka * nb;  // A^T A, ka x ka
      auto aa = [&](int i, int j) { return 0.5 * (AA[i + (size_t)j * ka] + AA[j + (size_t)i * ka]); };
      std::vector<double> G((size_t)nb * na), XG((size_t)nb * na), Gp((size_t)na * na), Rw((size_t)na * na),
          Rwi((size_t)na * na), K((size_t)ka * na, 0.0);
      for (int a = 0; a < na; ++a)
        for (int i = 0; i < nb; ++i) G[i + (size_t)a * nb] = aa(i, nb + a);
      for (int a = 0; a < na; ++a)
        for (int i = 0; i < nb; ++i) {
          double t = 0.0;
          for (int q = 0; q < nb; ++q) t += aa(i, q) * G[q + (size_t)a * nb];
          XG[i + (size_t)a * nb] = t;
        }
      for (int b = 0; b < na; ++b)
        for (int a = 0; a < na; ++a) {
          double gg = 0.0, gxg = 0.0;
          for (int q = 0; q < nb; ++q) {
            gg += G[q + (size_t)a * nb] * G[q + (size_t)b * nb];
            gxg += G[q + (size_t)a * nb] * XG[q + (size_t)b * nb];
          }
          Gp[a + (size_t)b * na] = aa(nb + a, nb + b) - 2.0 * gg + gxg;
        }
      const bool w_ortho = sd::cholesky_upper(na, Gp.data(), Rw.data());
      if (w_ortho) sd::tri_upper_inv(na, Rw.data(), Rwi.data());
      for (int b = 0; b < na; ++b)
        for (int a = 0; a < na; ++a) {
          // R^-1, or I when W^T W is not numerically positive definite (the
          // projected, unnormalised W)
          const double r = w_ortho ? Rwi[a + (size_t)b * na] : (a == b ? 1.0 : 0.0);
          K[nb + a + (size_t)b * ka] = r;
        }
      for (int b = 0; b < na; ++b)
        for (int i = 0; i < nb; ++i) {
          double t = 0.0;
          for (int a = 0; a < na; ++a) t += G[i + (size_t)a * nb] * K[nb + a + (size_t)b * ka];
          K[i + (size_t)b * ka] = -t;
        }
      R.t_small += ms_since(t1);
      HY_CHECK(h2d(ctx, Kd, K.data(), sizeof(double) * K.size()));
      HY_CHECK(launch_block_update_bs(ctx, R.n, ka, na, col(cur, false, 0), lds, planar ? bs : 0, Kd,
                                      col(cur, false, nb), lds, R.dt));
      if (!w_ortho) R.rep->events_orth_w++;  // rank deficient: the plain projected W
    }
    // H W, the only product of the iteration (Section 2.3)
    HY_CHECK(R.spmm(na, col(cur, false, nb), lds, col(cur, true, nb), lds));
    if (na < nb) HY_CHECK(launch_fill(ctx, R.n, nb - na, col(cur, true, nb + na), lds, R.dt, 0.0));
    bool useP = haveP;
    for (int attempt = 0; attempt < 3; ++attempt) {
      double* G = dG.as<double>();
      // [S^T HS, S^T S] in one pass over S
      HY_CHECK(launch_gram2(ctx, R.n, ld, col(cur, false, 0), lds, ld, col(cur, true, 0), lds, ld, col(cur, false, 0),
                            lds, R.dt, R.gmode, G, planar ? bs : 0));
      std::vector<double> h(2 * ld * ld);
      HY_CHECK(d2h(ctx, h.data(), G, sizeof(double) * 2 * ld * ld));
      auto t0 = Clock::now();
      // active subspace: X, active W (compacted), P of the active columns
      std::vector<int> sel;
      for (int j = 0; j < nb; ++j) sel.push_back(j);
      for (int a = 0; a < na; ++a) sel.push_back(nb + a);
      const bool stable = stable_basis();
      if (useP && !stable)
        for (int a = 0; a < na; ++a) sel.push_back(2 * nb + idx[a]);
      if (useP && stable)
        for (int a = 0; a < prank; ++a) sel.push_back(2 * nb + a);
      const int q = (int)sel.size();
      std::vector<double> A(q * q), B(q * q), dsc(q), th(nb), Cs(q * nb);
      for (int b = 0; b < q; ++b) dsc[b] = 1.0 / std::sqrt(std::max(h[ld * ld + sel[b] + sel[b] * ld], 1e-300));
      for (int b = 0; b < q; ++b)
        for (int a = 0; a < q; ++a) {
          const int ia = sel[a], ib = sel[b];
          A[a + b * q] = 0.5 * (h[ia + ib * ld] + h[ib + ia * ld]) * dsc[a] * dsc[b];
          B[a + b * q] = 0.5 * (h[ld * ld + ia + ib * ld] + h[ld * ld + ib + ia * ld]) * dsc[a] * dsc[b];
        }
      bool finite = true;
      for (double v : A) finite = finite && std::isfinite(v);
      for (double v : B) finite = finite && std::isfinite(v);
      if (!finite) return set_err(ctx, HYEIG_ENUMERIC, "lobpcg: NaN/Inf in projected matrices");
      // P is dropped when cond_2 of the scaled S^T S exceeds 1e12; a cheap upper bound
      // settles that in the usual case, and the exact value (reported) is then
      // formed after the update kernels are queued, off the critical path
      double bound = INFINITY, cond = NAN;
      bool ok = sd::gen_eig(q, A.data(), B.data(), nb, th.data(), Cs.data(), nullptr, &bound);
      if (ok && !(bound <= 1e12)) {
        cond = sd::spd_cond(q, B.data());
        ok = std::isfinite(cond) && cond <= 1e12;
      }
      R.t_small += ms_since(t0);
      if (ok) {
        std::vector<double> C(2 * ld * nb + nb, 0.0);  // C_full, C_P (X rows zero), then the Ritz values
        for (int c = 0; c < nb; ++c)
          for (int a = 0; a < q; ++a) {
            double v = Cs[a + c * q] * dsc[a];
            C[sel[a] + c * ld] = v;
            if (sel[a] >= nb && !stable) C[ld * nb + sel[a] + c * ld] = v;
          }
        if (stable) {
          // P' spanning the same space as eq. (pupd) together with X', but made
          // B-orthogonal to X' and B-orthonormal (FP64, on the projected basis)
          std::vector<double> Y(q * nb, 0.0), BY(q * nb), BX(q * nb), XtBY(nb * nb), Mt(nb * nb), mu(nb),
              U(nb * nb);
          for (int c = 0; c < nb; ++c)
            for (int a = nb; a < q; ++a) Y[a + c * q] = Cs[a + c * q];
          auto Bmul = [&](const std::vector<double>& Z, std::vector<double>& out) {
            for (int c = 0; c < nb; ++c)
              for (int a = 0; a < q; ++a) {
                double t = 0.0;
                for (int b = 0; b < q; ++b) t += B[a + b * q] * Z[b + c * q];
                out[a + c * q] = t;
              }
          };
          Bmul(Y, BY);
          for (int c = 0; c < nb; ++c)
            for (int r = 0; r < nb; ++r) {
              double t = 0.0;
              for (int a = 0; a < q; ++a) t += Cs[a + r * q] * BY[a + c * q];
              XtBY[r + c * nb] = t;
            }
          for (int c = 0; c < nb; ++c)
            for (int a = 0; a < q; ++a) {
              double t = 0.0;
              for (int r = 0; r < nb; ++r) t += Cs[a + r * q] * XtBY[r + c * nb];
              Y[a + c * q] -= t;
            }
          Bmul(Y, BY);
          for (int c = 0; c < nb; ++c)
            for (int r = 0; r < nb; ++r) {
              double t = 0.0;
              for (int a = 0; a < q; ++a) t += Y[a + r * q] * BY[a + c * q];
              Mt[r + c * nb] = t;
            }
          int rank = 0;
          if (sd::sym_eig(nb, Mt.data(), mu.data(), U.data())) {
            const double mmax = mu[nb - 1];
            for (int t = nb - 1; t >= 0; --t) {
              if (!(mmax > 0) || mu[t] <= 1e-10 * mmax) break;
              const double sc = 1.0 / std::sqrt(mu[t]);
              for (int a = 0; a < q; ++a) {
                double v = 0.0;
                for (int r = 0; r < nb; ++r) v += Y[a + r * q] * U[r + t * nb];
                C[ld * nb + sel[a] + rank * ld] = v * sc * dsc[a];
              }
              ++rank;
            }
          }
          prank = rank;
          if (rank == 0) R.rep->events_drop_p++;
        }
        std::copy(th.begin(), th.end(), C.begin() + 2 * ld * nb);
        HY_CHECK(h2d(ctx, dC.p, C.data(), sizeof(double) * C.size()));
        const double* C1 = dC.as<double>();
        const double* C2 = C1 + ld * nb;
        const int nx = cur ^ 1;
        theta = th;
        // the updates of S and HS, and with them the next iteration's residual
        // pass (on the device positions pos_dev, as that pass would use)
        if (!pos_dev.empty() &&
            update_resid_fits(R.n, ld, nb, lds, col(nx, false, 0), col(nx, false, 2 * nb), col(nx, true, 0),
                              col(nx, true, 2 * nb), R.dt)) {
          int nad = 0;
          for (int j = 0; j < nb; ++j) nad += pos_dev[j] >= 0;
          const float* dd = (pk == HYEIG_PRECOND_JACOBI) ? d : nullptr;
          HY_CHECK(launch_update_resid(ctx, R.n, ld, nb, S[cur].p, HS[cur].p, lds, planar ? bs : 0, C1, C2,
                                       col(nx, false, 0), col(nx, false, 2 * nb), col(nx, true, 0),
                                       col(nx, true, 2 * nb), lds, dth(), dd, floor_, dpos.as<int>(), nad,
                                       col(nx, false, nb), lds, R.dt, dnrm.as<double>()));
          resid_fused = true;
        } else {
          HY_CHECK(launch_block_update2(ctx, R.n, ld, nb, S[cur].p, lds, C1, col(nx, false, 0), lds, C2,
                                        col(nx, false, 2 * nb), lds, R.dt, planar ? bs : 0));
          HY_CHECK(launch_block_update2(ctx, R.n, ld, nb, HS[cur].p, lds, C1, col(nx, true, 0), lds, C2,
                                        col(nx, true, 2 * nb), lds, R.dt, planar ? bs : 0));
        }
        cur = nx;
        haveP = !stable || prank > 0;
        if (std::isnan(cond)) {
          auto t1 = Clock::now();
          cond = sd::spd_cond(q, B.data());
          R.t_small += ms_since(t1);
        }
        R.rep->max_cond = std::max(R.rep->max_cond, cond);
        R.cond_now = cond;
        return HYEIG_OK;
      }
      if (useP) {
        useP = false;
        R.rep->events_drop_p++;
        continue;
      }
      // orthogonalise W against X, orthonormalise it, recompute H W
      R.rep->events_orth_w++;
      double* Gx = dG.as<double>();
      HY_CHECK(launch_gram(ctx, R.n, nb, col(cur, false, 0), lds, na, col(cur, false, nb), lds, R.dt, HYEIG_MMA_F64, Gx));
      HY_CHECK(launch_block_update_a(ctx, R.n, nb, na, col(cur, false, 0), lds, Gx, -1.0, 1.0, col(cur, false, nb), lds,
                                     R.dt));
      hyeig_status st = hyeig_cholqr(ctx, R.n, na, col(cur, false, nb), lds, R.dt, 2, nullptr);
      if (st != HYEIG_OK) return set_err(ctx, HYEIG_ENUMERIC, "lobpcg: W is rank deficient after orthogonalisation");
      HY_CHECK(R.spmm(na, col(cur, false, nb), lds, col(cur, true, nb), lds));
    }
    return set_err(ctx, HYEIG_ENUMERIC, "lobpcg: Rayleigh-Ritz failed after all safeguards");
  }

  hyeig_status refresh() {
    resid_fused = false;  // H X changes: the residual pass runs again
    HY_CHECK(R.spmm(nb, col(cur, false, 0), lds, col(cur, true, 0), lds));
    R.rep->refreshes++;
    return HYEIG_OK;
  }

  // run until the leading k converge, maxiter, or the switch fires
  hyeig_status run(int maxiter, Switch* sw, bool* switched) {
    const hyeig_status st = run_steps(maxiter, sw, switched);
    const hyeig_status se = mlp_events();
    return st != HYEIG_OK ? st : se;
  }
  double worst_rel() const {
    double w = 0.0;
    for (int j = 0; j < k; ++j) w = std::isnan(rel[j]) ? INFINITY : std::max(w, rel[j]);
    return w;
  }
  hyeig_status keep_best() {
    const double w = worst_rel();
    if (!(w <= std::max(100.0 * R.p->tol, 1e-4) && w <= 0.5 * best_worst)) return HYEIG_OK;
    if (!best) {
      hyeig_status st;
      best = ws_get(R.ctx, WS_BEST, (size_t)R.n * nb * dsize(R.dt), &st);
      if (!best) return st;
    }
    HY_CHECK(launch_copy(R.ctx, R.n, nb, col(cur, false, 0), lds, R.dt, best, nb, R.dt));
    best_worst = w;
    return HYEIG_OK;
  }
  // the kept iterate in place of the current one when that is worse (or
  // unknown, after a breakdown)
  hyeig_status restore_best(bool known) {
    if (!(best_worst < INFINITY) || (known && worst_rel() <= best_worst)) return HYEIG_OK;
    return launch_copy(R.ctx, R.n, nb, best, nb, R.dt, col(cur, false, 0), lds, R.dt);
  }
  // a breakdown after a kept iterate: that iterate, unconverged
  hyeig_status recover(hyeig_status st) {
    if (st != HYEIG_ENUMERIC || !(best_worst < INFINITY)) return st;
    HY_CHECK(restore_best(false));
    return set_err(R.ctx, HYEIG_ENOCONV, "lobpcg: breakdown near the tolerance; the best iterate is returned");
  }
  hyeig_status run_steps(int maxiter, Switch* sw, bool* switched) {
    const hyeig_params* p = R.p;
    if (switched) *switched = false;
    int since_refresh = 0;
    best_worst = INFINITY;
    for (;;) {
      if (R.dt == HYEIG_F32 && p->refresh_every > 0 && since_refresh >= p->refresh_every) {
        HY_CHECK(refresh());
        since_refresh = 0;
      }
      const hyeig_status sr = residual_norms(p->precond);
      if (sr != HYEIG_OK) return recover(sr);
      R.clk.collect();
      R.hist(rel.data(), k);
      bool conv = true;
      for (int j = 0; j < k; ++j) conv = conv && rel[j] <= p->tol;
      if (conv) return HYEIG_OK;
      HY_CHECK(keep_best());
      if (sw && sw->fire(it, theta.data(), rel.data(), k)) {
        if (switched) *switched = true;
        return HYEIG_OK;
      }
      if (it >= maxiter) {
        // a hybrid hands over at the front end's limit (a fixed switch point)
        if (sw && sw->enabled && switched) {
          *switched = true;
          return HYEIG_OK;
        }
        HY_CHECK(restore_best(true));
        return HYEIG_ENOCONV;
      }
      const hyeig_status ss = step(p->precond);
      if (ss != HYEIG_OK) return recover(ss);
      ++since_refresh;
    }
  }
};

// ---------------------------------------------------------------------------
// RMM-DIIS, batched (Algorithm 4; one product per sweep, Section 4.2)
// ---------------------------------------------------------------------------
struct Rmm {
  hyeig_ctx* ctx;
  const hyeig_mat* H;
  int64_t n;
  int k, smax;
  hyeig_dtype dt;
  DBuf X, HX, Rr, Xt, HXt, Zt, HZ, Xh, Rh, dalpha, dthh, dact, dcoef, dg, ddots, dgram;
  std::vector<double> theta, rel, thetat, best;
  std::vector<int> conv, best_it;
  std::vector<std::vector<double>> best_log;  // best residuals after each sweep
  std::vector<std::vector<double>> thetah;   // [j][slot]
  std::vector<std::vector<double>> Bfull;    // [j] smax x smax Gram over ring slots
  int count = 0;                              // entries pushed so far
  int sweeps = 0;
  double tol = 1e-6, hnorm = 1.0;
  int precond = 0;
  const float* d = nullptr;
  double floor_ = 0.0;
  bool theta_norm = false;
  int decouple_after = 0;  // > 0: one SpMV per unconverged column once that many have converged
  SpmmClock* clk = nullptr;
  hyeig_report* rep = nullptr;

  size_t bs() const { return (size_t)n * k * dsize(dt); }
  char* slot_ptr(DBuf& b, int s) { return (char*)b.p + (size_t)s * bs(); }
  double scale(double th) const { return theta_norm ? std::max(std::fabs(th), 1e-300) : hnorm; }

  hyeig_status alloc() {
    for (DBuf* b : {&X, &HX, &Rr, &Xt, &HXt, &Zt, &HZ}) HY_CHECK(b->alloc(ctx, bs()));
    HY_CHECK(Xh.alloc(ctx, bs() * smax));
    HY_CHECK(Rh.alloc(ctx, bs() * smax));
    HY_CHECK(dalpha.alloc(ctx, sizeof(double) * k * RMM_SMAX));
    HY_CHECK(dthh.alloc(ctx, sizeof(double) * k * RMM_SMAX));
    HY_CHECK(dact.alloc(ctx, sizeof(int) * k));
    HY_CHECK(dcoef.alloc(ctx, sizeof(double) * 3 * k));
    HY_CHECK(dg.alloc(ctx, sizeof(double) * 6 * k));
    HY_CHECK(ddots.alloc(ctx, sizeof(double) * k * (RMM_SMAX + 1)));
    HY_CHECK(dgram.alloc(ctx, sizeof(double) * k * k));
    theta.assign(k, 0.0);
    rel.assign(k, INFINITY);
    thetat.assign(k, 0.0);
    best.assign(k, INFINITY);
    best_it.assign(k, 0);
    best_log.clear();
    conv.assign(k, 0);
    thetah.assign(k, std::vector<double>(RMM_SMAX, 0.0));
    Bfull.assign(k, std::vector<double>(RMM_SMAX * RMM_SMAX, 0.0));
    return HYEIG_OK;
  }

  hyeig_status spmm_block(const void* src, void* dst) {
    if (clk) clk->start(ctx);
    HY_CHECK(launch_spmm(ctx, H, k, src, k, dt, dst, k, dt, HYEIG_F32));
    const double b = spmm_bytes(H, k, dt, dt, HYEIG_F32);
    if (clk) clk->stop(spmm_on_matrix_cores(H, k, dt, dt, HYEIG_F32), b);
    if (rep) {
      rep->spmm_count++;
      rep->spmv_count += k;
      rep->bytes_spmm += b;
    }
    return HYEIG_OK;
  }

  // column j alone (the decoupled form): an SpMV on the strided column j of
  // the n x k block; the other columns of dst are left as they are
  hyeig_status spmv_col(const void* src, void* dst, int j) {
    const size_t off = (size_t)j * dsize(dt);
    if (clk) clk->start(ctx);
    HY_CHECK(launch_spmm(ctx, H, 1, (const char*)src + off, k, dt, (char*)dst + off, k, dt, HYEIG_F32));
    if (clk) clk->stop(false, spmm_bytes(H, 1, dt, dt, HYEIG_F32));
    if (rep) {
      rep->spmm_count++;
      rep->spmv_count += 1;
      rep->bytes_spmm += spmm_bytes(H, 1, dt, dt, HYEIG_F32);
    }
    return HYEIG_OK;
  }

  std::vector<int> window() const {
    int w = std::min(count, smax);
    std::vector<int> s(w);
    for (int l = 0; l < w; ++l) s[l] = (count - w + l) % smax;
    return s;
  }

  // start: x <- x/||x||, theta, r (the set-up of Algorithm 4); HX given or computed
  hyeig_status start(const void* Xin, int64_t ldx, hyeig_dtype xdt, const void* HXin, int64_t ldhx) {
    HY_CHECK(launch_copy(ctx, n, k, Xin, ldx, xdt, X.p, k, dt));
    if (HXin)
      HY_CHECK(launch_copy(ctx, n, k, HXin, ldhx, xdt, HX.p, k, dt));
    else
      HY_CHECK(spmm_block(X.p, HX.p));
    double* dd = ddots.as<double>();
    HY_CHECK(launch_col_dots(ctx, n, k, X.p, k, X.p, k, dt, dd));
    HY_CHECK(launch_col_dots(ctx, n, k, X.p, k, HX.p, k, dt, dd + k));
    std::vector<double> h(2 * k);
    HY_CHECK(d2h(ctx, h.data(), dd, sizeof(double) * 2 * k));
    std::vector<double> sc(k);
    for (int j = 0; j < k; ++j) {
      if (!(h[j] > 0)) return set_err(ctx, HYEIG_ENUMERIC, "rmm: zero start vector");
      sc[j] = 1.0 / std::sqrt(h[j]);
      theta[j] = h[k + j] / h[j];
    }
    HY_CHECK(h2d(ctx, dcoef.p, sc.data(), sizeof(double) * k));
    HY_CHECK(launch_col_scale(ctx, n, k, X.p, k, dcoef.as<double>(), dt));
    HY_CHECK(launch_col_scale(ctx, n, k, HX.p, k, dcoef.as<double>(), dt));
    // r = Hx - theta x, pushed as history entry 0, with its DIIS Gram entry
    std::vector<double> g(3 * k);
    std::vector<int> act(k, 1);
    for (int j = 0; j < k; ++j) {
      g[3 * j] = 1.0;
      g[3 * j + 1] = 0.0;
      g[3 * j + 2] = theta[j];
    }
    HY_CHECK(h2d(ctx, dg.p, g.data(), sizeof(double) * 3 * k));
    HY_CHECK(h2d(ctx, dact.p, act.data(), sizeof(int) * k));
    HY_CHECK(launch_fill(ctx, n, k, Zt.p, k, dt, 0.0));
    HY_CHECK(launch_fill(ctx, n, k, HZ.p, k, dt, 0.0));
    HY_CHECK(launch_copy(ctx, n, k, X.p, k, dt, Xt.p, k, dt));
    HY_CHECK(launch_copy(ctx, n, k, HX.p, k, dt, HXt.p, k, dt));
    HY_CHECK(push_update(g, act));
    best = rel;
    std::fill(best_it.begin(), best_it.end(), 0);
    return HYEIG_OK;
  }

  // x = g0 x~ + g1 z, etc.; pushes (x, r) and refreshes the DIIS Gram rows
  hyeig_status push_update(const std::vector<double>& g, const std::vector<int>& act) {
    const int slot = count % smax;
    std::vector<int> win_after;
    {
      int cnt = count + 1, w = std::min(cnt, smax);
      for (int l = 0; l < w; ++l) win_after.push_back((cnt - w + l) % smax);
    }
    HY_CHECK(launch_rmm_update(ctx, dt, n, k, dg.as<double>(), dact.as<int>(), Xt.p, Zt.p, HXt.p, HZ.p, X.p, HX.p,
                               Rr.p, Xh.p, Rh.p, slot, (int)win_after.size(), win_after.data(), ddots.as<double>()));
    std::vector<double> h(k * (RMM_SMAX + 1));
    HY_CHECK(d2h(ctx, h.data(), ddots.p, sizeof(double) * k * (RMM_SMAX + 1)));
    ++count;
    for (int j = 0; j < k; ++j) {
      if (!act[j]) continue;
      theta[j] = g[3 * j + 2];
      thetah[j][slot] = theta[j];
      const double rr = h[j * (RMM_SMAX + 1)];
      if (!std::isfinite(rr)) return set_err(ctx, HYEIG_ENUMERIC, "rmm: NaN/Inf residual");
      rel[j] = std::sqrt(rr) / scale(theta[j]);
      auto& B = Bfull[j];
      for (size_t l = 0; l < win_after.size(); ++l) {
        const int s2 = win_after[l];
        const double v = h[j * (RMM_SMAX + 1) + 1 + l];
        B[slot + s2 * RMM_SMAX] = v;
        B[s2 + slot * RMM_SMAX] = v;
      }
      if (rel[j] <= tol) conv[j] = 1;
    }
    return HYEIG_OK;
  }

  // one sweep (the body of Algorithm 4's loop for all unconverged columns)
  hyeig_status sweep() {
    ++sweeps;
    std::vector<int> act(k);
    for (int j = 0; j < k; ++j) act[j] = !conv[j];
    HY_CHECK(h2d(ctx, dact.p, act.data(), sizeof(int) * k));
    std::vector<int> win = window();
    const int w = (int)win.size();
    if (sweeps == 1) {
      // x~ = x^(0), r~ = r^(0)
      HY_CHECK(launch_copy(ctx, n, k, X.p, k, dt, Xt.p, k, dt));
      HY_CHECK(launch_copy(ctx, n, k, HX.p, k, dt, HXt.p, k, dt));
      std::vector<double> coef(2 * k);
      for (int j = 0; j < k; ++j) {
        coef[2 * j] = 1.0;
        coef[2 * j + 1] = theta[j];
        thetat[j] = theta[j];
      }
      HY_CHECK(h2d(ctx, dcoef.p, coef.data(), sizeof(double) * 2 * k));
    } else {
      // DIIS coefficients (eq. (xsum)-(rmm)) per column, FP64 on the host
      std::vector<double> alpha(k * RMM_SMAX, 0.0), th(k * RMM_SMAX, 0.0);
      for (int j = 0; j < k; ++j) {
        if (!act[j]) continue;
        std::vector<double> Bw(w * w), a(w);
        for (int b = 0; b < w; ++b)
          for (int c = 0; c < w; ++c) Bw[b + c * w] = Bfull[j][win[b] + win[c] * RMM_SMAX];
        sd::diis(w, Bw.data(), a.data());

        for (int l = 0; l < w; ++l) {
          alpha[j * RMM_SMAX + l] = a[l];
          th[j * RMM_SMAX + l] = thetah[j][win[l]];
        }
      }
      HY_CHECK(h2d(ctx, dalpha.p, alpha.data(), sizeof(double) * k * RMM_SMAX));
      HY_CHECK(h2d(ctx, dthh.p, th.data(), sizeof(double) * k * RMM_SMAX));
      double* dd = ddots.as<double>();
      HY_CHECK(launch_rmm_combine(ctx, dt, n, k, Xh.p, Rh.p, w, win.data(), dalpha.as<double>(), dthh.as<double>(),
                                  dact.as<int>(), Xt.p, HXt.p, dd));
      std::vector<double> h(2 * k);
      HY_CHECK(d2h(ctx, h.data(), dd, sizeof(double) * 2 * k));
      std::vector<double> coef(2 * k, 0.0);
      for (int j = 0; j < k; ++j) {
        if (!act[j]) continue;
        if (!(h[2 * j] > 0) || !std::isfinite(h[2 * j]))
          return set_err(ctx, HYEIG_ENUMERIC, "rmm: degenerate DIIS combination");
        thetat[j] = h[2 * j + 1] / h[2 * j];
        coef[2 * j] = 1.0 / std::sqrt(h[2 * j]);
        coef[2 * j + 1] = thetat[j];
      }
      HY_CHECK(h2d(ctx, dcoef.p, coef.data(), sizeof(double) * 2 * k));
    }
    // x~ normalised, r~ = H x~ - theta~ x~, optional preconditioning, into Zt
    HY_CHECK(launch_rmm_scale(ctx, dt, n, k, dcoef.as<double>(), dact.as<int>(), Xt.p, HXt.p, Zt.p,
                              precond ? d : nullptr, floor_));
    // the product of the sweep (Section 4.2): coupled, one product over all k
    // columns with the converged ones frozen in it; or decoupled, once
    // decouple_after columns have converged, one SpMV per unconverged column
    // (the columns of converged ones are cleared: their terms are not used)
    int nconv = 0;
    for (int j = 0; j < k; ++j) nconv += conv[j] ? 1 : 0;
    if (decouple_after > 0 && nconv >= decouple_after) {
      for (int j = 0; j < k; ++j) {
        if (act[j])
          HY_CHECK(spmv_col(Zt.p, HZ.p, j));
        else
          HY_CHECK(launch_fill(ctx, n, 1, (char*)HZ.p + (size_t)j * dsize(dt), k, dt, 0.0));
      }
    } else {
      HY_CHECK(spmm_block(Zt.p, HZ.p));
    }
    HY_CHECK(launch_rmm_gram6(ctx, dt, n, k, Xt.p, Zt.p, HXt.p, HZ.p, ddots.as<double>()));
    std::vector<double> g6(6 * k);
    HY_CHECK(d2h(ctx, g6.data(), ddots.p, sizeof(double) * 6 * k));
    std::vector<double> g(3 * k, 0.0);
    for (int j = 0; j < k; ++j) {
      if (!act[j]) continue;
      const double* q = &g6[6 * j];
      double th, g0, g1;
      // 2x2 pencil on span{x~, z} (eq. (rr)-(xuwg)); degenerate z keeps x~
      if (!(q[5] > 1e-300) || !sd::rr2(q[0], q[1], q[2], q[3], q[4], q[5], &th, &g0, &g1)) {
        g0 = 1.0 / std::sqrt(std::max(q[3], 1e-300));
        g1 = 0.0;
        th = q[0] / std::max(q[3], 1e-300);
      }
      g[3 * j] = g0;
      g[3 * j + 1] = g1;
      g[3 * j + 2] = th;

    }
    HY_CHECK(h2d(ctx, dg.p, g.data(), sizeof(double) * 3 * k));
    HY_CHECK(push_update(g, act));
    for (int j = 0; j < k; ++j) {
      if (!act[j]) continue;
      if (rel[j] < best[j]) {
        best[j] = rel[j];
        best_it[j] = sweeps;
      }
    }
    best_log.push_back(best);
    return HYEIG_OK;
  }

  // Columns that converged onto the same eigenpairs (RMM-DIIS refines each
  // column on its own, and on clustered spectra several can reach one pair,
  // leaving wanted pairs out): the largest off-diagonal entry of the
  // normalised Gram matrix of X above 1e-4.
  hyeig_status collapsed(bool* out) {
    HY_CHECK(launch_gram(ctx, n, k, X.p, k, k, X.p, k, dt, HYEIG_MMA_F64, dgram.as<double>()));
    std::vector<double> G((size_t)k * k);
    HY_CHECK(d2h(ctx, G.data(), dgram.p, sizeof(double) * k * k));
    double worst = 0.0;
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i)
        if (i != j)
          worst = std::max(worst, std::fabs(G[i + j * k]) / std::sqrt(std::max(G[i + i * k] * G[j + j * k], 1e-300)));
    *out = !(worst <= 1e-4);
    return HYEIG_OK;
  }

  bool all_converged(int kk) const {
    for (int j = 0; j < kk; ++j)
      if (!conv[j]) return false;
    return true;
  }

  // stagnation: an unconverged column 10x above its best, no new best for
  // 2 s_max sweeps, or a best that has not halved over the last s_max sweeps,
  // one DIIS window (where RMM-DIIS works it gains orders of magnitude in that many)
  bool stagnated(int kk) const {
    const size_t w = (size_t)smax;
    for (int j = 0; j < kk; ++j) {
      if (conv[j]) continue;
      if (rel[j] > 10 * best[j] || sweeps - best_it[j] > 2 * smax) return true;
      if (best_log.size() > w && best[j] > 0.5 * best_log[best_log.size() - 1 - w][j]) return true;
    }
    return false;
  }
};

// ---------------------------------------------------------------------------
// block Lanczos (Algorithm 1).  The basis is one row-major n x (cap * nb)
// block (ld = cap * nb); block i is the column slice i * nb.
// ---------------------------------------------------------------------------
struct BLanczos {
  Run& R;
  int nb, k, cap;
  int64_t ldv;
  DBuf V, U, dG, dR;
  std::vector<std::vector<double>> As, Rs;
  std::vector<double> theta, Q, rel;
  int it = 0;
  // deflation: dead[c] marks a zero column c of the current block (and of
  // every later one); live[b] counts the nonzero columns of block b and
  // dead_at[b] lists them
  std::vector<char> dead;
  std::vector<int> live;
  std::vector<std::vector<int>> dead_at;

  BLanczos(Run& r, int nb_, int k_, int cap_)
      : R(r), nb(nb_), k(k_), cap(cap_), ldv((int64_t)cap_ * nb_), dead(nb_, 0), live(1, nb_), dead_at(1) {}
  char* vcol(int blk) { return (char*)V.p + (size_t)blk * nb * dsize(R.dt); }
  // dimension of the Krylov basis behind T (the zero columns left out)
  int real_dim() const {
    int s = 0;
    for (int b = 0; b < it; ++b) s += live[b];
    return s;
  }
  // a column of W whose part independent of the columns before it is below
  // this size is taken as a rounding-level remainder of an exhausted direction
  double dep_tol() const { return (R.dt == HYEIG_F64 ? 1e-7 : 1e-5) * R.hnorm; }

  // W (in U) has numerically dependent columns.  A Cholesky factorisation of
  // its Gram matrix that passes over columns whose remaining pivot is below
  // dep_tol() picks the independent set J in column order; CholeskyQR of W_J
  // gives the columns J of V_{i+1}, the others are set to zero, and
  // R_{i+1} = V_{i+1}^T W is upper triangular (each dropped column lies in the
  // span of the kept ones before it) with zero rows outside J.  A zero column
  // stays zero (H 0 = 0 and its entries of A and R are zero), so it is
  // decoupled from T for the rest of the run.
  hyeig_status deflate(int i, std::vector<double>& Rn) {
    hyeig_ctx* ctx = R.ctx;
    const size_t es = dsize(R.dt);
    HY_CHECK(launch_gram(ctx, R.n, nb, U.p, nb, nb, U.p, nb, R.dt, R.gmode, dG.as<double>()));
    std::vector<double> G(nb * nb), L(nb * nb, 0.0);
    HY_CHECK(d2h(ctx, G.data(), dG.p, sizeof(double) * nb * nb));
    const double t2 = dep_tol() * dep_tol();
    std::vector<int> J;
    for (int c = 0; c < nb; ++c) {
      if (dead[c]) continue;
      double d = G[c + c * nb];
      for (int a : J) d -= L[a + c * nb] * L[a + c * nb];
      if (!(d > t2)) continue;
      const double r = std::sqrt(d);
      L[c + c * nb] = r;
      for (int e = c + 1; e < nb; ++e) {
        double s = 0.5 * (G[c + e * nb] + G[e + c * nb]);
        for (int a : J) s -= L[a + c * nb] * L[a + e * nb];
        L[c + e * nb] = s / r;
      }
      J.push_back(c);
    }
    const int nj = (int)J.size();
    char* Vn = vcol(i + 1);
    if (nj > 0) {
      for (int t = 0; t < nj; ++t)
        HY_CHECK(launch_copy(ctx, R.n, 1, (const char*)U.p + (size_t)J[t] * es, nb, R.dt, Vn + (size_t)t * es, ldv, R.dt));
      hyeig_status st = hyeig_cholqr(ctx, R.n, nj, Vn, ldv, R.dt, 2, nullptr);
      if (st != HYEIG_OK)
        return set_err(ctx, HYEIG_ENUMERIC, "blanczos: the independent columns of the new block are not orthonormalisable");
      // spread back to the positions J (J[t] >= t: from the last one down)
      for (int t = nj - 1; t >= 0; --t)
        if (J[t] != t)
          HY_CHECK(launch_copy(ctx, R.n, 1, Vn + (size_t)t * es, ldv, R.dt, Vn + (size_t)J[t] * es, ldv, R.dt));
    }
    std::vector<char> keep(nb, 0);
    for (int c : J) keep[c] = 1;
    for (int c = 0; c < nb; ++c)
      if (!keep[c]) HY_CHECK(launch_fill(ctx, R.n, 1, Vn + (size_t)c * es, ldv, R.dt, 0.0));
    HY_CHECK(launch_gram(ctx, R.n, nb, Vn, ldv, nb, U.p, nb, R.dt, R.gmode, dG.as<double>()));
    HY_CHECK(d2h(ctx, Rn.data(), dG.p, sizeof(double) * nb * nb));
    for (int c = 0; c < nb; ++c)
      for (int a = 0; a < nb; ++a)
        if (a > c || !keep[a]) Rn[a + c * nb] = 0.0;
    for (int c = 0; c < nb; ++c) dead[c] = !keep[c];
    R.rep->events_deflation++;
    return HYEIG_OK;
  }

  hyeig_status alloc() {
    HY_CHECK(V.alloc(R.ctx, (size_t)R.n * ldv * dsize(R.dt)));
    HY_CHECK(U.alloc(R.ctx, (size_t)R.n * nb * dsize(R.dt)));
    HY_CHECK(dG.alloc(R.ctx, sizeof(double) * 64 * std::max(2 * nb, 32)));
    HY_CHECK(dR.alloc(R.ctx, sizeof(double) * std::max(nb * nb, 32)));
    return HYEIG_OK;
  }

  // W -= Vall (Vall^T W) over the first nblk blocks, in chunks of up to 64 columns
  hyeig_status project_out(int nblk) {
    hyeig_ctx* ctx = R.ctx;
    const int cols = nblk * nb;
    for (int c0 = 0; c0 < cols; c0 += 64) {
      const int w = std::min(64, cols - c0);
      const char* Vc = (const char*)V.p + (size_t)c0 * dsize(R.dt);
      HY_CHECK(launch_gram(ctx, R.n, w, Vc, ldv, nb, U.p, nb, R.dt, R.gmode, dG.as<double>()));
      HY_CHECK(launch_block_update_a(ctx, R.n, w, nb, Vc, ldv, dG.as<double>(), -1.0, 1.0, U.p, nb, R.dt));
    }
    return HYEIG_OK;
  }

  hyeig_status start(const float* X0, int64_t ldx) {
    HY_CHECK(launch_copy(R.ctx, R.n, nb, X0, ldx, HYEIG_F32, vcol(0), ldv, R.dt));
    hyeig_status st = hyeig_cholqr(R.ctx, R.n, nb, vcol(0), ldv, R.dt, 2, nullptr);
    if (st != HYEIG_OK) return st;
    return HYEIG_OK;
  }

  // one iteration: product, three-term recurrence, CGS2, QR; Ritz pairs of T_i
  hyeig_status step() {
    hyeig_ctx* ctx = R.ctx;
    const int i = it;  // V_i = block i (0-based)
    if (live[i] == 0)
      return set_err(ctx, HYEIG_ENOCONV, "blanczos: the Krylov space is exhausted before the wanted pairs converged");
    HY_CHECK(R.spmm(nb, vcol(i), ldv, U.p, nb));
    HY_CHECK(launch_gram(ctx, R.n, nb, vcol(i), ldv, nb, U.p, nb, R.dt, R.gmode, dG.as<double>()));
    std::vector<double> A(nb * nb);
    HY_CHECK(d2h(ctx, A.data(), dG.p, sizeof(double) * nb * nb));
    for (int b = 0; b < nb; ++b)
      for (int a = 0; a < b; ++a) {
        double v = 0.5 * (A[a + b * nb] + A[b + a * nb]);
        A[a + b * nb] = A[b + a * nb] = v;
      }
    for (int c = 0; c < nb; ++c)
      if (dead[c])
        for (int a = 0; a < nb; ++a) A[a + c * nb] = A[c + a * nb] = 0.0;
    As.push_back(A);
    // W = U - V_i A_i - V_{i-1} R_i^T  (full re-orthogonalisation follows)
    HY_CHECK(h2d(ctx, dG.p, A.data(), sizeof(double) * nb * nb));
    HY_CHECK(launch_block_update_a(ctx, R.n, nb, nb, vcol(i), ldv, dG.as<double>(), -1.0, 1.0, U.p, nb, R.dt));
    if (i > 0) {
      std::vector<double> Rt(nb * nb);
      const auto& Rp = Rs.back();
      for (int b = 0; b < nb; ++b)
        for (int a = 0; a < nb; ++a) Rt[a + b * nb] = Rp[b + a * nb];
      HY_CHECK(h2d(ctx, dG.p, Rt.data(), sizeof(double) * nb * nb));
      HY_CHECK(launch_block_update_a(ctx, R.n, nb, nb, vcol(i - 1), ldv, dG.as<double>(), -1.0, 1.0, U.p, nb, R.dt));
    }
    // eq. (bgs) as two classical Gram-Schmidt passes against all blocks
    HY_CHECK(project_out(i + 1));
    HY_CHECK(project_out(i + 1));
    // W = V_{i+1} R_{i+1}
    if (i + 1 >= cap) return set_err(ctx, HYEIG_ENOCONV, "blanczos: basis capacity reached");
    std::vector<double> Rn(nb * nb);
    bool dependent = std::count(dead.begin(), dead.end(), 1) > 0;
    if (!dependent) {
      HY_CHECK(launch_copy(ctx, R.n, nb, U.p, nb, R.dt, vcol(i + 1), ldv, R.dt));
      hyeig_status st = hyeig_cholqr(ctx, R.n, nb, vcol(i + 1), ldv, R.dt, 2, dR.as<double>());
      if (st == HYEIG_OK) {
        HY_CHECK(d2h(ctx, Rn.data(), dR.p, sizeof(double) * nb * nb));
        for (int c = 0; c < nb; ++c) dependent = dependent || !(std::fabs(Rn[c + c * nb]) > dep_tol());
      } else {
        dependent = true;
      }
    }
    if (dependent) HY_CHECK(deflate(i, Rn));
    live.push_back(nb - (int)std::count(dead.begin(), dead.end(), 1));
    dead_at.emplace_back();
    for (int c = 0; c < nb; ++c)
      if (dead[c]) dead_at.back().push_back(c);
    Rs.push_back(Rn);
    ++it;
    // T_it: block tridiagonal from A and R (eq. (blanfac))
    const int m = nb * it;
    std::vector<double> T((size_t)m * m, 0.0);
    for (int b = 0; b < it; ++b) {
      for (int c = 0; c < nb; ++c)
        for (int a = 0; a < nb; ++a) T[(b * nb + a) + (size_t)(b * nb + c) * m] = As[b][a + c * nb];
      if (b + 1 < it)
        for (int c = 0; c < nb; ++c)
          for (int a = 0; a < nb; ++a) {
            const double v = Rs[b][a + c * nb];  // R_{b+1}: row block b+1, column block b
            T[((b + 1) * nb + a) + (size_t)(b * nb + c) * m] = v;
            T[(b * nb + c) + (size_t)((b + 1) * nb + a) * m] = v;
          }
    }
    // a zero column's row and column of T are zero: its diagonal entry is set
    // above every Ritz value of the rest (2 ||T||_F + 1 > ||T||_2), so that its
    // decoupled eigenvalue comes after all of them
    if (real_dim() < m) {
      double f2 = 0.0;
      for (double v : T) f2 += v * v;
      const double big = 2.0 * std::sqrt(f2) + 1.0;
      for (int b = 0; b < it; ++b)
        for (int c : dead_at[b]) T[(b * nb + c) + (size_t)(b * nb + c) * m] = big;
    }
    // the lowest Ritz pairs only (up to the 32 columns a hand-over may take):
    // T is a band matrix of half-width nb (the R blocks are upper triangular)
    const int want = std::min(m, 32);
    theta.assign(want, 0.0);
    Q.assign((size_t)m * want, 0.0);
    auto t0 = Clock::now();
    bool ok = sd::sym_band_eig_lowest(m, T.data(), want, theta.data(), Q.data());
    R.t_small += ms_since(t0);
    if (!ok) return set_err(ctx, HYEIG_ENUMERIC, "blanczos: eigensolver of T failed");
    // Ritz residuals ||R_{i+1} E_i^T q_j||
    const int kk = std::min(k, m);
    rel.assign(kk, 0.0);
    for (int j = 0; j < kk; ++j) {
      double s = 0.0;
      for (int a = 0; a < nb; ++a) {
        double v = 0.0;
        for (int c = a; c < nb; ++c) v += Rn[a + c * nb] * Q[(m - nb + c) + (size_t)j * m];
        s += v * v;
      }
      rel[j] = std::sqrt(s) / R.scale(theta[j]);
    }
    // past the basis dimension the values are the decoupled zero columns
    for (int j = real_dim(); j < kk; ++j) rel[j] = INFINITY;
    return HYEIG_OK;
  }

  // X = V Q(:, :cnt) and H X = X Theta + V_{i+1} R_{i+1} E_i^T Q(:, :cnt) (n x cnt, ldx, dtype
  // R.dt; cnt <= min(32, nb * it))
  hyeig_status extract(void* X, int64_t ldx, void* HX, int64_t ldhx, int cnt) {
    hyeig_ctx* ctx = R.ctx;
    const int m = nb * it;
    if (cnt > std::min(32, m)) return set_err(ctx, HYEIG_EINVAL, "blanczos: too many Ritz vectors asked for");
    const int k = cnt;
    std::vector<double> Ck(64 * k);
    for (int c0 = 0; c0 < m; c0 += 64) {
      const int w = std::min(64, m - c0);
      for (int j = 0; j < k; ++j)
        for (int a = 0; a < w; ++a) Ck[a + j * w] = Q[(c0 + a) + (size_t)j * m];
      HY_CHECK(h2d(ctx, dG.p, Ck.data(), sizeof(double) * w * k));
      HY_CHECK(launch_block_update_a(ctx, R.n, w, k, (const char*)V.p + (size_t)c0 * dsize(R.dt), ldv,
                                     dG.as<double>(), 1.0, c0 == 0 ? 0.0 : 1.0, X, ldx, R.dt));
    }
    // H X = X Theta + V_{it} (R E^T Q)
    HY_CHECK(launch_copy(ctx, R.n, k, X, ldx, R.dt, HX, ldhx, R.dt));
    std::vector<double> th(theta.begin(), theta.begin() + k);
    HY_CHECK(h2d(ctx, dR.p, th.data(), sizeof(double) * k));
    HY_CHECK(launch_col_scale(ctx, R.n, k, HX, ldhx, dR.as<double>(), R.dt));
    const auto& Rn = Rs.back();
    std::vector<double> RQ(nb * k, 0.0);
    for (int j = 0; j < k; ++j)
      for (int a = 0; a < nb; ++a) {
        double v = 0.0;
        for (int c = a; c < nb; ++c) v += Rn[a + c * nb] * Q[(m - nb + c) + (size_t)j * m];
        RQ[a + j * nb] = v;
      }
    HY_CHECK(h2d(ctx, dG.p, RQ.data(), sizeof(double) * nb * k));
    HY_CHECK(launch_block_update_a(ctx, R.n, nb, k, vcol(it), ldv, dG.as<double>(), 1.0, 1.0, HX, ldhx, R.dt));
    return HYEIG_OK;
  }
};

// ---------------------------------------------------------------------------
// Chebyshev-filtered subspace iteration (Algorithm 3, Section 2.4).  Q and HQ
// (n x nb, row-major) hold the Ritz vectors and their images.  Per iteration
// the unlocked columns are gathered into the filter buffers (n x na) and run
// through the first-kind recurrence of eq. (chebypoly) on the interval
// [lambda_F, lambda_ub] (degree - 1 products: the first step uses H Q); the
// filtered block is projected against the locked columns, orthonormalised by
// CholeskyQR (twice) and multiplied by H (one product); Rayleigh-Ritz on
// [locked | filtered] with the stored H Q of the locked columns gives the next
// Q, HQ.  Converged columns of the leading k are locked (Section 3).
// ---------------------------------------------------------------------------
struct ChebFsi {
  Run& R;
  int nb, k, degree;
  DBuf Q, HQ, Qn, HQn, F[3], HF, dG, dS, dth, dnrm, dpos, didx;
  std::vector<double> theta, rel;
  double lub = 0.0;
  int it = 0;

  ChebFsi(Run& r, int nb_, int k_, int d_) : R(r), nb(nb_), k(k_), degree(d_) {}
  size_t es() const { return dsize(R.dt); }
  char* col(DBuf& b, int c) { return (char*)b.p + (size_t)c * es(); }

  hyeig_status alloc() {
    const size_t blk = (size_t)R.n * nb * es();
    for (DBuf* b : {&Q, &HQ, &Qn, &HQn, &F[0], &F[1], &F[2], &HF}) HY_CHECK(b->alloc(R.ctx, blk));
    HY_CHECK(dG.alloc(R.ctx, sizeof(double) * nb * nb));
    HY_CHECK(dS.alloc(R.ctx, sizeof(double) * nb * nb));
    HY_CHECK(dth.alloc(R.ctx, sizeof(double) * nb));
    HY_CHECK(dnrm.alloc(R.ctx, sizeof(double) * nb));
    HY_CHECK(dpos.alloc(R.ctx, sizeof(int) * nb));
    HY_CHECK(didx.alloc(R.ctx, sizeof(int) * nb));
    theta.assign(nb, 0.0);
    rel.assign(nb, INFINITY);
    return HYEIG_OK;
  }

  // Rayleigh-Ritz on (Qn, HQn): T = Qn^T H Qn, T S = S Theta; Q = Qn S, HQ = HQn S
  hyeig_status rayleigh_ritz() {
    hyeig_ctx* ctx = R.ctx;
    HY_CHECK(launch_gram(ctx, R.n, nb, Qn.p, nb, nb, HQn.p, nb, R.dt, R.gmode, dG.as<double>()));
    std::vector<double> T(nb * nb), S(nb * nb), th(nb);
    HY_CHECK(d2h(ctx, T.data(), dG.p, sizeof(double) * nb * nb));
    auto t0 = Clock::now();
    const bool ok = sd::sym_eig(nb, T.data(), th.data(), S.data());
    R.t_small += ms_since(t0);
    if (!ok) return set_err(ctx, HYEIG_ENUMERIC, "chebfsi: eigensolver of the projected matrix failed");
    HY_CHECK(h2d(ctx, dS.p, S.data(), sizeof(double) * nb * nb));
    HY_CHECK(launch_block_update_a(ctx, R.n, nb, nb, Qn.p, nb, dS.as<double>(), 1.0, 0.0, Q.p, nb, R.dt));
    HY_CHECK(launch_block_update_a(ctx, R.n, nb, nb, HQn.p, nb, dS.as<double>(), 1.0, 0.0, HQ.p, nb, R.dt));
    theta = th;
    return h2d(ctx, dth.p, theta.data(), sizeof(double) * nb);
  }

  // Q0 = CholeskyQR(X0) (twice), H Q0, Rayleigh-Ritz (the set-up of Algorithm 3)
  hyeig_status init(const float* X0, int64_t ldx) {
    HY_CHECK(launch_copy(R.ctx, R.n, nb, X0, ldx, HYEIG_F32, Qn.p, nb, R.dt));
    hyeig_status st = hyeig_cholqr(R.ctx, R.n, nb, Qn.p, nb, R.dt, 2, nullptr);
    if (st != HYEIG_OK) return st;
    HY_CHECK(R.spmm(nb, Qn.p, nb, HQn.p, nb));
    return rayleigh_ritz();
  }

  // relative residuals ||H q_j - theta_j q_j|| / scale of all nb columns
  hyeig_status norms() {
    std::vector<int> none(nb, -1);
    HY_CHECK(h2d(R.ctx, dpos.p, none.data(), sizeof(int) * nb));
    HY_CHECK(launch_resid_precond(R.ctx, R.n, nb, Q.p, nb, HQ.p, nb, dth.as<double>(), nullptr, 0.0, 0,
                                  dpos.as<int>(), F[0].p, nb, 0, R.dt, dnrm.as<double>()));
    std::vector<double> nr(nb);
    HY_CHECK(d2h(R.ctx, nr.data(), dnrm.p, sizeof(double) * nb));
    for (int j = 0; j < nb; ++j) {
      if (!std::isfinite(nr[j])) return set_err(R.ctx, HYEIG_ENUMERIC, "chebfsi: NaN/Inf residual");
      rel[j] = std::sqrt(nr[j]) / R.scale(theta[j]);
    }
    return HYEIG_OK;
  }

  hyeig_status step() {
    hyeig_ctx* ctx = R.ctx;
    const hyeig_params* p = R.p;
    ++it;
    std::vector<int> act, lck;
    for (int j = 0; j < nb; ++j) {
      if (p->lock && j < k && rel[j] <= p->tol)
        lck.push_back(j);
      else
        act.push_back(j);
    }
    const int na = (int)act.size(), nl = (int)lck.size();
    // the damped interval [lambda_F, lambda_ub] mapped to [-1, 1]
    const double lf = p->cheb_fixed_cutoff ? p->cheb_cutoff : theta[nb - 1];
    if (!(lub > lf)) return set_err(ctx, HYEIG_ENUMERIC, "chebfsi: lambda_ub not above the cutoff");
    const double e = 0.5 * (lub - lf), c = 0.5 * (lub + lf);
    HY_CHECK(h2d(ctx, didx.p, act.data(), sizeof(int) * na));
    HY_CHECK(launch_gather_cols(ctx, R.n, na, didx.as<int>(), Q.p, nb, F[0].p, na, R.dt));
    HY_CHECK(launch_gather_cols(ctx, R.n, na, didx.as<int>(), HQ.p, nb, HF.p, na, R.dt));
    // T_1: W = (H Q - c Q) / e
    HY_CHECK(launch_lincomb(ctx, R.n, na, 1.0 / e, HF.p, na, -c / e, F[0].p, na, 0.0, nullptr, 0, F[1].p, na, R.dt));
    int qp = 0, w = 1, y = 2;
    for (int j = 2; j <= degree; ++j) {
      // T_j = 2 (H - cI)/e T_{j-1} - T_{j-2}
      HY_CHECK(R.spmm(na, F[w].p, na, HF.p, na));
      HY_CHECK(launch_lincomb(ctx, R.n, na, 2.0 / e, HF.p, na, -2.0 * c / e, F[w].p, na, -1.0, F[qp].p, na, F[y].p,
                              na, R.dt));
      const int t = qp;
      qp = w;
      w = y;
      y = t;
    }
    DBuf& Wf = F[w];
    // the locked columns and their stored images first
    if (nl > 0) {
      HY_CHECK(h2d(ctx, didx.p, lck.data(), sizeof(int) * nl));
      HY_CHECK(launch_gather_cols(ctx, R.n, nl, didx.as<int>(), Q.p, nb, Qn.p, nb, R.dt));
      HY_CHECK(launch_gather_cols(ctx, R.n, nl, didx.as<int>(), HQ.p, nb, HQn.p, nb, R.dt));
      for (int pass = 0; pass < 2; ++pass) {
        HY_CHECK(launch_gram(ctx, R.n, nl, Qn.p, nb, na, Wf.p, na, R.dt, R.gmode, dG.as<double>()));
        HY_CHECK(launch_block_update_a(ctx, R.n, nl, na, Qn.p, nb, dG.as<double>(), -1.0, 1.0, Wf.p, na, R.dt));
      }
    }
    // unit columns, then CholeskyQR twice (the filter leaves columns of very
    // different lengths)
    HY_CHECK(launch_col_dots(ctx, R.n, na, Wf.p, na, Wf.p, na, R.dt, dnrm.as<double>()));
    std::vector<double> cn(na);
    HY_CHECK(d2h(ctx, cn.data(), dnrm.p, sizeof(double) * na));
    for (int j = 0; j < na; ++j) {
      if (!(cn[j] > 0.0) || !std::isfinite(cn[j])) return set_err(ctx, HYEIG_ENUMERIC, "chebfsi: filtered column vanished");
      cn[j] = 1.0 / std::sqrt(cn[j]);
    }
    HY_CHECK(h2d(ctx, dnrm.p, cn.data(), sizeof(double) * na));
    HY_CHECK(launch_col_scale(ctx, R.n, na, Wf.p, na, dnrm.as<double>(), R.dt));
    hyeig_status st = hyeig_cholqr(ctx, R.n, na, Wf.p, na, R.dt, 2, nullptr);
    if (st != HYEIG_OK) return set_err(ctx, HYEIG_ENUMERIC, "chebfsi: filtered block is rank deficient");
    HY_CHECK(launch_copy(ctx, R.n, na, Wf.p, na, R.dt, col(Qn, nl), nb, R.dt));
    // H times the new columns (the product that closes the iteration)
    HY_CHECK(R.spmm(na, col(Qn, nl), nb, col(HQn, nl), nb));
    return rayleigh_ritz();
  }
};

// Single-vector Lanczos (Section 2.1) with full re-orthogonalisation, FP64:
// `steps` products from x0 (column 0 of an FP32 block; the normalised ones
// vector when null); returns the extreme Ritz values of the tridiagonal matrix
// and their residual norms from the Lanczos relation (beta_m |last component|).
// stream of the pseudo-random vectors the library draws itself (the norm
// estimate's start, the columns added to a start block of a zero matrix)
constexpr uint64_t NORM_SEED = 0x5EED5EED5EED5EEDull;

hyeig_status lanczos_extremes(Run& R, const float* x0, int64_t ldx, int steps, double* th_min, double* th_max,
                              double* r_min, double* r_max) {
  hyeig_ctx* ctx = R.ctx;
  const int64_t n = R.n;
  const int nv = (int)std::min<int64_t>(std::min(steps, 31) + 1, n);
  DBuf V, w, dc;
  HY_CHECK(V.alloc(ctx, (size_t)n * 32 * sizeof(double)));
  HY_CHECK(w.alloc(ctx, (size_t)n * sizeof(double)));
  HY_CHECK(dc.alloc(ctx, sizeof(double) * 64));
  // the given start, or a pseudo-random one (a constant vector would miss
  // matrices that map it to zero or to a multiple of itself, such as a graph
  // Laplacian, and report a norm of zero for them)
  if (x0)
    HY_CHECK(launch_copy(ctx, n, 1, x0, ldx, HYEIG_F32, V.p, 32, HYEIG_F64));
  else
    HY_CHECK(launch_fill_hash(ctx, n, 1, V.p, 32, HYEIG_F64, NORM_SEED));
  HY_CHECK(launch_col_dots(ctx, n, 1, V.p, 32, V.p, 32, HYEIG_F64, dc.as<double>()));
  double nn;
  HY_CHECK(d2h(ctx, &nn, dc.p, sizeof(double)));
  if (!(nn > 0.0) || !std::isfinite(nn)) return set_err(ctx, HYEIG_ENUMERIC, "lanczos: zero or non-finite start");
  const double sc = 1.0 / std::sqrt(nn);
  HY_CHECK(h2d(ctx, dc.p, &sc, sizeof(double)));
  HY_CHECK(launch_col_scale(ctx, n, 1, V.p, 32, dc.as<double>(), HYEIG_F64));
  std::vector<double> al, be;
  hyeig_dtype save = R.dt, savev = R.vdt;
  R.dt = HYEIG_F64;
  R.vdt = HYEIG_F32;
  hyeig_status st = HYEIG_OK;
  double tsc = 0.0;  // largest |alpha| or beta so far: the scale of T
  for (int j = 0; j < nv - 1; ++j) {
    double* vj = V.as<double>() + j;
    if ((st = R.spmm(1, vj, 32, w.p, 1)) != HYEIG_OK) break;
    // full re-orthogonalisation against v_0..v_j (twice)
    for (int pass = 0; pass < 2 && st == HYEIG_OK; ++pass) {
      if ((st = launch_gram(ctx, n, j + 1, V.p, 32, 1, w.p, 1, HYEIG_F64, HYEIG_MMA_F64, dc.as<double>())) != HYEIG_OK)
        break;
      if (pass == 0) {
        double a;
        if ((st = d2h(ctx, &a, dc.as<double>() + j, sizeof(double))) != HYEIG_OK) break;
        al.push_back(a);
        tsc = std::max(tsc, std::fabs(a));
      }
      st = launch_block_update_a(ctx, n, j + 1, 1, V.p, 32, dc.as<double>(), -1.0, 1.0, w.p, 1, HYEIG_F64);
    }
    if (st != HYEIG_OK) break;
    if ((st = launch_col_dots(ctx, n, 1, w.p, 1, w.p, 1, HYEIG_F64, dc.as<double>())) != HYEIG_OK) break;
    double b2;
    if ((st = d2h(ctx, &b2, dc.p, sizeof(double))) != HYEIG_OK) break;
    double b = std::sqrt(std::max(b2, 0.0));
    // a remainder at the rounding level of T's entries: the Krylov space is
    // invariant (H = c I meets this at the first step).  Normalising that
    // remainder would give a vector that is not orthogonal to the basis.
    if (b <= 1e-13 * tsc) b = 0.0;
    tsc = std::max(tsc, b);
    be.push_back(b);
    if (b == 0.0 || j == nv - 2) break;
    double s = 1.0 / b;
    if ((st = h2d(ctx, dc.p, &s, sizeof(double))) != HYEIG_OK) break;
    if ((st = launch_col_scale(ctx, n, 1, w.p, 1, dc.as<double>(), HYEIG_F64)) != HYEIG_OK) break;
    if ((st = launch_copy(ctx, n, 1, w.p, 1, HYEIG_F64, V.as<double>() + j + 1, 32, HYEIG_F64)) != HYEIG_OK) break;
  }
  R.dt = save;
  R.vdt = savev;
  if (st != HYEIG_OK) return st;
  const int m = (int)al.size();
  std::vector<double> T((size_t)m * m, 0.0), wv(m), Q((size_t)m * m);
  for (int i = 0; i < m; ++i) {
    T[i + (size_t)i * m] = al[i];
    if (i + 1 < m) T[i + 1 + (size_t)i * m] = T[i + (size_t)(i + 1) * m] = be[i];
  }
  if (!sd::sym_eig(m, T.data(), wv.data(), Q.data())) return set_err(ctx, HYEIG_ENUMERIC, "lanczos: eigensolver failed");
  const double bl = be.empty() ? 0.0 : be.back();
  *th_min = wv[0];
  *th_max = wv[m - 1];
  if (r_min) *r_min = bl * std::fabs(Q[(m - 1) + (size_t)0 * m]);
  if (r_max) *r_max = bl * std::fabs(Q[(m - 1) + (size_t)(m - 1) * m]);
  return HYEIG_OK;
}

// ||H||_2 estimate: 30-step single-vector Lanczos from a pseudo-random vector;
// returns max |Ritz value| (a lower bound of ||H||_2, hence a conservative
// normaliser).  Zero only when H maps that vector to zero, i.e. (for any H met
// in practice) H = 0.
hyeig_status estimate_hnorm(Run& R, double* out) {
  double lo, hi;
  HY_CHECK(lanczos_extremes(R, nullptr, 0, 30, &lo, &hi, nullptr, nullptr));
  *out = std::max(std::fabs(lo), std::fabs(hi));
  return HYEIG_OK;
}

// explicit FP64 check of the returned pairs: theta, ||Hx - theta x|| / ||H||, / |theta|, ||X^T X - I||
hyeig_status final_check(Run& R, const void* X, int64_t ldx, hyeig_dtype xdt, int k, double* evals, double* resid) {
  hyeig_ctx* ctx = R.ctx;
  const int64_t n = R.n;
  DBuf X64, HX64, dd, dth;
  HY_CHECK(X64.alloc(ctx, (size_t)n * k * 8));
  HY_CHECK(HX64.alloc(ctx, (size_t)n * k * 8));
  HY_CHECK(dd.alloc(ctx, sizeof(double) * (3 * k + k * k)));
  HY_CHECK(dth.alloc(ctx, sizeof(double) * k));
  HY_CHECK(launch_copy(ctx, n, k, X, ldx, xdt, X64.p, k, HYEIG_F64));
  // FP64-accumulated product of the (stored) vectors
  R.clk.start(ctx);
  HY_CHECK(launch_spmm(ctx, R.H, k, X, ldx, xdt, HX64.p, k, HYEIG_F64, HYEIG_F32));
  // (another instance than the solve's own products: not counted with them)
  R.clk.stop(false, spmm_bytes(R.H, k, xdt, HYEIG_F64, HYEIG_F32));
  R.rep->spmm_count++;
  R.rep->spmv_count += k;
  R.rep->bytes_spmm += spmm_bytes(R.H, k, xdt, HYEIG_F64, HYEIG_F32);
  double* d = dd.as<double>();
  HY_CHECK(launch_col_dots(ctx, n, k, X64.p, k, X64.p, k, HYEIG_F64, d));
  HY_CHECK(launch_col_dots(ctx, n, k, X64.p, k, HX64.p, k, HYEIG_F64, d + k));
  std::vector<double> h(2 * k);
  HY_CHECK(d2h(ctx, h.data(), d, sizeof(double) * 2 * k));
  std::vector<double> th(k);
  for (int j = 0; j < k; ++j) th[j] = h[k + j] / h[j];
  HY_CHECK(h2d(ctx, dth.p, th.data(), sizeof(double) * k));
  std::vector<int> none(k, -1);
  DBuf dpos;
  HY_CHECK(dpos.alloc(ctx, sizeof(int) * k));
  HY_CHECK(h2d(ctx, dpos.p, none.data(), sizeof(int) * k));
  HY_CHECK(launch_resid_precond(ctx, n, k, X64.p, k, HX64.p, k, dth.as<double>(), nullptr, 0.0, 0, dpos.as<int>(),
                                HX64.p, k, 0, HYEIG_F64, d + 2 * k));
  std::vector<double> nr(k);
  HY_CHECK(d2h(ctx, nr.data(), d + 2 * k, sizeof(double) * k));
  HY_CHECK(launch_gram(ctx, n, k, X64.p, k, k, X64.p, k, HYEIG_F64, HYEIG_MMA_F64, d + 3 * k));
  std::vector<double> G(k * k);
  HY_CHECK(d2h(ctx, G.data(), d + 3 * k, sizeof(double) * k * k));
  double orth = 0.0, rtm = 0.0;
  for (int j = 0; j < k; ++j) {
    const double rn = std::sqrt(nr[j] / h[j]);
    evals[j] = th[j];
    // relative to ||H||_2; for H = 0 (norm 0) a residual is 0 or infinitely large
    resid[j] = R.hnorm > 0 ? rn / R.hnorm : (rn == 0.0 ? 0.0 : INFINITY);
    rtm = std::max(rtm, rn / std::max(std::fabs(th[j]), 1e-300));
    for (int i = 0; i < k; ++i) {
      double v = G[i + j * k] / std::sqrt(h[i] * h[j]) - (i == j ? 1.0 : 0.0);
      orth += v * v;
    }
  }
  R.rep->resid_theta_max = rtm;
  R.rep->orth_err = std::sqrt(orth);
  return HYEIG_OK;
}

// sort the first k pairs ascending (columns of X permuted accordingly)
hyeig_status sort_pairs(Run& R, float* X, int64_t ldx, int k, double* ev, double* rs) {
  std::vector<int> idx(k);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return ev[a] < ev[b]; });
  bool same = true;
  for (int j = 0; j < k; ++j) same = same && idx[j] == j;
  if (same) return HYEIG_OK;
  DBuf tmp;
  HY_CHECK(tmp.alloc(R.ctx, (size_t)R.n * k * 4));
  for (int j = 0; j < k; ++j)
    HY_CHECK(launch_copy(R.ctx, R.n, 1, X + idx[j], ldx, HYEIG_F32, tmp.as<float>() + j, k, HYEIG_F32));
  HY_CHECK(launch_copy(R.ctx, R.n, k, tmp.p, k, HYEIG_F32, X, ldx, HYEIG_F32));
  std::vector<double> e(ev, ev + k), r(rs, rs + k);
  for (int j = 0; j < k; ++j) {
    ev[j] = e[idx[j]];
    rs[j] = r[idx[j]];
  }
  HY_HIP(R.ctx, hipStreamSynchronize(R.ctx->stream));
  return HYEIG_OK;
}

}  // namespace

// ---- the RMM-DIIS state of the C-ABI ------------------------------------------
struct hyeig_rmm_state {
  Rmm* r = nullptr;
  hyeig_report rep{};
  ~hyeig_rmm_state() { delete r; }
};

extern "C" {

void hyeig_params_default(hyeig_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->k = 8;
  p->nb = 8;
  p->method = HYEIG_LOBPCG;
  p->tol = 1e-6;
  p->tol_norm = HYEIG_NORM_HNORM;
  p->hnorm = 0.0;
  p->maxiter = 1000;
  p->min_front = 3;
  p->switch_rule = HYEIG_SWITCH_TAU;
  p->switch_thr = 1e-7;
  p->s_max = 10;
  p->rmm_maxiter = 300;
  p->rmm_precond = 0;
  p->fallback = 1;
  p->precond = HYEIG_PRECOND_JACOBI;
  p->mlp = nullptr;
  p->jacobi_floor = 0.0;
  p->precision = HYEIG_PREC_F32;
  p->refresh_every = 20;
  p->seed = 0;
  p->lock = 1;
  p->basis = -1;
  p->maxiter_back = 0;
  p->nb_back = 0;
  p->rmm_decouple = 0;
  p->cheb_degree = 10;
  p->cheb_fixed_cutoff = 0;
  p->cheb_cutoff = 0.0;
  p->cheb_upper = 0.0;
}

hyeig_status hyeig_rmm_state_create(hyeig_ctx* ctx, const hyeig_mat* H, int64_t n, int k, int s_max, const float* d_X,
                                    int64_t ldx, const float* d_HX, int64_t ldhx, double tol, double hnorm,
                                    int precond, hyeig_rmm_state** out) {
  if (!ctx || !out) return HYEIG_EINVAL;
  *out = nullptr;
  if (!H || !d_X || n != H->n || k < 1 || k > 32 || s_max < 1 || s_max > RMM_SMAX || ldx < k ||
      (d_HX && ldhx < k))
    return set_err(ctx, HYEIG_EINVAL, "rmm_state_create: bad arguments (1 <= k <= 32, 1 <= s_max <= 20)");
  hyeig_rmm_state* s = new (std::nothrow) hyeig_rmm_state();
  if (!s) return HYEIG_ENOMEM;
  s->r = new (std::nothrow) Rmm();
  if (!s->r) {
    delete s;
    return HYEIG_ENOMEM;
  }
  Rmm& r = *s->r;
  r.ctx = ctx;
  r.H = H;
  r.n = n;
  r.k = k;
  r.smax = s_max;
  r.dt = HYEIG_F32;
  r.tol = tol;
  r.hnorm = hnorm > 0 ? hnorm : 1.0;
  r.theta_norm = hnorm <= 0;
  r.precond = precond;
  r.d = H->diag;
  r.floor_ = 1e-2 * r.hnorm;
  r.rep = &s->rep;
  hyeig_status st = r.alloc();
  if (st == HYEIG_OK) st = r.start(d_X, ldx, HYEIG_F32, d_HX, ldhx);
  if (st != HYEIG_OK) {
    delete s;
    return st;
  }
  *out = s;
  return HYEIG_OK;
}

hyeig_status hyeig_rmm_diis_step(hyeig_ctx* ctx, const hyeig_mat* H, hyeig_rmm_state* st) {
  if (!ctx || !H || !st || !st->r || st->r->H != H) return set_err(ctx, HYEIG_EINVAL, "rmm_diis_step: bad arguments");
  return st->r->sweep();
}

hyeig_status hyeig_rmm_state_get(hyeig_ctx* ctx, const hyeig_rmm_state* st, float* d_X, int64_t ldx, double* h_theta,
                                 double* h_resid, int* h_conv) {
  if (!ctx || !st || !st->r) return HYEIG_EINVAL;
  Rmm& r = *st->r;
  if (d_X) {
    if (ldx < r.k) return set_err(ctx, HYEIG_EINVAL, "rmm_state_get: ldx < k");
    HY_CHECK(launch_copy(ctx, r.n, r.k, r.X.p, r.k, r.dt, d_X, ldx, HYEIG_F32));
  }
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int j = 0; j < r.k; ++j) {
    if (h_theta) h_theta[j] = r.theta[j];
    if (h_resid) h_resid[j] = r.rel[j];
    if (h_conv) h_conv[j] = r.conv[j];
  }
  return HYEIG_OK;
}

void hyeig_rmm_state_destroy(hyeig_rmm_state* st) {
  if (!st) return;
  hipDeviceSynchronize();
  delete st;
}

hyeig_status hyeig_solve_lowest_k(hyeig_ctx* ctx, const hyeig_mat* H, const hyeig_params* p, float* d_X, int64_t ldx,
                                  double* h_evals, double* h_resid, hyeig_report* rep_in) {
  if (!ctx) return HYEIG_EINVAL;
  if (!H || !p || !d_X || !h_evals || !h_resid) return set_err(ctx, HYEIG_EINVAL, "solve: null argument");
  // block Lanczos alone may look for more pairs than its block has columns
  // (n_b = 1 is the single-vector Lanczos method); X then holds k columns
  const int kmax = p->method == HYEIG_BLANCZOS ? 32 : p->nb;
  if (p->k < 1 || p->nb < 1 || p->k > kmax || p->nb > 32 || ldx < std::max(p->nb, p->k) || p->tol <= 0 ||
      p->maxiter < 0 || H->n < 3 * std::max(p->nb, p->k))
    return set_err(ctx, HYEIG_EINVAL,
                   "solve: need 1 <= k <= nb <= 32 (k <= 32 for block Lanczos alone), ldx >= max(nb, k), tol > 0, "
                   "n >= 3 max(nb, k)");
  if (p->method < HYEIG_LOBPCG || p->method > HYEIG_CHEBFSI_RMMDIIS)
    return set_err(ctx, HYEIG_EINVAL, "solve: unknown method");
  const bool cheb_method = p->method == HYEIG_CHEBFSI || p->method == HYEIG_CHEBFSI_RMMDIIS;
  if (cheb_method && p->nb_back > p->nb)
    return set_err(ctx, HYEIG_EINVAL, "solve: after ChebFSI the LOBPCG block takes at most nb columns");
  if (cheb_method && (p->cheb_degree < 1 || p->cheb_degree > 200 || !(p->cheb_upper >= 0.0)))
    return set_err(ctx, HYEIG_EINVAL, "solve: ChebFSI needs 1 <= cheb_degree <= 200 and cheb_upper >= 0");
  if (p->nb_back > 0 && (p->nb_back < p->k || p->nb_back > 32 || H->n < 3 * p->nb_back))
    return set_err(ctx, HYEIG_EINVAL, "solve: need k <= nb_back <= 32 and n >= 3 nb_back");
  if (p->precond == HYEIG_PRECOND_MLP && !p->mlp) return set_err(ctx, HYEIG_EINVAL, "solve: MLP preconditioner without weights");
  if (p->precond == HYEIG_PRECOND_MLP && (!H->rowabs || !H->rownnz))
    return set_err(ctx, HYEIG_EINVAL, "solve: the MLP preconditioner needs a matrix prepared with HYEIG_MAT_ROWSTATS");
  const bool rmm_method = p->method == HYEIG_LOBPCG_RMMDIIS || p->method == HYEIG_BLANCZOS_RMMDIIS ||
                          p->method == HYEIG_CHEBFSI_RMMDIIS;
  if (rmm_method && (p->s_max < 1 || p->s_max > RMM_SMAX)) return set_err(ctx, HYEIG_EINVAL, "solve: 1 <= s_max <= 20");
  if (p->precision == HYEIG_PREC_BF16_SPMM && p->method != HYEIG_LOBPCG && p->method != HYEIG_LOBPCG_RMMDIIS)
    return set_err(ctx, HYEIG_EUNSUPPORTED, "solve: the BF16 form refines with FP32 values in LOBPCG only");
  if (p->precision == HYEIG_PREC_BF16_SPMM && !H->vals_bf16)
    return set_err(ctx, HYEIG_EINVAL, "solve: BF16 form needs a matrix created with HYEIG_MAT_BF16");
  hyeig_report local{};
  hyeig_report* rep = rep_in ? rep_in : &local;
  double* hist = rep->hist;
  double* hist_t = rep->hist_t;
  int hist_cap = rep->hist_cap;
  std::memset(rep, 0, sizeof(*rep));
  rep->hist = hist;
  rep->hist_t = hist_t;
  rep->hist_cap = hist_cap;
  auto t0 = Clock::now();
  HY_HIP(ctx, hipSetDevice(ctx->device));

  // internal tolerance with a margin for the FP32 rounding of the returned vectors;
  // the explicit FP64 check at the end decides
  hyeig_params pin = *p;
  pin.tol = 0.9 * p->tol;
  Run R{ctx, H, &pin, rep};
  R.n = H->n;
  R.dt = (p->precision == HYEIG_PREC_PLAIN_F64) ? HYEIG_F64 : HYEIG_F32;
  // Grams: FP64 matrix cores (exact products of FP32 data, FP64 sums) in both
  // the plain and the FP32 form; FP32 sums over long row chunks cap the
  // attainable residual near 1e-6 relative.
  R.gmode = HYEIG_MMA_F64;
  if (p->precision == HYEIG_PREC_BF16_SPMM) {
    R.vdt = HYEIG_BF16;
    R.gmode = HYEIG_MMA_SPLIT_BF16;
  }
  if (p->hnorm > 0)
    R.hnorm = p->hnorm;
  else
    HY_CHECK(estimate_hnorm(R, &R.hnorm));
  rep->hnorm_used = R.hnorm;
  const int k = p->k, nb = p->nb;
  hyeig_status st = HYEIG_OK;
  // H = 0 (no stored entries, or a norm estimate of zero): every vector is an
  // eigenvector with eigenvalue 0, and the iterations have nothing to work on
  // (a zero W, an invariant first Krylov block, an empty Chebyshev interval).
  // The start block, orthonormalised, is the result; columns past the start
  // block's nb come from the pseudo-random fill.  The final check decides.
  const bool zero = H->nnz == 0 || !(R.hnorm > 0);
  if (zero) {
    const int c = std::max(nb, k);
    if (c > nb) HY_CHECK(launch_fill_hash(ctx, R.n, c - nb, d_X + nb, ldx, HYEIG_F32, NORM_SEED));
    if (hyeig_cholqr(ctx, R.n, c, d_X, ldx, HYEIG_F32, 2, nullptr) != HYEIG_OK)
      return set_err(ctx, HYEIG_ENOTSPD, "solve: H = 0 and the start block is rank deficient");
  }
  const bool front_bl = p->method == HYEIG_BLANCZOS || p->method == HYEIG_BLANCZOS_RMMDIIS;
  const bool cheb = p->method == HYEIG_CHEBFSI || p->method == HYEIG_CHEBFSI_RMMDIIS;

  Switch sw{&pin};
  sw.enabled = rmm_method;
  bool switched = false, done = false;
  // LOBPCG block: n_b, or n_b_back when it takes over from a block Lanczos front end
  const int nbb = (front_bl || cheb) && p->nb_back > 0 ? p->nb_back : nb;
  Lobpcg lob(R, nbb, k);
  lob.d = H->diag;
  lob.floor_ = p->jacobi_floor > 0 ? p->jacobi_floor : 1e-2 * R.hnorm;
  DBuf hxk;  // H X of the hand-off (n x k)
  DBuf xk;
  // ---- BF16 front end: LOBPCG with BF16 values until 100x the tolerance, then FP32
  // values (the refinement sweeps of the precision form) ----
  int it_bf16 = -1;
  std::unique_ptr<ChebFsi> cfp;
  if (cheb && !zero) {
    // ---- Chebyshev-filtered subspace iteration (Algorithm 3) ----
    cfp.reset(new (std::nothrow) ChebFsi(R, nb, k, p->cheb_degree));
    if (!cfp) return HYEIG_ENOMEM;
    ChebFsi& cf = *cfp;
    HY_CHECK(cf.alloc());
    HY_CHECK(cf.init(d_X, ldx));
    if (p->cheb_upper > 0) {
      cf.lub = p->cheb_upper;
    } else {
      double lo, hi, rhi;
      HY_CHECK(lanczos_extremes(R, d_X, ldx, 10, &lo, &hi, nullptr, &rhi));
      cf.lub = hi + rhi;
    }
    st = HYEIG_ENOCONV;
    for (;;) {
      HY_CHECK(cf.norms());
      R.clk.collect();
      R.hist(cf.rel.data(), k);
      bool conv = true;
      for (int j = 0; j < k; ++j) conv = conv && cf.rel[j] <= pin.tol;
      if (conv) {
        st = HYEIG_OK;
        break;
      }
      if (sw.fire(cf.it, cf.theta.data(), cf.rel.data(), k)) {
        switched = true;
        st = HYEIG_OK;
        break;
      }
      if (cf.it >= p->maxiter) {
        // a hybrid hands over at the front end's limit (a fixed switch point)
        if (sw.enabled) {
          switched = true;
          st = HYEIG_OK;
        }
        break;
      }
      HY_CHECK(cf.step());
    }
    rep->iters_front = cf.it;
    if (!switched) HY_CHECK(launch_copy(ctx, R.n, nb, cf.Q.p, nb, R.dt, d_X, ldx, HYEIG_F32));
  }
  if (!front_bl && !cheb && !zero) {
    HY_CHECK(lob.alloc());
    st = lob.init(d_X, ldx);
    if (st != HYEIG_OK) return st;
    if (p->precision == HYEIG_PREC_BF16_SPMM) {
      hyeig_params q = pin;
      q.tol = std::min(1e-3, 100.0 * p->tol);
      R.p = &q;
      st = lob.run(p->maxiter, nullptr, nullptr);
      R.p = &pin;
      if (st != HYEIG_OK && st != HYEIG_ENOCONV) return st;
      R.vdt = HYEIG_F32;
      R.gmode = HYEIG_MMA_F64;
      it_bf16 = lob.it;
      HY_CHECK(lob.refresh());  // explicit H X with FP32 values
      lob.haveP = false;
      std::fill(lob.active.begin(), lob.active.end(), 1);
    }
    st = lob.run(p->maxiter, rmm_method ? &sw : nullptr, &switched);
    rep->iters_front = lob.it;
    if (it_bf16 >= 0) rep->iters_refine = lob.it - it_bf16;
    if (st != HYEIG_OK && st != HYEIG_ENOCONV) return st;
    if (!switched) {
      done = true;
      // eigenvectors back to the caller (all nb columns)
      HY_CHECK(launch_copy(ctx, R.n, nb, lob.col(lob.cur, false, 0), lob.lds, R.dt, d_X, ldx, HYEIG_F32));
    } else {
      if (R.dt == HYEIG_F32) {
        HY_CHECK(lob.refresh());  // explicit H X before the hand-off
      }
    }
  }
  DBuf blX, blHX;
  int ne = 0;  // columns of blX
  if (front_bl && !zero) {
    int cap = std::min(p->maxiter + 2, 4096 / nb);
    std::unique_ptr<BLanczos> bl(new (std::nothrow) BLanczos(R, nb, k, cap));
    if (!bl) return HYEIG_ENOMEM;
    HY_CHECK(bl->alloc());
    HY_CHECK(bl->start(d_X, ldx));
    st = HYEIG_ENOCONV;
    while (bl->it < p->maxiter && bl->it + 1 < cap) {
      if (bl->live[bl->it] == 0) break;  // Krylov space exhausted: T is final
      HY_CHECK(bl->step());
      R.clk.collect();
      const int kk = (int)bl->rel.size();
      std::vector<double> r(k, INFINITY);
      for (int j = 0; j < kk; ++j) r[j] = bl->rel[j];
      R.hist(r.data(), k);
      if (kk < k) continue;
      bool conv = true;
      for (int j = 0; j < k; ++j) conv = conv && bl->rel[j] <= pin.tol;
      if (conv) {
        st = HYEIG_OK;
        break;
      }
      // (a hand-over needs nbb Ritz vectors for a possible LOBPCG fallback)
      if (sw.fire(bl->it, bl->theta.data(), bl->rel.data(), k) && bl->real_dim() >= nbb) {
        switched = true;
        st = HYEIG_OK;
        break;
      }
    }
    rep->iters_front = bl->it;
    // a hybrid hands over at the front end's limit (a fixed switch point)
    if (st == HYEIG_ENOCONV && sw.enabled && (int)bl->rel.size() >= k && bl->real_dim() >= nbb) {
      switched = true;
      st = HYEIG_OK;
    }
    if ((int)bl->rel.size() < k) return set_err(ctx, HYEIG_ENOCONV, "blanczos: too few iterations for k pairs");
    // the k wanted Ritz pairs, and for a hand-over the next ones up to the
    // block of the LOBPCG that takes over if RMM-DIIS stagnates
    ne = switched ? std::min(nbb, bl->real_dim()) : k;
    HY_CHECK(blX.alloc(ctx, (size_t)R.n * ne * dsize(R.dt)));
    HY_CHECK(blHX.alloc(ctx, (size_t)R.n * ne * dsize(R.dt)));
    HY_CHECK(bl->extract(blX.p, ne, blHX.p, ne, ne));
    if (!switched) {
      done = true;
      HY_CHECK(launch_copy(ctx, R.n, k, blX.p, ne, R.dt, d_X, ldx, HYEIG_F32));
    }
  }
  rep->switched = switched;
  if (switched) {
    // ---- RMM-DIIS refinement of the leading k pairs ----
    Rmm rm;
    rm.ctx = ctx;
    rm.H = H;
    rm.n = R.n;
    rm.k = k;
    rm.smax = p->s_max;
    rm.dt = R.dt;
    rm.tol = pin.tol;
    rm.hnorm = R.hnorm;
    rm.theta_norm = p->tol_norm == HYEIG_NORM_THETA;
    rm.precond = p->rmm_precond;
    rm.decouple_after = p->rmm_decouple;
    rm.d = H->diag;
    rm.floor_ = lob.floor_ > 0 ? lob.floor_ : 1e-2 * R.hnorm;
    rm.clk = &R.clk;
    rm.rep = rep;
    HY_CHECK(rm.alloc());
    if (cheb)
      HY_CHECK(rm.start(cfp->Q.p, nb, R.dt, cfp->HQ.p, nb));
    else if (!front_bl)
      HY_CHECK(rm.start(lob.col(lob.cur, false, 0), lob.lds, R.dt, lob.col(lob.cur, true, 0), lob.lds));
    else
      HY_CHECK(rm.start(blX.p, ne, R.dt, blHX.p, ne));
    blHX.release();
    if (!front_bl || !p->fallback) blX.release();
    bool stag = false;
    while (!rm.all_converged(k) && rm.sweeps < p->rmm_maxiter) {
      HY_CHECK(rm.sweep());
      R.clk.collect();
      R.hist(rm.rel.data(), k);
      if (p->fallback && rm.stagnated(k)) {
        stag = true;
        rep->events_stagnation++;
        break;
      }
    }
    rep->iters_rmm = rm.sweeps;
    // converged columns that fell onto the same pairs count as a stagnation
    bool collapsed = false;
    if (rm.all_converged(k)) {
      HY_CHECK(rm.collapsed(&collapsed));
      if (collapsed) rep->events_stagnation++;
    }
    if (rm.all_converged(k) && !collapsed) {
      done = true;
      HY_CHECK(launch_copy(ctx, R.n, k, rm.X.p, k, R.dt, d_X, ldx, HYEIG_F32));
    } else if (p->fallback) {
      // resume LOBPCG from the refined vectors and the remaining front-end columns
      rep->fallback_used = 1;
      if (front_bl || cheb) {
        // block Lanczos or ChebFSI front end: LOBPCG (block nbb) from the
        // refined vectors and the next nbb - k Ritz vectors of the front end
        // (from the front end's own k leading ones when the refined columns
        // collapsed)
        HY_CHECK(lob.alloc());
        DBuf x0;
        HY_CHECK(x0.alloc(ctx, (size_t)R.n * nbb * sizeof(float)));
        const int k0 = collapsed ? 0 : k;
        if (!collapsed) HY_CHECK(launch_copy(ctx, R.n, k, rm.X.p, k, R.dt, x0.p, nbb, HYEIG_F32));
        if (cheb && nbb > k0)
          HY_CHECK(launch_copy(ctx, R.n, nbb - k0, cfp->col(cfp->Q, k0), nb, R.dt, (float*)x0.p + k0, nbb,
                               HYEIG_F32));
        if (!cheb && ne > k0)
          HY_CHECK(launch_copy(ctx, R.n, ne - k0, (const char*)blX.p + (size_t)k0 * dsize(R.dt), ne, R.dt,
                               (float*)x0.p + k0, nbb, HYEIG_F32));
        blX.release();
        cfp.reset();
        st = lob.init((const float*)x0.p, nbb);
        if (st != HYEIG_OK) return st;
        lob.it = 0;
      }
      // LOBPCG front end: resume from the state saved at the switch (X, W, P and
      // their images are untouched by RMM-DIIS, which works on its own copies),
      // with X merged with the refined vectors unless they collapsed
      if (!front_bl && !cheb && !collapsed) {
        bool merged = false;
        HY_CHECK(lob.merge_refined(rm.X.p, k, k, &merged));
        rep->merged_back = merged ? 1 : 0;
      }
      const int it0 = lob.it;
      st = lob.run(it0 + (p->maxiter_back > 0 ? p->maxiter_back : p->maxiter), nullptr, nullptr);
      lob.it -= it0;
      rep->iters_back = lob.it;
      if (st != HYEIG_OK && st != HYEIG_ENOCONV) return st;
      HY_CHECK(launch_copy(ctx, R.n, std::min(nb, nbb), lob.col(lob.cur, false, 0), lob.lds, R.dt, d_X, ldx,
                           HYEIG_F32));
      done = st == HYEIG_OK;
    } else {
      HY_CHECK(launch_copy(ctx, R.n, k, rm.X.p, k, R.dt, d_X, ldx, HYEIG_F32));
      st = HYEIG_ENOCONV;
    }
    (void)stag;
    if (collapsed && !p->fallback) set_err(ctx, HYEIG_ENOCONV, "rmm-diis: columns converged onto the same pairs");
  }
  (void)done;
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  auto tf = Clock::now();
  // ---- final FP64 check on the returned FP32 vectors ----
  HY_CHECK(final_check(R, d_X, ldx, HYEIG_F32, k, h_evals, h_resid));
  HY_CHECK(sort_pairs(R, d_X, ldx, k, h_evals, h_resid));
  R.clk.collect();
  rep->ms_final = ms_since(tf);
  rep->ms_total = ms_since(t0);
  rep->ms_spmm = R.clk.ms;
  rep->ms_spmm_mc = R.clk.ms_mc;
  rep->bytes_spmm_mc = R.clk.bytes_mc;
  rep->spmm_mc_count = R.clk.n_mc;
  rep->ms_small = R.t_small;
  rep->ms_dense = std::max(0.0, rep->ms_total - rep->ms_spmm - rep->ms_small);
  // the final FP64 check decides, in the normalisation the caller chose; the
  // returned vectors must also be orthonormal (small residuals alone do not
  // show that no wanted pair was missed)
  bool conv = true;
  if (p->tol_norm == HYEIG_NORM_THETA)
    conv = rep->resid_theta_max <= p->tol;
  else
    for (int j = 0; j < k; ++j) conv = conv && h_resid[j] <= p->tol;
  conv = conv && rep->orth_err <= 1e-4;
  rep->converged = conv;
  if (st == HYEIG_ENOCONV || !conv) return set_err(ctx, HYEIG_ENOCONV, "solve: tolerance not reached");
  return HYEIG_OK;
}

}  // extern "C"
