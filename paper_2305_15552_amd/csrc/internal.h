// Internal declarations shared by the HIP kernels and the host drivers of libhyeig.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hyeig.h"

// pinned ring for asynchronous host-to-device copies of small arrays
constexpr int H2D_SLOTS = 16;
constexpr size_t H2D_SLOT_BYTES = (size_t)64 << 10;

// workspace slots
enum {
  WS_REDUCE = 0,
  WS_GRAM = 1,
  WS_SMALL = 2,
  WS_TMP = 3,
  WS_TMP2 = 4,
  WS_MLP = 5,
  WS_MLP2 = 6,
  WS_MISC = 7,
  WS_BEST = 8,  // LOBPCG's kept iterate
  WS_COUNT = 9
};

struct hyeig_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int num_cu = 256;
  // device workspace slots (WS_*), grown on demand
  void* ws[WS_COUNT] = {nullptr};
  size_t ws_size[WS_COUNT] = {0};
  // pinned host staging
  void* pin = nullptr;
  size_t pin_size = 0;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  bool spmm_timed = false;
  // host-to-device ring: a slot is reused once the copy recorded on it has run
  char* h2d_ring = nullptr;
  hipEvent_t h2d_ev[H2D_SLOTS] = {};
  bool h2d_used[H2D_SLOTS] = {};
  int h2d_next = 0;
  // device address of this device's fixed scratch buffer (allocation-free calls)
  double* scratch = nullptr;
  // completion of small device-to-host reads, waited on by polling
  hipEvent_t d2h_ev = nullptr;
};

struct hyeig_mat {
  hyeig_ctx* ctx = nullptr;
  int64_t n = 0, nnz = 0, nbr = 0, ntiles = 0;
  int64_t* tile_ptr = nullptr;     // [nbr + 1] first tile of each block row
  int32_t* tile_col = nullptr;     // [ntiles] block column
  int64_t* tile_val = nullptr;     // [ntiles + 1] offset of the tile's packed values; [ntiles] = nvals
  uint32_t* tile_mask = nullptr;   // [ntiles][32] row bitmasks (bit c of word r: entry (r, c))
  uint32_t* tile_cmask = nullptr;  // [ntiles][32] column bitmasks (bit r of word c), diagonal excluded
  int64_t* col_ptr = nullptr;      // [nbr + 1] first entry of each block column in col_tiles
  int32_t* col_tiles = nullptr;    // [ntiles] tile ids ordered by block column, then block row
  int32_t* col_brow = nullptr;     // [ntiles] block row of each entry of col_tiles
  int64_t nvals = 0;               // length of vals: nnz plus alignment padding
  float* vals = nullptr;           // [nvals] packed row-major within each tile, tile starts 8-aligned
  uint16_t* vals_bf16 = nullptr;   // [nvals] BF16 copy or null
  float* tvals = nullptr;          // [nvals] the same values packed column-major within each tile
  uint16_t* tvals_bf16 = nullptr;  // [nvals] BF16 copy of tvals or null
  float* diag = nullptr;           // [n]
  float* rowabs = nullptr;         // [n] or null
  float* rownnz = nullptr;         // [n] or null
  double rownnz_mean = 1.0;        // mean of rownnz (with row statistics)
  // matrix-core operand slots of the stored values (built on the first
  // matrix-core product; see k_tile_pos): pos[v] for vals[v], tpos[v] for tvals[v]
  uint16_t* pos = nullptr;
  uint16_t* tpos = nullptr;
  bool pos_tried = false;
};

// zero values allocated past the last tile of each value array
constexpr int64_t VAL_PAD = 64;


hyeig_status set_err(hyeig_ctx* ctx, hyeig_status st, const std::string& msg);
hyeig_status hip_err(hyeig_ctx* ctx, hipError_t e, const char* what);
void* ws_get(hyeig_ctx* ctx, int slot, size_t bytes, hyeig_status* st);
void* pin_get(hyeig_ctx* ctx, size_t bytes, hyeig_status* st);
// host-to-device copy on the context's stream; h may be reused on return (small
// arrays through the pinned ring without waiting, larger ones synchronously)
hyeig_status h2d_queued(hyeig_ctx* ctx, void* d, const void* h, size_t bytes);

#define HY_HIP(ctx, call)                                   \
  do {                                                      \
    hipError_t e__ = (call);                                \
    if (e__ != hipSuccess) return hip_err((ctx), e__, #call); \
  } while (0)
#define HY_CHECK(expr)                 \
  do {                                 \
    hyeig_status s__ = (expr);         \
    if (s__ != HYEIG_OK) return s__;   \
  } while (0)

// ---- launchers (spmm.hip) ----
hyeig_status launch_tile_count(hyeig_ctx* ctx, int64_t n, int64_t nbr, const int64_t* rowptr, const int32_t* colidx,
                               int64_t* counts, int64_t* pvals);
hyeig_status launch_tile_fill(hyeig_ctx* ctx, hyeig_mat* M, const int64_t* rowptr, const int32_t* colidx,
                              const float* vals, const int64_t* vbase);
hyeig_status launch_validate(hyeig_ctx* ctx, int64_t n, const int64_t* rowptr, const int32_t* colidx, int* flag);
hyeig_status launch_rowstats(hyeig_ctx* ctx, int64_t n, const int64_t* rowptr, const int32_t* colidx,
                             const float* vals, float* rowabs, float* rownnz);
hyeig_status launch_to_bf16(hyeig_ctx* ctx, int64_t nnz, const float* src, uint16_t* dst);
hyeig_status launch_tile_tvals(hyeig_ctx* ctx, hyeig_mat* M);
// xfull: every row of X holds ldx >= the kernel width readable elements (an
// internal buffer), so x rows may be read in 16-byte pieces for any m
hyeig_status launch_spmm(hyeig_ctx* ctx, const hyeig_mat* H, int m, const void* X, int64_t ldx, hyeig_dtype xdt,
                         void* Y, int64_t ldy, hyeig_dtype acc, hyeig_dtype vdt, bool xfull = false);
// whether launch_spmm takes a matrix-core kernel for these arguments
bool spmm_on_matrix_cores(const hyeig_mat* H, int m, hyeig_dtype xdt, hyeig_dtype acc, hyeig_dtype vdt);

// ---- launchers (dense.hip) ----
// Y[i, j] = value for i < n, j < m (row-major, ld)
hyeig_status launch_fill(hyeig_ctx* ctx, int64_t n, int m, void* Y, int64_t ld, hyeig_dtype dt, double value);
// Y = pseudo-random values in [-1, 1), a fixed function of (i, j, seed)
hyeig_status launch_fill_hash(hyeig_ctx* ctx, int64_t n, int m, void* Y, int64_t ld, hyeig_dtype dt, uint64_t seed);
// G (ka x kb col-major FP64, device) = A^T B
// G = A^T [B1 B2] (column-major ka x (kb1 + kb2)): A is read once for both products
// bs > 0: A and B1 (= B2 = A for the fused pair) are three n x 16 blocks, bs
// elements apart, each with leading dimension lda (the solver's [X W P])
// fixed_part (nullable): device buffer of fixed_cap doubles for the per-workgroup
// partials instead of the context workspace (the workgroup count is cut to fit)
hyeig_status launch_gram2(hyeig_ctx* ctx, int64_t n, int ka, const void* A, int64_t lda, int kb1, const void* B1,
                          int64_t ldb1, int kb2, const void* B2, int64_t ldb2, hyeig_dtype dt, hyeig_mma_mode mode,
                          double* G, int64_t bs = 0, double* fixed_part = nullptr, int64_t fixed_cap = 0);
// the fixed device buffer of the allocation-free Gram: SCRATCH_DOUBLES FP64 per
// device, its address looked up once per device (scratch_init, at context creation)
constexpr int64_t SCRATCH_DOUBLES = (int64_t)1 << 19;  // 4 MiB
constexpr int HYEIG_MAX_DEVICES = 64;
hyeig_status scratch_init(hyeig_ctx* ctx);
hyeig_status launch_gram_noalloc(hyeig_ctx* ctx, int64_t n, int ka, const void* A, int64_t lda, int kb,
                                 const void* B, int64_t ldb, hyeig_dtype dt, hyeig_mma_mode mode, double* G);
hyeig_status launch_gram(hyeig_ctx* ctx, int64_t n, int ka, const void* A, int64_t lda, int kb, const void* B,
                         int64_t ldb, hyeig_dtype dt, hyeig_mma_mode mode, double* G);
// Y = S C + beta Y ; C col-major k x m FP64 (device)
hyeig_status launch_block_update(hyeig_ctx* ctx, int64_t n, int k, int m, const void* S, int64_t lds,
                                 const double* C, double beta, void* Y, int64_t ldy, hyeig_dtype dt);
// Y = S C with S block-strided when bs > 0 (k / 16 blocks of n x 16, bs elements
// apart).  Y may be columns of S itself: each row is read whole before it is written.
hyeig_status launch_block_update_bs(hyeig_ctx* ctx, int64_t n, int k, int m, const void* S, int64_t lds, int64_t bs,
                                    const double* C, void* Y, int64_t ldy, hyeig_dtype dt);
// Two outputs from one pass over S: Y1 = S C1, Y2 = S C2 (C's col-major k x m; Y2 may be null)
// bs > 0: S is k / 16 blocks of n x 16 (leading dimension lds = 16), bs elements apart
hyeig_status launch_block_update2(hyeig_ctx* ctx, int64_t n, int k, int m, const void* S, int64_t lds,
                                  const double* C1, void* Y1, int64_t ld1, const double* C2, void* Y2, int64_t ld2,
                                  hyeig_dtype dt, int64_t bs = 0);
// residual / preconditioner:
//   for a < na: src = cols[a]; r = HX[:, src] - theta[src] X[:, src]; W[:, a] = r / max(|d - theta|, floor)
//   (or W = r when d == null); norms2[src] = sum r^2 over all rows, for all src < nb (device FP64;
//   null: not formed).  guard (device int, nullable): when it holds zero the kernel writes nothing.
// The two LOBPCG updates [X1 P1] = S [C1 C2], [HX1 HP1] = HS [C1 C2] and the
// residual pass of launch_resid_precond on X1, HX1 (W, squared column norms
// into norms2), in one sweep; nb <= 16, k <= 48, and for FP32 16-byte aligned
// outputs with ldy % 4 == 0 (update_resid_fits).  The grid's per-block
// partials need at most num_cu * 8 * nb doubles of the WS_REDUCE workspace.
bool update_resid_fits(int64_t n, int k, int nb, int64_t ldy, const void* X1, const void* P1, const void* HX1,
                       const void* HP1, hyeig_dtype dt);
hyeig_status launch_update_resid(hyeig_ctx* ctx, int64_t n, int k, int nb, const void* S, const void* HS, int64_t lds,
                                 int64_t bss, const double* C1, const double* C2, void* X1, void* P1, void* HX1,
                                 void* HP1, int64_t ldy, const double* theta, const float* d, double floor,
                                 const int* pos, int na, void* W, int64_t ldw, hyeig_dtype dt, double* norms2);
hyeig_status launch_resid_precond(hyeig_ctx* ctx, int64_t n, int nb, const void* X, int64_t ldx, const void* HX,
                                  int64_t ldhx, const double* theta, const float* d, double floor, int na,
                                  const int* cols, void* W, int64_t ldw, int wcols_total, hyeig_dtype dt,
                                  double* norms2, const int* guard = nullptr);
// column scaling Y[:, j] *= s[j] (device FP64 s)
// Y = a A + b B + g C (C may be null), FP64 combination of FP32 or FP64 blocks
hyeig_status launch_lincomb(hyeig_ctx* ctx, int64_t n, int m, double a, const void* A, int64_t lda, double b,
                            const void* B, int64_t ldb, double g, const void* C, int64_t ldc, void* Y, int64_t ldy,
                            hyeig_dtype dt);
// Y[:, j] = X[:, idx[j]], j < m (idx on the device)
hyeig_status launch_gather_cols(hyeig_ctx* ctx, int64_t n, int m, const int* idx, const void* X, int64_t ldx,
                                void* Y, int64_t ldy, hyeig_dtype dt);
hyeig_status launch_col_scale(hyeig_ctx* ctx, int64_t n, int m, void* Y, int64_t ld, const double* s,
                              hyeig_dtype dt);
// dots[j] = sum_i A[i, j] * B[i, j], j < m (device FP64 out)
hyeig_status launch_col_dots(hyeig_ctx* ctx, int64_t n, int m, const void* A, int64_t lda, const void* B,
                             int64_t ldb, hyeig_dtype dt, double* dots);
// convert / copy a block between dtypes: Y[:, :m] = X[:, :m]
// Y (n x mp, contiguous) = X's first m columns, zero-padded to mp
hyeig_status launch_gather_pad(hyeig_ctx* ctx, int64_t n, int m, int mp, const void* X, int64_t ldx, void* Y,
                               hyeig_dtype dt);
hyeig_status launch_copy(hyeig_ctx* ctx, int64_t n, int m, const void* X, int64_t ldx, hyeig_dtype xdt, void* Y,
                         int64_t ldy, hyeig_dtype ydt);
// RMM-DIIS device kernels (FP32 data, FP64 coefficients); history window up to RMM_SMAX
#define RMM_SMAX 20
hyeig_status launch_rmm_combine(hyeig_ctx* ctx, hyeig_dtype dt, int64_t n, int k, const void* Xh, const void* Rh,
                                int w, const int* slots, const double* alpha, const double* thetah,
                                const int* active, void* Xt, void* HXt, double* dots2);
hyeig_status launch_rmm_scale(hyeig_ctx* ctx, hyeig_dtype dt, int64_t n, int k, const double* coef,
                              const int* active, void* Xt, void* HXt, void* Zt, const float* d, double floor);
hyeig_status launch_rmm_gram6(hyeig_ctx* ctx, hyeig_dtype dt, int64_t n, int k, const void* Xt, const void* Zt,
                              const void* HXt, const void* HZ, double* g6);
hyeig_status launch_rmm_update(hyeig_ctx* ctx, hyeig_dtype dt, int64_t n, int k, const double* g, const int* active,
                               const void* Xt, const void* Zt, const void* HXt, const void* HZ, void* X, void* HX,
                               void* R, void* Xh, void* Rh, int push, int w, const int* slots, double* dots);
// Y = alpha S C + beta Y
hyeig_status launch_block_update_a(hyeig_ctx* ctx, int64_t n, int k, int m, const void* S, int64_t lds,
                                   const double* C, double alpha, double beta, void* Y, int64_t ldy, hyeig_dtype dt);

// ---- learned preconditioner (mlp.hip) ----
// W[:, a] (holding residual column a on entry) <- MLP preconditioned residual.
// Column a of W is column j of the caller's ncol-column block with pos[j] = a
// (pos null: a = j and ncol = na); theta and nrm2 (squared residual norms) are
// device FP64 indexed by j; *d_bad is set on a non-finite output.
hyeig_status launch_mlp_precond(hyeig_ctx* ctx, const hyeig_mlp* mlp, const hyeig_mat* H, int64_t n, int na,
                                void* W, int64_t ldw, hyeig_dtype dt, const double* theta, const double* nrm2,
                                const int* pos, int ncol, double hnorm, int* d_bad);
// flags[1] += (flags[0] != 0); flags[0] = 0 (device ints)
hyeig_status launch_mlp_flag_count(hyeig_ctx* ctx, int* flags);
hyeig_status reduce_cols(hyeig_ctx* ctx, int nblk, int ncols, const double* part, double* out);

// ---- small dense FP64 (smalldense.cpp) ----
namespace sd {
// A (k x k col-major) symmetric: eigenvalues ascending in w, eigenvectors in V (col-major). returns false on failure
bool sym_eig(int k, const double* A, double* w, double* V);
// the `want` lowest eigenpairs of a symmetric band matrix (dense k x k col-major
// input, band width found from its nonzeros): w[want] ascending, V (k x want
// col-major); for the block tridiagonal matrices of block Lanczos
bool sym_band_eig_lowest(int k, const double* A, int want, double* w, double* V);
// R upper (col-major) with R^T R = G; returns false if not SPD
bool cholesky_upper(int k, const double* G, double* R);
// X <- R^{-1} (upper triangular inverse, col-major)
void tri_upper_inv(int k, const double* R, double* Rinv);
// generalized pencil (A, B): nwant leftmost; C (k x nwant col-major); condB
// optional (cond_2(B)); cond_bound optional, an upper bound on cond_2(B) from
// the Cholesky factor at O(k^2) cost
bool gen_eig(int k, const double* A, const double* B, int nwant, double* theta, double* C, double* condB,
             double* cond_bound = nullptr);
// cond_2 of a symmetric positive definite B (its extreme eigenvalues by bisection); inf if not positive
double spd_cond(int k, const double* B);
// DIIS constrained least squares on Gram Bm (s x s col-major) -> alpha[s]
void diis(int s, const double* Bm, double* alpha);
// 2x2 pencil smaller root: A = [a00 a01; a01 a11], B = [b00 b01; b01 b11]; g with g^T B g = 1
bool rr2(double a00, double a01, double a11, double b00, double b01, double b11, double* theta, double* g0,
         double* g1);
}  // namespace sd
