/*
 * hyeig: hybrid eigensolver hot path for one MI355X (gfx950) GPU.
 *
 * Computes a few algebraically smallest eigenpairs of a huge sparse symmetric
 * matrix H given by half: the upper triangle U including the diagonal, so that
 * H = U + U^T - diag(U).  The methods are those of arXiv 2305.15552 ("Hybrid
 * Eigensolvers for Nuclear Configuration Interaction Calculations"): LOBPCG
 * (Algorithm 2), block Lanczos (Algorithm 1), batched RMM-DIIS (Algorithm 4)
 * and the hybrids that switch from the block method to RMM-DIIS (Section 2.7,
 * switch metric eq. (switchtau)).
 *
 * Conventions for every call below.
 *   Pointers named d_* are HIP device pointers, h_* host pointers.  The caller
 *   owns every buffer it passes; the library owns its context workspace, the
 *   prepared matrix and RMM-DIIS states.
 *   Dense blocks ("tall-skinny" n x m) are row-major: element (i, j) at
 *   base[i * ld + j], ld >= m.  Small matrices (Gram matrices, coefficient
 *   matrices C) are column-major FP64: element (a, b) at base[a + b * rows].
 *   All device work is enqueued on the context's stream.  A call that writes
 *   host memory synchronises that stream before it returns; other calls are
 *   asynchronous.
 *   Errors are status codes; nothing throws or aborts across this interface.
 *   Arguments are checked before anything is enqueued.  The message of the
 *   last failure is kept in the context (hyeig_last_error).
 *   A context is not thread-safe; distinct contexts are.
 */
#ifndef HYEIG_H
#define HYEIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HYEIG_OK = 0,
  HYEIG_EINVAL = 1,        /* bad argument (null pointer, size, leading dimension, layout) */
  HYEIG_ENOMEM = 2,        /* device or host allocation failed */
  HYEIG_EDEVICE = 3,       /* a HIP call failed; message in hyeig_last_error */
  HYEIG_ENOTSPD = 4,       /* a Gram matrix is not positive definite (Cholesky failed) */
  HYEIG_ENOCONV = 5,       /* iteration limit reached; best results so far are returned */
  HYEIG_EUNSUPPORTED = 6,  /* valid but unsupported combination (dtype, width) */
  HYEIG_ENUMERIC = 7       /* NaN or Inf met */
} hyeig_status;

typedef enum { HYEIG_F64 = 0, HYEIG_F32 = 1, HYEIG_BF16 = 2 } hyeig_dtype;

/* How the dense Gram / update contractions are computed. */
typedef enum {
  HYEIG_MMA_F64 = 0,        /* FP64 matrix cores, FP64 data */
  HYEIG_MMA_F32 = 1,        /* FP32 matrix cores, FP32 data, FP32 partial sums reduced in FP64 */
  HYEIG_MMA_SPLIT_BF16 = 2  /* FP32 data split as hi + lo BF16 pairs on BF16 matrix cores */
} hyeig_mma_mode;

typedef struct hyeig_ctx hyeig_ctx;
typedef struct hyeig_mat hyeig_mat;
typedef struct hyeig_rmm_state hyeig_rmm_state;
typedef struct hyeig_mlp hyeig_mlp;

/* ---- context --------------------------------------------------------------
 * hyeig_ctx_create: binds HIP device `device` and the stream `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  The stream must outlive
 * the context. */
hyeig_status hyeig_ctx_create(int device, void* hip_stream, hyeig_ctx** out);
void hyeig_ctx_destroy(hyeig_ctx* ctx);
/* Message of the last failed call on ctx; valid until the next call on ctx. */
const char* hyeig_last_error(const hyeig_ctx* ctx);
/* Elapsed milliseconds of the most recent spmm_sym call's product kernel (the
 * clearing of Y excluded), measured with HIP events on the context stream
 * (synchronises the stream). */
hyeig_status hyeig_last_spmm_ms(hyeig_ctx* ctx, double* h_ms);

/* ---- matrix ---------------------------------------------------------------
 * The half-stored symmetric H of the paper (Section 3.1: the tables count the
 * non-zeros of half the symmetric matrix).  Input: upper-triangle CSR of an
 * n x n matrix, on the device: d_rowptr int64[n+1], d_colidx int32[nnz],
 * d_vals[nnz] in dtype vdt (HYEIG_F32).  Every stored column satisfies
 * row <= col < n; columns ascend within a row.  The call builds the prepared
 * form used by every product (32 x 32 tiles: a row bitmask and a column bitmask
 * per tile, values packed row-major inside the tile), extracts the diagonal
 * and, with HYEIG_MAT_ROWSTATS, the full-row 1-norms and full-row counts of H.
 * The CSR buffers are only read during the call.
 * flags: HYEIG_MAT_VALIDATE checks the layout on the device first (EINVAL if
 * violated); HYEIG_MAT_BF16 also keeps a BF16 copy of the values (round to
 * nearest even) for products with BF16 values. */
#define HYEIG_MAT_VALIDATE 1u
#define HYEIG_MAT_BF16 2u
#define HYEIG_MAT_ROWSTATS 4u
hyeig_status hyeig_mat_create(hyeig_ctx* ctx, int64_t n, int64_t nnz, const int64_t* d_rowptr,
                              const int32_t* d_colidx, const void* d_vals, hyeig_dtype vdt, uint32_t flags,
                              hyeig_mat** out);
void hyeig_mat_destroy(hyeig_mat* mat);

typedef struct {
  int64_t n, nnz, ntiles, nblockrows;
  int64_t prepared_bytes;   /* bytes of the prepared form (both value copies, BF16 ones included) */
  const float* d_diag;      /* device: diagonal of H (n floats), owned by the matrix */
  const float* d_rowabs;    /* device: full-row 1-norms sum_j |H_kj| (n floats) or NULL */
  const float* d_rownnz;    /* device: full-row stored counts (n floats) or NULL */
} hyeig_mat_info;
hyeig_status hyeig_mat_get_info(const hyeig_mat* mat, hyeig_mat_info* info);

/* ---- products -------------------------------------------------------------
 * hyeig_spmm_sym: Y = H X with H = U + U^T - diag(U), both halves applied by
 * one kernel launch (the block product every method of Section 2 is built on;
 * LOBPCG needs only H W per iteration, eq. (upd1)-(upd2)).  The workgroup of
 * block row J forms y_J whole from the tiles of block row J and of block
 * column J, so every stored tile is read twice per product (once by its row
 * owner, once by its column owner) and Y is written once.  X is n x m
 * (leading dimension ldx) of dtype xdt, Y is n x m (ldy) of dtype ydt,
 * 1 <= m <= 32.  acc is the accumulation type.  Supported (xdt, ydt, acc):
 * (F32, F32, F32), (F64, F64, F64), (F32, F64, F64).  vdt selects the stored
 * values: HYEIG_F32, or HYEIG_BF16 (matrix created with HYEIG_MAT_BF16, FP32
 * accumulation only).  X and Y must not overlap.  Y is overwritten.
 * With F32 values and 9 <= m <= 16, (F32, F32, F32) runs on FP32 matrix cores
 * and (F64, F64, F64) and (F32, F64, F64) on FP64 matrix cores (each 32 x 32
 * tile as a dense product, absent entries exact zeros); other widths and forms
 * walk the tiles on vector units.  Both sum within the same error bound, in
 * different orders, so one column of a product at such a width may differ in
 * its last bits from the same column computed alone. */
hyeig_status hyeig_spmm_sym(hyeig_ctx* ctx, const hyeig_mat* H, int m, const void* d_X, int64_t ldx,
                            hyeig_dtype xdt, void* d_Y, int64_t ldy, hyeig_dtype ydt, hyeig_dtype acc,
                            hyeig_dtype vdt);

/* hyeig_gram: G = A^T B for tall-skinny A (n x ka, lda) and B (n x kb, ldb), both
 * of dtype dt, into d_G (device, ka x kb column-major FP64).  The projected
 * matrices S^T H S and S^T S of the Rayleigh-Ritz step (eq. (rreig)) and the
 * block Gram-Schmidt coefficients V^T W (eq. (bgs)).  1 <= ka, kb <= 64.
 * mode: HYEIG_MMA_F64 (F64 or F32 data; FP32 inputs are widened exactly, so the
 * products are exact and the sums FP64); HYEIG_MMA_F32 and HYEIG_MMA_SPLIT_BF16
 * need dt = F32. */
hyeig_status hyeig_gram(hyeig_ctx* ctx, int64_t n, int ka, const void* d_A, int64_t lda, int kb,
                        const void* d_B, int64_t ldb, hyeig_dtype dt, hyeig_mma_mode mode, double* d_G);

/* hyeig_gram_noalloc: hyeig_gram for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and error codes as hyeig_gram; it calls
 * no hipMalloc, hipFree or other allocating routine and records no memset.
 * The per-workgroup FP64 partial sums go to a fixed 4 MiB device buffer that
 * the library holds once per device until the process ends (its address is
 * looked up when a context is created on that device); the number of
 * workgroups is cut so that their partials fit it.  Limit: the rows one wave
 * walks times max(lda, ldb) times the element size must stay below 2^31 bytes,
 * else HYEIG_EUNSUPPORTED (n * max(lda, ldb) * size below about 2^38 bytes).
 * Every call on one device shares that buffer: calls that overlap on one
 * device (two streams, two host threads) race and must be serialised by the
 * caller. */
hyeig_status hyeig_gram_noalloc(hyeig_ctx* ctx, int64_t n, int ka, const void* d_A, int64_t lda, int kb,
                                const void* d_B, int64_t ldb, hyeig_dtype dt, hyeig_mma_mode mode, double* d_G);

/* hyeig_block_update: Y = S C + beta Y with S n x k (lds), C k x m column-major
 * FP64 on the device, Y n x m (ldy); S and Y of dtype dt (F32 or F64).  The
 * block updates of eq. (xupd), (pupd), (upd1), (upd2) and the projection of
 * eq. (bgs).  1 <= k <= 64, 1 <= m <= 32.  Y must not overlap S unless
 * d_Y == d_S, ldy == lds, m == k and beta == 0 (in-place right multiplication).
 * The products are formed on matrix cores in the data type (FP64 MFMA for F64,
 * FP32 MFMA for F32; these updates are bandwidth bound); mode is accepted for
 * interface symmetry and ignored. */
hyeig_status hyeig_block_update(hyeig_ctx* ctx, int64_t n, int k, int m, const void* d_S, int64_t lds,
                                const double* d_C, double beta, void* d_Y, int64_t ldy, hyeig_dtype dt,
                                hyeig_mma_mode mode);

/* hyeig_cholqr: CholeskyQR (Algorithm 3, on the start block and each filtered block): G = X^T X in FP64,
 * G = R^T R (FP64 Cholesky on the host), X <- X R^{-1} in place.  passes = 2
 * repeats it (CholQR2); R is then the product of both factors.  d_R (device,
 * m x m column-major upper triangular FP64) may be NULL.  ENOTSPD if a
 * Cholesky factorisation fails (X is left unchanged by that pass). */
hyeig_status hyeig_cholqr(hyeig_ctx* ctx, int64_t n, int m, void* d_X, int64_t ldx, hyeig_dtype dt,
                          int passes, double* d_R);

/* hyeig_rayleigh_ritz: the nwant leftmost eigenpairs of the pencil (A, B),
 * A C = B C diag(theta), C^T B C = I (eq. (rreig); B = NULL means B = I as in
 * eq. (trideig) and (btrideig)).  A, B: k x k column-major FP64, symmetric
 * (only symmetrised parts are used); k <= 4096.  theta: nwant values ascending;
 * C: k x nwant column-major.  condB (nullable): condition number of B.
 * on_device = 0: all pointers are host pointers; 1: all are device pointers.
 * FP64 throughout (computed on the host).  ENOTSPD if B is not positive definite. */
hyeig_status hyeig_rayleigh_ritz(hyeig_ctx* ctx, int k, const double* A, const double* B, int nwant,
                                 double* theta, double* C, double* condB, int on_device);

/* ---- RMM-DIIS (Algorithm 4, batched over columns as in Section 4.2) --------
 * A state holds, per column j, x_j, H x_j, theta_j, r_j and a ring of the last
 * s_max pairs (x^(l), r^(l)).  hyeig_rmm_state_create copies X (n x k, ldx,
 * FP32) and H X (nullable: then one product computes it), normalises each
 * column (the set-up of Algorithm 4) and forms theta and r.
 * hyeig_rmm_diis_step performs one sweep for all unconverged columns: DIIS
 * coefficients (eq. (xsum)-(rmm), FP64 on the host), x~ and H x~ by linearity,
 * r~ = H x~ - theta~ x~, optional preconditioning, ONE product H [r~_1..r~_k],
 * the 2x2 Rayleigh-Ritz of eq. (rr)-(xuwg) and the new residual.  Converged
 * columns stay in the product but are frozen (the coupled variant of Section
 * 4.2).  tol is the relative residual tolerance (scale hnorm, or |theta| when
 * hnorm <= 0).  precond: 0 none, 1 shifted Jacobi. */
hyeig_status hyeig_rmm_state_create(hyeig_ctx* ctx, const hyeig_mat* H, int64_t n, int k, int s_max,
                                    const float* d_X, int64_t ldx, const float* d_HX, int64_t ldhx,
                                    double tol, double hnorm, int precond, hyeig_rmm_state** out);
hyeig_status hyeig_rmm_diis_step(hyeig_ctx* ctx, const hyeig_mat* H, hyeig_rmm_state* st);
/* Copies out X (n x k, ldx, FP32, device), and on the host theta[k], the
 * relative residuals resid[k] and converged flags conv[k] (any may be NULL). */
hyeig_status hyeig_rmm_state_get(hyeig_ctx* ctx, const hyeig_rmm_state* st, float* d_X, int64_t ldx,
                                 double* h_theta, double* h_resid, int* h_conv);
void hyeig_rmm_state_destroy(hyeig_rmm_state* st);

/* ---- the solver -----------------------------------------------------------*/
typedef enum {
  HYEIG_LOBPCG = 0,            /* Algorithm 2 */
  HYEIG_BLANCZOS = 1,          /* Algorithm 1 */
  HYEIG_LOBPCG_RMMDIIS = 2,    /* Section 2.7 hybrid, LOBPCG front end */
  HYEIG_BLANCZOS_RMMDIIS = 3,  /* Section 2.7 hybrid, block Lanczos front end */
  HYEIG_CHEBFSI = 4,           /* Algorithm 3, Chebyshev-filtered subspace iteration */
  HYEIG_CHEBFSI_RMMDIIS = 5    /* Section 2.7 hybrid, ChebFSI front end */
} hyeig_method;
typedef enum { HYEIG_SWITCH_TAU = 0, HYEIG_SWITCH_RESID = 1, HYEIG_SWITCH_ITERS = 2 } hyeig_switch_rule;
typedef enum { HYEIG_PRECOND_NONE = 0, HYEIG_PRECOND_JACOBI = 1, HYEIG_PRECOND_MLP = 2 } hyeig_precond_kind;
typedef enum {
  HYEIG_PREC_PLAIN_F64 = 0,    /* FP64 blocks, FP64 accumulation, FP32 stored values */
  HYEIG_PREC_F32 = 1,          /* FP32 blocks and accumulation, FP64 small problems and final check */
  HYEIG_PREC_BF16_SPMM = 2     /* as F32 but BF16 stored values in the front end, FP32 refinement
                                   (LOBPCG and the LOBPCG hybrid only) */
} hyeig_precision;
typedef enum { HYEIG_NORM_HNORM = 0, HYEIG_NORM_THETA = 1 } hyeig_tol_norm;

typedef struct {
  int k;                        /* n_ev: wanted eigenpairs */
  int nb;                       /* block size n_b >= k (<= 32); block Lanczos alone accepts n_b < k
                                   (n_b = 1: the single-vector Lanczos method of Section 2.1) */
  hyeig_method method;
  double tol;                   /* relative residual tolerance (default 1e-6) */
  hyeig_tol_norm tol_norm;      /* scale: ||H||_2 (default) or |theta| (the paper's form) */
  double hnorm;                 /* ||H||_2; <= 0: estimated by a 30-step Lanczos run from a
                                   pseudo-random start vector */
  int maxiter;                  /* front-end iteration limit; in a hybrid, reaching it hands over to
                                   RMM-DIIS (a fixed switch point) instead of ending the solve.  With a
                                   block Lanczos front end it also sizes the stored basis:
                                   (maxiter + 2) n_b columns of n elements */
  int min_front;                /* tau switch: least front-end iterations (default 3) */
  hyeig_switch_rule switch_rule;
  double switch_thr;            /* tau threshold, residual threshold, or iteration count */
  int s_max;                    /* DIIS window (default 10) */
  int rmm_maxiter;              /* RMM-DIIS sweep limit */
  int rmm_precond;              /* 0: unpreconditioned r~ (as printed), 1: shifted Jacobi */
  int fallback;                 /* 1: on RMM-DIIS stagnation resume LOBPCG (default 1); after a LOBPCG
                                   front end it resumes from its state at the switch with X replaced by
                                   the nb lowest Ritz vectors of span[X, RMM-DIIS's refined vectors]
                                   (unless those collapsed onto the same pairs) */
  hyeig_precond_kind precond;   /* LOBPCG preconditioner K */
  const hyeig_mlp* mlp;         /* for HYEIG_PRECOND_MLP */
  double jacobi_floor;          /* floor of |d_k - theta_j|; <= 0: 1e-2 * hnorm */
  hyeig_precision precision;
  int refresh_every;            /* explicit H X refresh period in FP32 forms (default 20) */
  uint64_t seed;                /* unused unless x0 is generated by the caller */
  int lock;                     /* soft locking of converged columns (default 1) */
  int basis;                    /* LOBPCG basis: 0 = as printed (P from eq. (pupd), P dropped when
                                   cond(S^T S) > 1e12); 1 = W orthogonalised against X and
                                   orthonormalised, P made orthonormal and orthogonal to X in the
                                   projected metric (same subspace); -1 = 1 for FP32 forms, 0 for
                                   the plain FP64 form (default) */
  int maxiter_back;             /* LOBPCG iteration limit after an RMM-DIIS stagnation; <= 0: maxiter */
  int nb_back;                  /* block size (k..32) of the LOBPCG that takes over from a block Lanczos
                                   or ChebFSI front end when RMM-DIIS stagnates (k refined vectors and
                                   the next Ritz vectors of the front end; block Lanczos hands over once
                                   it has that many, ChebFSI needs nb_back <= nb); <= 0: nb */
  int rmm_decouple;             /* RMM-DIIS products (Section 4.2): 0 = coupled, one product over all k
                                   columns every sweep with converged columns frozen (default); c > 0 =
                                   decoupled once c columns have converged, one SpMV per unconverged
                                   column */
  int cheb_degree;              /* ChebFSI: degree d of the filter (Alg. 3; default 10) */
  int cheb_fixed_cutoff;        /* ChebFSI: 1 = lambda_F is cheb_cutoff (the paper's 0 for bound states);
                                   0 = the largest Ritz value of the block after each Rayleigh-Ritz step
                                   (default; it needs nb > k: with nb = k that value is a wanted one and
                                   the filter cannot separate the k-th eigenvalue from the next) */
  double cheb_cutoff;
  double cheb_upper;            /* ChebFSI: lambda_ub; <= 0: theta + ||r|| of the largest Ritz pair after 10
                                   Lanczos steps from the first column of X0 (Section 3) */
} hyeig_params;
void hyeig_params_default(hyeig_params* p);

typedef struct {
  int iters_front, iters_rmm, iters_back;
  int spmm_count;               /* products H @ block */
  int64_t spmv_count;           /* vectors multiplied by H (the paper's SpMV count) */
  int switched, converged, fallback_used;
  int events_drop_p, events_orth_w, events_stagnation, events_mlp_fallback, refreshes;
  int events_deflation;         /* block Lanczos steps whose new block had numerically dependent
                                   columns (an exhausted Krylov direction), kept as zero columns */
  int merged_back;              /* 1: the LOBPCG after an RMM-DIIS hand-back resumed with X replaced by
                                   the lowest Ritz vectors of span[X, refined vectors] */
  double hnorm_used;
  double max_cond;              /* largest condition number of S^T S seen (Section 4.2) */
  double ms_total;
  double ms_spmm;               /* kernel time of the products (HIP events around each product kernel) */
  double ms_dense, ms_small, ms_final;
  double resid_theta_max;       /* final max ||Hx - theta x|| / |theta| */
  double orth_err;              /* final ||X^T X - I||_F */
  double bytes_spmm;            /* algorithmic bytes of all products: per product
                                   nnz (s_v + 4) + 8 (n + 1) + n m (s_x + s_y) */
  /* optional per-iteration history: caller sets hist/hist_cap (host, doubles);
   * row it holds the k relative residuals of iteration it */
  double* hist;
  int hist_cap;
  int hist_len;
  /* optional (NULL or hist_cap x 4 doubles, host): for each history row, the
     milliseconds since the solve started, the product-kernel milliseconds so
     far, the host small-problem milliseconds so far (the split of each
     iteration between products, small problems and the rest), and the
     condition number of S^T S in the last LOBPCG Rayleigh-Ritz step (0 before
     the first; Section 4.2 follows its growth) */
  double* hist_t;
  int iters_refine;             /* BF16 form: front-end iterations with FP32 values after the BF16 phase
                                   (the refinement sweeps; included in iters_front) */
  int spmm_mc_count;            /* the solve's products that ran on a matrix-core kernel (widths 9-16, FP32
                                   or FP64 values and sums; the final check's product is not counted) */
  double ms_spmm_mc;            /* their kernel time (HIP events) */
  double bytes_spmm_mc;         /* their algorithmic bytes */
} hyeig_report;

/* hyeig_solve_lowest_k: the k lowest eigenpairs of H (problem statement of
 * Section 2: H X = X Lambda; inputs and outputs of Algorithms 1, 2, 4).
 * d_X: n x max(nb, k) (ldx >= max(nb, k)) FP32 on the device; on entry the start
 * block X0 in its first nb columns, on exit the eigenvector approximations in
 * its first k columns.  h_evals[k]:
 * eigenvalues ascending; h_resid[k]: final relative residuals
 * ||H x - theta x|| / ||H||_2 from an explicit FP64-accumulated product.
 * rep may be NULL.  EINVAL unless 1 <= k <= nb <= 32 (block Lanczos alone:
 * k <= 32), tol > 0 and n >= 3 max(nb, k) (the LOBPCG basis [X W P] needs 3 nb
 * independent columns).  ENOCONV with best results filled when the limits are hit;
 * a LOBPCG phase that ends unconverged (its limit, or a breakdown after its
 * worst wanted residual fell below 1e-4 or 100 times the tolerance) returns the
 * iterate with the lowest such residual (kept when it halves), not its last one.  H = 0 (no stored entries, or a
 * norm estimate of zero): every vector is an eigenvector, so the start block
 * is returned orthonormalised (columns past nb filled pseudo-randomly) with
 * eigenvalues 0; for ||H||_2 = 0 a residual reads 0 when H x - theta x = 0
 * exactly, infinity otherwise.  ENOTSPD if that start block is rank deficient.
 * Block Lanczos keeps the numerically dependent columns of a new block (an
 * exhausted Krylov space) as zero columns decoupled from T, and stops once a
 * block has none left: T then holds the exact pairs of an invariant subspace. */
hyeig_status hyeig_solve_lowest_k(hyeig_ctx* ctx, const hyeig_mat* H, const hyeig_params* p, float* d_X,
                                  int64_t ldx, double* h_evals, double* h_resid, hyeig_report* rep);

/* ---- learned preconditioner (per-row MLP: 4 -> 64 -> 1, ReLU) -------------
 * Weights in FP32 master copies with BF16 copies used by the kernels.
 * Layout of the 385 parameters: W1[64][4], b1[64], w2[64], b2. */
#define HYEIG_MLP_HIDDEN 64
#define HYEIG_MLP_FEATURES 4
#define HYEIG_MLP_NPARAM (HYEIG_MLP_HIDDEN * HYEIG_MLP_FEATURES + 2 * HYEIG_MLP_HIDDEN + 1)
hyeig_status hyeig_mlp_create(hyeig_ctx* ctx, const float* h_params, hyeig_mlp** out);
hyeig_status hyeig_mlp_get(hyeig_ctx* ctx, const hyeig_mlp* mlp, float* h_params);
void hyeig_mlp_destroy(hyeig_mlp* mlp);
/* out[i] = MLP(feat[i, 0:4]) for N samples (feat row-major N x 4, device). */
hyeig_status hyeig_mlp_forward(hyeig_ctx* ctx, const hyeig_mlp* mlp, int64_t N, const float* d_feat,
                               float* d_out);
/* Mean-squared-error loss L = mean((MLP(f_i) - t_i)^2) and its gradient with
 * respect to the 385 parameters (d_grad, device FP32, same layout). */
hyeig_status hyeig_mlp_backward(hyeig_ctx* ctx, const hyeig_mlp* mlp, int64_t N, const float* d_feat,
                                const float* d_target, float* d_grad, double* h_loss);
/* hyeig_mlp_precond: W = K^{-1} R with the learned K, the preconditioned
 * residual block of eq. (wblock) (the paper leaves K open; this learned K is a
 * project addition).  d_W (n x k, ldw, FP32 or FP64, device) holds R on entry
 * and W on exit; h_theta[k] (host) are the columns' Ritz values.  Entry (i, j):
 * features f = ((d_i - theta_j) / hnorm, r_ij sqrt(n) / ||r_j||, rowabs_i /
 * hnorm, rownnz_i / mean rownnz) from the matrix's diagonal and row statistics
 * (HYEIG_MAT_ROWSTATS, else EINVAL), then w_ij = MLP(f) ||r_j|| / (hnorm
 * sqrt(n)), 1 <= k <= 32.  Features and the rescale in FP32 (d_i - theta_j kept
 * accurate where the two are close), BF16 weights, features and hidden
 * activations with FP32 sums, ||r_j|| summed in FP64 on the device.  ENUMERIC
 * if an output is not finite.  Synchronises the stream. */
hyeig_status hyeig_mlp_precond(hyeig_ctx* ctx, const hyeig_mlp* mlp, const hyeig_mat* H, int k, void* d_W,
                               int64_t ldw, hyeig_dtype dt, const double* h_theta, double hnorm);
typedef struct {
  int epochs;
  int64_t batch;
  double lr, beta1, beta2, eps;
  uint64_t seed;                /* shuffling */
} hyeig_train_params;
/* Adam on FP32 master weights; h_loss_per_epoch (nullable) gets `epochs` values. */
hyeig_status hyeig_mlp_train(hyeig_ctx* ctx, hyeig_mlp* mlp, int64_t N, const float* d_feat,
                             const float* d_target, const hyeig_train_params* tp, double* h_loss_per_epoch);

/* Training samples from the correction equation: the k columns of d_X (n x k,
 * row-major, FP32 or FP64, device) are orthonormalised (CholeskyQR2) into a
 * Ritz block X with Ritz values theta_j = x_j^T H x_j and residuals r_j; the
 * target of entry (row, j) is t_{row j} ||H|| sqrt(n) / ||r_j|| with t_j from
 * `steps` MINRES iterations on (I - X X^T)(H - theta_j)(I - X X^T) t = -r_j.
 * Writes d_feat (n k x 4, FP32, 16-byte aligned, sample row * k + j),
 * d_target (n k, FP32) and h_theta (k, nullable).  1 <= k <= 32.  The matrix
 * must carry row statistics (HYEIG_MAT_ROWSTATS), else EINVAL.  Workspace is
 * allocated and freed inside the call. */
hyeig_status hyeig_mlp_labels(hyeig_ctx* ctx, const hyeig_mat* H, int k, const void* d_X, int64_t ldx,
                              hyeig_dtype dt, double hnorm, int steps, float* d_feat, float* d_target,
                              double* h_theta);

#ifdef __cplusplus
}
#endif
#endif /* HYEIG_H */
