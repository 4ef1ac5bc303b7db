// C-ABI of libhyeig: context, matrix, products and small problems.
#include <cstdlib>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

hyeig_status set_err(hyeig_ctx* ctx, hyeig_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

hyeig_status hip_err(hyeig_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return HYEIG_OK;
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory) return set_err(ctx, HYEIG_ENOMEM, m);
  return set_err(ctx, HYEIG_EDEVICE, m);
}

void* ws_get(hyeig_ctx* ctx, int slot, size_t bytes, hyeig_status* st) {
  *st = HYEIG_OK;
  if (bytes == 0) bytes = 256;
  if (ctx->ws_size[slot] >= bytes) return ctx->ws[slot];
  if (ctx->ws[slot]) {
    hipStreamSynchronize(ctx->stream);
    hipFree(ctx->ws[slot]);
    ctx->ws[slot] = nullptr;
    ctx->ws_size[slot] = 0;
  }
  size_t sz = bytes + bytes / 4;
  hipError_t e = hipMalloc(&ctx->ws[slot], sz);
  if (e != hipSuccess) {
    *st = hip_err(ctx, e, "workspace hipMalloc");
    ctx->ws[slot] = nullptr;
    return nullptr;
  }
  ctx->ws_size[slot] = sz;
  return ctx->ws[slot];
}

void* pin_get(hyeig_ctx* ctx, size_t bytes, hyeig_status* st) {
  *st = HYEIG_OK;
  if (ctx->pin_size >= bytes) return ctx->pin;
  if (ctx->pin) {
    hipStreamSynchronize(ctx->stream);
    hipHostFree(ctx->pin);
    ctx->pin = nullptr;
    ctx->pin_size = 0;
  }
  size_t sz = std::max<size_t>(bytes + bytes / 4, 1 << 20);
  hipError_t e = hipHostMalloc(&ctx->pin, sz, hipHostMallocDefault);
  if (e != hipSuccess) {
    *st = hip_err(ctx, e, "pinned hipHostMalloc");
    ctx->pin = nullptr;
    return nullptr;
  }
  ctx->pin_size = sz;
  return ctx->pin;
}

hyeig_status h2d_queued(hyeig_ctx* ctx, void* d, const void* h, size_t bytes) {
  // h may be reused on return.  Arrays up to one ring slot are copied into
  // pinned memory and queued on the stream without waiting for it (kernels
  // already queued keep running while the host goes on); larger ones wait.
  if (bytes == 0) return HYEIG_OK;
  if (bytes <= H2D_SLOT_BYTES) {
    if (!ctx->h2d_ring) {
      hipError_t e = hipHostMalloc((void**)&ctx->h2d_ring, H2D_SLOTS * H2D_SLOT_BYTES, hipHostMallocDefault);
      if (e != hipSuccess) {
        ctx->h2d_ring = nullptr;
        return hip_err(ctx, e, "pinned hipHostMalloc (copy ring)");
      }
      for (int s = 0; s < H2D_SLOTS; ++s)
        HY_HIP(ctx, hipEventCreateWithFlags(&ctx->h2d_ev[s], hipEventDisableTiming));
    }
    const int s = ctx->h2d_next;
    ctx->h2d_next = (s + 1) % H2D_SLOTS;
    if (ctx->h2d_used[s]) HY_HIP(ctx, hipEventSynchronize(ctx->h2d_ev[s]));
    char* slot = ctx->h2d_ring + (size_t)s * H2D_SLOT_BYTES;
    std::memcpy(slot, h, bytes);
    HY_HIP(ctx, hipMemcpyAsync(d, slot, bytes, hipMemcpyHostToDevice, ctx->stream));
    HY_HIP(ctx, hipEventRecord(ctx->h2d_ev[s], ctx->stream));
    ctx->h2d_used[s] = true;
    return HYEIG_OK;
  }
  HY_HIP(ctx, hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, ctx->stream));
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return HYEIG_OK;
}

extern "C" {

hyeig_status hyeig_ctx_create(int device, void* hip_stream, hyeig_ctx** out) {
  if (!out) return HYEIG_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HYEIG_EDEVICE;
  hyeig_ctx* c = new (std::nothrow) hyeig_ctx();
  if (!c) return HYEIG_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return HYEIG_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
  if (hipEventCreate(&c->ev_a) != hipSuccess || hipEventCreate(&c->ev_b) != hipSuccess) {
    hyeig_ctx_destroy(c);
    return HYEIG_EDEVICE;
  }
  // device address of the fixed buffer of the allocation-free calls, once per device
  if (scratch_init(c) != HYEIG_OK) {
    hyeig_ctx_destroy(c);
    return HYEIG_EDEVICE;
  }
  *out = c;
  return HYEIG_OK;
}

void hyeig_ctx_destroy(hyeig_ctx* ctx) {
  if (!ctx) return;
  hipStreamSynchronize(ctx->stream);
  for (int i = 0; i < WS_COUNT; ++i)
    if (ctx->ws[i]) hipFree(ctx->ws[i]);
  if (ctx->pin) hipHostFree(ctx->pin);
  if (ctx->h2d_ring) hipHostFree(ctx->h2d_ring);
  for (int s = 0; s < H2D_SLOTS; ++s)
    if (ctx->h2d_ev[s]) hipEventDestroy(ctx->h2d_ev[s]);
  if (ctx->d2h_ev) hipEventDestroy(ctx->d2h_ev);
  if (ctx->ev_a) hipEventDestroy(ctx->ev_a);
  if (ctx->ev_b) hipEventDestroy(ctx->ev_b);
  delete ctx;
}

const char* hyeig_last_error(const hyeig_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

hyeig_status hyeig_last_spmm_ms(hyeig_ctx* ctx, double* h_ms) {
  if (!ctx || !h_ms) return HYEIG_EINVAL;
  if (!ctx->spmm_timed) return set_err(ctx, HYEIG_EINVAL, "last_spmm_ms: no product timed yet");
  HY_HIP(ctx, hipEventSynchronize(ctx->ev_b));
  float ms = 0.f;
  HY_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev_a, ctx->ev_b));
  *h_ms = ms;
  return HYEIG_OK;
}

static void mat_free(hyeig_mat* M) {
  if (!M) return;
  void* ps[] = {M->tile_ptr, M->tile_col, M->tile_val, M->tile_mask, M->tile_cmask, M->col_ptr, M->col_tiles,
                M->col_brow, M->vals,     M->vals_bf16, M->tvals, M->tvals_bf16, M->diag,  M->rowabs,
                M->rownnz,   M->pos,      M->tpos};
  for (void* p : ps)
    if (p) hipFree(p);
  delete M;
}

hyeig_status hyeig_mat_create(hyeig_ctx* ctx, int64_t n, int64_t nnz, const int64_t* d_rowptr,
                              const int32_t* d_colidx, const void* d_vals, hyeig_dtype vdt, uint32_t flags,
                              hyeig_mat** out) {
  if (!ctx || !out) return HYEIG_EINVAL;
  *out = nullptr;
  if (n <= 0 || nnz < 0 || !d_rowptr || (nnz > 0 && (!d_colidx || !d_vals)))
    return set_err(ctx, HYEIG_EINVAL, "mat_create: bad sizes or null pointers");
  if (n > (int64_t)INT32_MAX) return set_err(ctx, HYEIG_EINVAL, "mat_create: n above 2^31-1");
  if (vdt != HYEIG_F32) return set_err(ctx, HYEIG_EUNSUPPORTED, "mat_create: values must be FP32");
  HY_HIP(ctx, hipSetDevice(ctx->device));
  // row pointer ends
  int64_t ends[2];
  HY_HIP(ctx, hipMemcpyAsync(&ends[0], d_rowptr, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  HY_HIP(ctx, hipMemcpyAsync(&ends[1], d_rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ends[0] != 0 || ends[1] != nnz) return set_err(ctx, HYEIG_EINVAL, "mat_create: rowptr[0] != 0 or rowptr[n] != nnz");
  hyeig_status st;
  if (flags & HYEIG_MAT_VALIDATE) {
    int* flag = (int*)ws_get(ctx, WS_MISC, sizeof(int), &st);
    if (!flag) return st;
    HY_HIP(ctx, hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
    HY_CHECK(launch_validate(ctx, n, d_rowptr, d_colidx, flag));
    int h = 0;
    HY_HIP(ctx, hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h) return set_err(ctx, HYEIG_EINVAL, "mat_create: CSR is not an upper triangle with ascending columns");
  }
  hyeig_mat* M = new (std::nothrow) hyeig_mat();
  if (!M) return HYEIG_ENOMEM;
  M->ctx = ctx;
  M->n = n;
  M->nnz = nnz;
  M->nbr = (n + 31) / 32;
  auto fail = [&](hyeig_status s) {
    mat_free(M);
    return s;
  };
  hipError_t e;
#define MALLOC(p, bytes)                                     \
  e = hipMalloc((void**)&(p), std::max<size_t>((bytes), 64)); \
  if (e != hipSuccess) return fail(hip_err(ctx, e, "mat_create hipMalloc"));
  MALLOC(M->tile_ptr, sizeof(int64_t) * (M->nbr + 1));
  {
    // tiles per block row and padded value counts -> tile pointers and value bases
    int64_t* d_pv = nullptr;
    MALLOC(d_pv, sizeof(int64_t) * (M->nbr + 1));
    st = launch_tile_count(ctx, n, M->nbr, d_rowptr, d_colidx, M->tile_ptr + 1, d_pv + 1);
    if (st) {
      hipFree(d_pv);
      return fail(st);
    }
    std::vector<int64_t> cnt(M->nbr + 1, 0), pv(M->nbr + 1, 0);
    e = hipMemcpyAsync(cnt.data() + 1, M->tile_ptr + 1, sizeof(int64_t) * M->nbr, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(pv.data() + 1, d_pv + 1, sizeof(int64_t) * M->nbr, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      hipFree(d_pv);
      return fail(hip_err(ctx, e, "mat_create tile counts"));
    }
    for (int64_t i = 0; i < M->nbr; ++i) {
      cnt[i + 1] += cnt[i];
      pv[i + 1] += pv[i];
    }
    M->ntiles = cnt[M->nbr];
    M->nvals = pv[M->nbr];
    if (M->ntiles >= (int64_t)INT32_MAX) {
      hipFree(d_pv);
      return fail(set_err(ctx, HYEIG_EUNSUPPORTED, "mat_create: more than 2^31 tiles"));
    }
    e = hipMemcpyAsync(M->tile_ptr, cnt.data(), sizeof(int64_t) * (M->nbr + 1), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_pv, pv.data(), sizeof(int64_t) * (M->nbr + 1), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      hipFree(d_pv);
      return fail(hip_err(ctx, e, "mat_create tile pointers"));
    }
    MALLOC(M->tile_col, sizeof(int32_t) * M->ntiles);
    MALLOC(M->tile_val, sizeof(int64_t) * (M->ntiles + 1));
    MALLOC(M->tile_mask, sizeof(uint32_t) * 32 * M->ntiles);
    MALLOC(M->tile_cmask, sizeof(uint32_t) * 32 * M->ntiles);
    // value arrays carry VAL_PAD zero values past the last tile: a product lane
    // past its last entry may read up to 34 values beyond its tile
    MALLOC(M->vals, sizeof(float) * (M->nvals + VAL_PAD));
    MALLOC(M->diag, sizeof(float) * n);
    e = hipMemsetAsync(M->vals, 0, sizeof(float) * (M->nvals + VAL_PAD), ctx->stream);
    if (e != hipSuccess) {
      hipFree(d_pv);
      return fail(hip_err(ctx, e, "mat_create memset"));
    }
    // tile_val[ntiles] = nvals closes the last tile's value range
    e = hipMemcpyAsync(M->tile_val + M->ntiles, &pv[M->nbr], sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) {
      hipFree(d_pv);
      return fail(hip_err(ctx, e, "mat_create tile values"));
    }
    st = launch_tile_fill(ctx, M, d_rowptr, d_colidx, (const float*)d_vals, d_pv);
    if (st == HYEIG_OK) st = hip_err(ctx, hipStreamSynchronize(ctx->stream), "mat_create fill");
    hipFree(d_pv);
    if (st) return fail(st);
    // column-major copy of the tile values (padding zero, as in vals)
    MALLOC(M->tvals, sizeof(float) * (M->nvals + VAL_PAD));
    e = hipMemsetAsync(M->tvals, 0, sizeof(float) * (M->nvals + VAL_PAD), ctx->stream);
    if (e != hipSuccess) return fail(hip_err(ctx, e, "mat_create memset"));
    st = launch_tile_tvals(ctx, M);
    if (st) return fail(st);
    // column index of the tiles (counting sort by block column; block rows ascending)
    std::vector<int32_t> tcol(M->ntiles);
    e = hipMemcpy(tcol.data(), M->tile_col, sizeof(int32_t) * M->ntiles, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(hip_err(ctx, e, "mat_create tile columns"));
    std::vector<int64_t> cp(M->nbr + 1, 0);
    for (int64_t t = 0; t < M->ntiles; ++t) cp[tcol[t] + 1]++;
    for (int64_t i = 0; i < M->nbr; ++i) cp[i + 1] += cp[i];
    std::vector<int32_t> ct(M->ntiles), cb(M->ntiles);
    std::vector<int64_t> fillp(cp.begin(), cp.end() - 1);
    for (int64_t I = 0; I < M->nbr; ++I)
      for (int64_t t = cnt[I]; t < cnt[I + 1]; ++t) {
        const int64_t q = fillp[tcol[t]]++;
        ct[q] = (int32_t)t;
        cb[q] = (int32_t)I;
      }
    MALLOC(M->col_ptr, sizeof(int64_t) * (M->nbr + 1));
    MALLOC(M->col_tiles, sizeof(int32_t) * M->ntiles);
    MALLOC(M->col_brow, sizeof(int32_t) * M->ntiles);
    e = hipMemcpy(M->col_ptr, cp.data(), sizeof(int64_t) * (M->nbr + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M->col_tiles, ct.data(), sizeof(int32_t) * M->ntiles, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M->col_brow, cb.data(), sizeof(int32_t) * M->ntiles, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(hip_err(ctx, e, "mat_create column index"));
  }
  if (flags & HYEIG_MAT_BF16) {
    MALLOC(M->vals_bf16, sizeof(uint16_t) * (M->nvals + VAL_PAD));
    st = launch_to_bf16(ctx, M->nvals + VAL_PAD, M->vals, M->vals_bf16);
    if (st) return fail(st);
    MALLOC(M->tvals_bf16, sizeof(uint16_t) * (M->nvals + VAL_PAD));
    st = launch_to_bf16(ctx, M->nvals + VAL_PAD, M->tvals, M->tvals_bf16);
    if (st) return fail(st);
  }
  if (flags & HYEIG_MAT_ROWSTATS) {
    MALLOC(M->rowabs, sizeof(float) * n);
    MALLOC(M->rownnz, sizeof(float) * n);
    e = hipMemsetAsync(M->rowabs, 0, sizeof(float) * n, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(M->rownnz, 0, sizeof(float) * n, ctx->stream);
    if (e != hipSuccess) return fail(hip_err(ctx, e, "mat_create memset"));
    st = launch_rowstats(ctx, n, d_rowptr, d_colidx, (const float*)d_vals, M->rowabs, M->rownnz);
    if (st) return fail(st);
    std::vector<float> nz(n);
    e = hipMemcpyAsync(nz.data(), M->rownnz, sizeof(float) * n, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(hip_err(ctx, e, "mat_create row statistics"));
    double t = 0.0;
    for (int64_t r = 0; r < n; ++r) t += nz[r];
    M->rownnz_mean = t > 0 ? t / (double)n : 1.0;
  }
#undef MALLOC
  e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(hip_err(ctx, e, "mat_create build"));
  *out = M;
  return HYEIG_OK;
}

void hyeig_mat_destroy(hyeig_mat* mat) {
  if (!mat) return;
  hipDeviceSynchronize();  // the matrix may outlive its context
  mat_free(mat);
}

hyeig_status hyeig_mat_get_info(const hyeig_mat* M, hyeig_mat_info* info) {
  if (!M || !info) return HYEIG_EINVAL;
  info->n = M->n;
  info->nnz = M->nnz;
  info->ntiles = M->ntiles;
  info->nblockrows = M->nbr;
  info->prepared_bytes = M->nvals * (4 + 4 + (M->vals_bf16 ? 2 + 2 : 0) + (M->pos ? 2 + 2 : 0)) +
                         M->ntiles * (4 + 8 + 256 + 8) + 2 * (M->nbr + 1) * 8;
  info->d_diag = M->diag;
  info->d_rowabs = M->rowabs;
  info->d_rownnz = M->rownnz;
  return HYEIG_OK;
}

static bool dt_ok(hyeig_dtype d) { return d == HYEIG_F32 || d == HYEIG_F64; }

hyeig_status hyeig_spmm_sym(hyeig_ctx* ctx, const hyeig_mat* H, int m, const void* d_X, int64_t ldx,
                            hyeig_dtype xdt, void* d_Y, int64_t ldy, hyeig_dtype ydt, hyeig_dtype acc,
                            hyeig_dtype vdt) {
  if (!ctx) return HYEIG_EINVAL;
  if (!H || !d_X || !d_Y || m < 1 || m > 32 || ldx < m || ldy < m)
    return set_err(ctx, HYEIG_EINVAL, "spmm_sym: bad arguments (1 <= m <= 32, ld >= m, non-null)");
  if (!dt_ok(xdt) || !dt_ok(ydt) || !dt_ok(acc) || ydt != acc)
    return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: Y dtype must equal the accumulation dtype");
  if (vdt == HYEIG_BF16 && !H->vals_bf16)
    return set_err(ctx, HYEIG_EINVAL, "spmm_sym: matrix has no BF16 copy (HYEIG_MAT_BF16)");
  if (vdt != HYEIG_F32 && vdt != HYEIG_BF16) return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: value dtype");
  HY_HIP(ctx, hipEventRecord(ctx->ev_a, ctx->stream));
  HY_CHECK(launch_spmm(ctx, H, m, d_X, ldx, xdt, d_Y, ldy, acc, vdt));
  HY_HIP(ctx, hipEventRecord(ctx->ev_b, ctx->stream));
  ctx->spmm_timed = true;
  return HYEIG_OK;
}

hyeig_status hyeig_gram(hyeig_ctx* ctx, int64_t n, int ka, const void* d_A, int64_t lda, int kb, const void* d_B,
                        int64_t ldb, hyeig_dtype dt, hyeig_mma_mode mode, double* d_G) {
  if (!ctx) return HYEIG_EINVAL;
  if (n < 0 || ka < 1 || kb < 1 || ka > 64 || kb > 64 || lda < ka || ldb < kb || !d_A || !d_B || !d_G)
    return set_err(ctx, HYEIG_EINVAL, "gram: bad arguments (1 <= ka, kb <= 64, ld >= width, non-null)");
  if (!dt_ok(dt)) return set_err(ctx, HYEIG_EUNSUPPORTED, "gram: dtype");
  if ((mode == HYEIG_MMA_F32 || mode == HYEIG_MMA_SPLIT_BF16) && dt != HYEIG_F32)
    return set_err(ctx, HYEIG_EUNSUPPORTED, "gram: FP32 and split-BF16 modes need FP32 data");
  // n = 0: G = 0 by a fill kernel (no memset node for callers that capture graphs)
  if (n == 0) return launch_fill(ctx, 1, ka * kb, d_G, ka * kb, HYEIG_F64, 0.0);
  return launch_gram(ctx, n, ka, d_A, lda, kb, d_B, ldb, dt, mode, d_G);
}

hyeig_status hyeig_gram_noalloc(hyeig_ctx* ctx, int64_t n, int ka, const void* d_A, int64_t lda, int kb,
                                const void* d_B, int64_t ldb, hyeig_dtype dt, hyeig_mma_mode mode, double* d_G) {
  if (!ctx) return HYEIG_EINVAL;
  if (n < 0 || ka < 1 || kb < 1 || ka > 64 || kb > 64 || lda < ka || ldb < kb || !d_A || !d_B || !d_G)
    return set_err(ctx, HYEIG_EINVAL, "gram_noalloc: bad arguments (1 <= ka, kb <= 64, ld >= width, non-null)");
  if (!dt_ok(dt)) return set_err(ctx, HYEIG_EUNSUPPORTED, "gram_noalloc: dtype");
  if ((mode == HYEIG_MMA_F32 || mode == HYEIG_MMA_SPLIT_BF16) && dt != HYEIG_F32)
    return set_err(ctx, HYEIG_EUNSUPPORTED, "gram_noalloc: FP32 and split-BF16 modes need FP32 data");
  // n = 0: G = 0 by a fill kernel (no memset node for callers that capture graphs)
  if (n == 0) return launch_fill(ctx, 1, ka * kb, d_G, ka * kb, HYEIG_F64, 0.0);
  return launch_gram_noalloc(ctx, n, ka, d_A, lda, kb, d_B, ldb, dt, mode, d_G);
}

hyeig_status hyeig_block_update(hyeig_ctx* ctx, int64_t n, int k, int m, const void* d_S, int64_t lds,
                                const double* d_C, double beta, void* d_Y, int64_t ldy, hyeig_dtype dt,
                                hyeig_mma_mode mode) {
  (void)mode;
  if (!ctx) return HYEIG_EINVAL;
  if (n < 0 || k < 1 || m < 1 || k > 64 || m > 32 || lds < k || ldy < m || !d_S || !d_C || !d_Y)
    return set_err(ctx, HYEIG_EINVAL, "block_update: bad arguments (1 <= k <= 64, 1 <= m <= 32)");
  if (!dt_ok(dt)) return set_err(ctx, HYEIG_EUNSUPPORTED, "block_update: dtype");
  if (d_Y == d_S && !(ldy == lds && m == k && beta == 0.0))
    return set_err(ctx, HYEIG_EINVAL, "block_update: in place needs ldy == lds, m == k, beta == 0");
  return launch_block_update(ctx, n, k, m, d_S, lds, d_C, beta, d_Y, ldy, dt);
}

hyeig_status hyeig_cholqr(hyeig_ctx* ctx, int64_t n, int m, void* d_X, int64_t ldx, hyeig_dtype dt, int passes,
                          double* d_R) {
  if (!ctx) return HYEIG_EINVAL;
  if (n < m || m < 1 || m > 32 || ldx < m || !d_X || passes < 1 || passes > 3)
    return set_err(ctx, HYEIG_EINVAL, "cholqr: bad arguments (n >= m, 1 <= m <= 32, 1 <= passes <= 3)");
  if (!dt_ok(dt)) return set_err(ctx, HYEIG_EUNSUPPORTED, "cholqr: dtype");
  hyeig_status st;
  double* dG = (double*)ws_get(ctx, WS_SMALL, sizeof(double) * 2 * m * m, &st);
  if (!dG) return st;
  double* dRi = dG + m * m;
  double* h = (double*)pin_get(ctx, sizeof(double) * m * m, &st);
  if (!h) return st;
  std::vector<double> Rtot(m * m, 0.0), R(m * m), Ri(m * m);
  for (int i = 0; i < m; ++i) Rtot[i + i * m] = 1.0;
  for (int p = 0; p < passes; ++p) {
    HY_CHECK(launch_gram(ctx, n, m, d_X, ldx, m, d_X, ldx, dt, HYEIG_MMA_F64, dG));
    HY_HIP(ctx, hipMemcpyAsync(h, dG, sizeof(double) * m * m, hipMemcpyDeviceToHost, ctx->stream));
    HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < m * m; ++i)
      if (!std::isfinite(h[i])) return set_err(ctx, HYEIG_ENUMERIC, "cholqr: NaN/Inf in X^T X");
    if (!sd::cholesky_upper(m, h, R.data())) return set_err(ctx, HYEIG_ENOTSPD, "cholqr: X^T X not positive definite");
    sd::tri_upper_inv(m, R.data(), Ri.data());
    HY_CHECK(h2d_queued(ctx, dRi, Ri.data(), sizeof(double) * m * m));
    HY_CHECK(launch_block_update(ctx, n, m, m, d_X, ldx, dRi, 0.0, d_X, ldx, dt));
    std::vector<double> T(m * m, 0.0);  // Rtot <- R * Rtot
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int q = 0; q < m; ++q) s += R[i + q * m] * Rtot[q + j * m];
        T[i + j * m] = s;
      }
    Rtot = T;
  }
  if (d_R) HY_CHECK(h2d_queued(ctx, d_R, Rtot.data(), sizeof(double) * m * m));
  return HYEIG_OK;
}

hyeig_status hyeig_rayleigh_ritz(hyeig_ctx* ctx, int k, const double* A, const double* B, int nwant, double* theta,
                                 double* C, double* condB, int on_device) {
  if (!ctx) return HYEIG_EINVAL;
  if (k < 1 || k > 4096 || nwant < 1 || nwant > k || !A || !theta || !C)
    return set_err(ctx, HYEIG_EINVAL, "rayleigh_ritz: bad arguments");
  std::vector<double> hA((size_t)k * k), hB, hC((size_t)k * nwant), ht(nwant);
  if (on_device) {
    HY_HIP(ctx, hipMemcpyAsync(hA.data(), A, sizeof(double) * k * k, hipMemcpyDeviceToHost, ctx->stream));
    if (B) {
      hB.resize((size_t)k * k);
      HY_HIP(ctx, hipMemcpyAsync(hB.data(), B, sizeof(double) * k * k, hipMemcpyDeviceToHost, ctx->stream));
    }
    HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  } else {
    std::memcpy(hA.data(), A, sizeof(double) * k * k);
    if (B) hB.assign(B, B + (size_t)k * k);
  }
  double cb = 1.0;
  if (!sd::gen_eig(k, hA.data(), B ? hB.data() : nullptr, nwant, ht.data(), hC.data(), condB ? &cb : nullptr))
    return set_err(ctx, HYEIG_ENOTSPD, "rayleigh_ritz: B not positive definite or eigensolver failed");
  if (condB) *condB = cb;
  if (on_device) {
    HY_CHECK(h2d_queued(ctx, theta, ht.data(), sizeof(double) * nwant));
    HY_CHECK(h2d_queued(ctx, C, hC.data(), sizeof(double) * k * nwant));
  } else {
    std::memcpy(theta, ht.data(), sizeof(double) * nwant);
    std::memcpy(C, hC.data(), sizeof(double) * k * nwant);
  }
  return HYEIG_OK;
}

}  // extern "C"
