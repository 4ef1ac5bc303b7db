// Half-stored symmetric block product Y = H X, H = U + U^T - diag(U), for gfx950.
//
// The prepared form groups the upper triangle U in 32 x 32 tiles.  For tile
// (I, J) (block row I, block column J >= I) it keeps the 32 row bitmasks, the 32
// column bitmasks (the diagonal excluded, so each diagonal entry is applied
// once) and the tile's values packed row-major.  One 64-lane wavefront owns one
// block row I at a time:
//   lanes  0..31  direct half:     y_I[r, :] += u_rc x_J[c, :]  (row r = lane)
//   lanes 32..63  transposed half: y_J[c, :] += u_rc x_I[r, :]  (column c = lane - 32)
// Both halves run the same instruction stream over their own bitmask (the
// direct half walks the set bits of its row, the transposed half the set bits
// of its column), reading the packed values, x_J and x_I from LDS.  The
// transposed partials of a tile are staged in LDS and added to Y with
// coalesced atomics; the direct partials of the block row are added once at
// the end.  Y is cleared first.  U is read exactly once per product.
#include <hip/hip_runtime.h>

#include <climits>

#include "internal.h"

namespace {

constexpr int WAVE = 64;

__device__ inline int wave_min_i32(int v) {
  for (int off = 32; off >= 1; off >>= 1) {
    int o = __shfl_xor(v, off, WAVE);
    v = o < v ? o : v;
  }
  return v;
}

// exclusive prefix sum over lanes 0..31 (lanes >= 32 take part but their values are ignored)
__device__ inline uint32_t excl_scan32(uint32_t v, int lane, uint32_t* total) {
  uint32_t x = v;
  for (int off = 1; off < 32; off <<= 1) {
    uint32_t o = __shfl_up(x, off, 32);
    if ((lane & 31) >= off) x += o;
  }
  *total = __shfl(x, 31, WAVE);
  return x - v;
}

// ---------------------------------------------------------------------------
// prepared-form construction from the upper-triangle CSR
// ---------------------------------------------------------------------------
__global__ void k_tile_count(int64_t n, int64_t nbr, const int64_t* __restrict__ rowptr,
                             const int32_t* __restrict__ colidx, int64_t* __restrict__ counts) {
  const int lane = threadIdx.x & 63;
  const int64_t br = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (br >= nbr) return;
  const int64_t row = br * 32 + lane;
  const bool own = lane < 32 && row < n;
  int64_t p = own ? rowptr[row] : 0, e = own ? rowptr[row + 1] : 0;
  int64_t cnt = 0;
  for (;;) {
    int cur = (p < e) ? (colidx[p] >> 5) : INT_MAX;
    int J = wave_min_i32(cur);
    if (J == INT_MAX) break;
    ++cnt;
    while (p < e && (colidx[p] >> 5) == J) ++p;
  }
  if (lane == 0) counts[br] = cnt;
}

__global__ void k_tile_fill(int64_t n, int64_t nbr, const int64_t* __restrict__ rowptr,
                            const int32_t* __restrict__ colidx, const float* __restrict__ vin,
                            const int64_t* __restrict__ tile_ptr, int32_t* __restrict__ tile_col,
                            int64_t* __restrict__ tile_val, uint32_t* __restrict__ tile_mask,
                            uint32_t* __restrict__ tile_cmask, float* __restrict__ vout, float* __restrict__ diag) {
  const int lane = threadIdx.x & 63;
  const int64_t br = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (br >= nbr) return;
  const int64_t row = br * 32 + lane;
  const bool own = lane < 32 && row < n;
  int64_t p = own ? rowptr[row] : 0, e = own ? rowptr[row + 1] : 0;
  int64_t vbase = rowptr[br * 32];
  int64_t t = tile_ptr[br];
  if (own) diag[row] = 0.0f;
  for (;;) {
    int cur = (p < e) ? (colidx[p] >> 5) : INT_MAX;
    int J = wave_min_i32(cur);
    if (J == INT_MAX) break;
    uint32_t mask = 0;
    int64_t p0 = p;
    while (p < e && (colidx[p] >> 5) == J) {
      int c = colidx[p] & 31;
      mask |= 1u << c;
      if ((int64_t)colidx[p] == row) diag[row] = vin[p];
      ++p;
    }
    uint32_t total;
    uint32_t cnt = (lane < 32) ? (uint32_t)__popc(mask) : 0u;
    uint32_t off = excl_scan32(cnt, lane, &total);
    for (uint32_t q = 0; q < cnt; ++q) vout[vbase + off + q] = vin[p0 + q];
    // column bitmasks by transposing the 32 row masks
    uint32_t cm = 0;
    for (int r = 0; r < 32; ++r) {
      uint32_t mr = __shfl(mask, r, WAVE);
      if (lane < 32) cm |= ((mr >> lane) & 1u) << r;
    }
    if ((int64_t)J == br && lane < 32) cm &= ~(1u << lane);  // diagonal applied once (direct half)
    if (lane < 32) {
      tile_mask[t * 32 + lane] = mask;
      tile_cmask[t * 32 + lane] = cm;
    }
    if (lane == 0) {
      tile_col[t] = J;
      tile_val[t] = vbase;
    }
    vbase += total;
    ++t;
  }
}

__global__ void k_validate(int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                           int* flag) {
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  int64_t p = rowptr[row], e = rowptr[row + 1];
  if (e < p) {
    atomicOr(flag, 1);
    return;
  }
  int prev = -1;
  for (int64_t q = p; q < e; ++q) {
    int c = colidx[q];
    if ((int64_t)c < row || (int64_t)c >= n || c <= prev) {
      atomicOr(flag, 2);
      return;
    }
    prev = c;
  }
}

__global__ void k_rowstats(int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                           const float* __restrict__ v, float* __restrict__ rowabs, float* __restrict__ rownnz) {
  int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  float s = 0.f, c = 0.f;
  for (int64_t q = rowptr[row]; q < rowptr[row + 1]; ++q) {
    float a = fabsf(v[q]);
    s += a;
    c += 1.f;
    int col = colidx[q];
    if ((int64_t)col != row) {
      atomicAdd(&rowabs[col], a);
      atomicAdd(&rownnz[col], 1.f);
    }
  }
  atomicAdd(&rowabs[row], s);
  atomicAdd(&rownnz[row], c);
}

__global__ void k_to_bf16(int64_t nnz, const float* __restrict__ src, uint16_t* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  uint32_t u = __float_as_uint(src[i]);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;  // round to nearest even (values are finite)
  dst[i] = (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// the product
// ---------------------------------------------------------------------------
template <typename VT>
__device__ inline float val_to_f32(VT v);
template <>
__device__ inline float val_to_f32<float>(float v) {
  return v;
}
template <>
__device__ inline float val_to_f32<uint16_t>(uint16_t v) {
  return __uint_as_float((uint32_t)v << 16);
}

template <typename T>
__device__ inline void atomic_add_y(T* p, T v);
template <>
__device__ inline void atomic_add_y<float>(float* p, float v) {
  unsafeAtomicAdd(p, v);
}
template <>
__device__ inline void atomic_add_y<double>(double* p, double v) {
  unsafeAtomicAdd(p, v);
}

// Per-wave LDS footprint (elements of AT for the x tiles and the staging tile).
template <int M, typename AT>
struct SpmmLds {
  static constexpr int XT_ELEMS = 32 * M;
  static constexpr int BYTES = 3 * XT_ELEMS * (int)sizeof(AT) + 1024 * 4 + 32 * 8;
  static constexpr int WAVES = (BYTES * 4 <= 65536) ? 4 : 2;
};

template <int M, typename XT, typename AT, typename VT>
__global__ __launch_bounds__(256) void k_spmm_sym(int64_t n, int64_t nbr, const int64_t* __restrict__ tile_ptr,
                                                  const int32_t* __restrict__ tile_col,
                                                  const int64_t* __restrict__ tile_val,
                                                  const uint32_t* __restrict__ tile_mask,
                                                  const uint32_t* __restrict__ tile_cmask,
                                                  const VT* __restrict__ vals, int m, const XT* __restrict__ X,
                                                  int64_t ldx, AT* __restrict__ Y, int64_t ldy) {
  using L = SpmmLds<M, AT>;
  constexpr int WAVES = L::WAVES;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t I = (int64_t)blockIdx.x * WAVES + wv;
  if (I >= nbr) return;  // wave-uniform

  unsigned char* base = lds_raw + (size_t)wv * L::BYTES;
  AT* XI = reinterpret_cast<AT*>(base);
  AT* XJ = XI + L::XT_ELEMS;
  AT* TS = XJ + L::XT_ELEMS;
  float* P = reinterpret_cast<float*>(TS + L::XT_ELEMS);
  uint2* RI = reinterpret_cast<uint2*>(P + 1024);

  const bool dir = lane < 32;
  const int self = lane & 31;

  // x_I of the block row
  for (int e = lane; e < 32 * M; e += WAVE) {
    int r = e / M, j = e % M;
    int64_t row = I * 32 + r;
    XI[e] = (row < n && j < m) ? (AT)X[row * ldx + j] : (AT)0;
  }

  AT a[M];
#pragma unroll
  for (int j = 0; j < M; ++j) a[j] = (AT)0;

  const int64_t t0 = tile_ptr[I], t1 = tile_ptr[I + 1];
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t J = tile_col[t];
    const int64_t vb = tile_val[t];
    uint32_t bits;
    uint32_t rowm = 0;
    if (dir) {
      rowm = tile_mask[t * 32 + self];
      bits = rowm;
    } else {
      bits = tile_cmask[t * 32 + self];
    }
    uint32_t total;
    uint32_t cnt = dir ? (uint32_t)__popc(rowm) : 0u;
    uint32_t off = excl_scan32(cnt, lane, &total);
    if (dir) RI[self] = make_uint2(off, rowm);
    for (int e = lane; e < (int)total; e += WAVE) P[e] = val_to_f32<VT>(vals[vb + e]);
    for (int e = lane; e < 32 * M; e += WAVE) {
      int r = e / M, j = e % M;
      int64_t row = J * 32 + r;
      XJ[e] = (row < n && j < m) ? (AT)X[row * ldx + j] : (AT)0;
    }
    if (!dir) {
#pragma unroll
      for (int j = 0; j < M; ++j) a[j] = (AT)0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const AT* xb = dir ? XJ : XI;
    while (bits) {
      const int idx = __builtin_ctz(bits);
      bits &= bits - 1u;
      const int r = dir ? self : idx;
      const int c = dir ? idx : self;
      const uint2 ri = RI[r];
      const uint32_t pos = ri.x + (uint32_t)__popc(ri.y & ((1u << c) - 1u));
      const AT v = (AT)P[pos];
      const AT* xr = xb + idx * M;
#pragma unroll
      for (int j = 0; j < M; ++j) a[j] += v * xr[j];
    }

    // transposed partials of this tile -> Y rows of block J
    if (!dir) {
#pragma unroll
      for (int j = 0; j < M; ++j) TS[self * M + j] = a[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int e = lane; e < 32 * M; e += WAVE) {
      int r = e / M, j = e % M;
      int64_t row = J * 32 + r;
      if (row < n && j < m) atomic_add_y<AT>(&Y[row * ldy + j], TS[e]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // direct partials of the block row
  if (dir) {
#pragma unroll
    for (int j = 0; j < M; ++j) TS[self * M + j] = a[j];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int e = lane; e < 32 * M; e += WAVE) {
    int r = e / M, j = e % M;
    int64_t row = I * 32 + r;
    if (row < n && j < m) atomic_add_y<AT>(&Y[row * ldy + j], TS[e]);
  }
}

template <int M, typename XT, typename AT, typename VT>
hyeig_status run_spmm(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                      const VT* vals) {
  using L = SpmmLds<M, AT>;
  const int waves = L::WAVES;
  const int64_t blocks = (H->nbr + waves - 1) / waves;
  if (blocks == 0) return HYEIG_OK;
  const size_t lds = (size_t)L::BYTES * waves;
  auto kern = k_spmm_sym<M, XT, AT, VT>;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), lds, ctx->stream, H->n, H->nbr, H->tile_ptr,
                     H->tile_col, H->tile_val, H->tile_mask, H->tile_cmask, vals, m, X, ldx, Y, ldy);
  return hip_err(ctx, hipGetLastError(), "k_spmm_sym launch");
}

template <typename XT, typename AT, typename VT>
hyeig_status spmm_width(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                        const VT* vals) {
  if (m <= 1) return run_spmm<1, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals);
  if (m <= 2) return run_spmm<2, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals);
  if (m <= 4) return run_spmm<4, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals);
  if (m <= 8) return run_spmm<8, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals);
  if (m <= 12) return run_spmm<12, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals);
  if (m <= 16) return run_spmm<16, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals);
  return run_spmm<32, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals);
}

}  // namespace

hyeig_status launch_tile_count(hyeig_ctx* ctx, int64_t n, int64_t nbr, const int64_t* rowptr, const int32_t* colidx,
                               int64_t* counts) {
  int64_t blocks = (nbr * 64 + 255) / 256;
  hipLaunchKernelGGL(k_tile_count, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, nbr, rowptr, colidx,
                     counts);
  return hip_err(ctx, hipGetLastError(), "k_tile_count launch");
}

hyeig_status launch_tile_fill(hyeig_ctx* ctx, hyeig_mat* M, const int64_t* rowptr, const int32_t* colidx,
                              const float* vals) {
  int64_t blocks = (M->nbr * 64 + 255) / 256;
  hipLaunchKernelGGL(k_tile_fill, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, M->n, M->nbr, rowptr, colidx,
                     vals, M->tile_ptr, M->tile_col, M->tile_val, M->tile_mask, M->tile_cmask, M->vals, M->diag);
  return hip_err(ctx, hipGetLastError(), "k_tile_fill launch");
}

hyeig_status launch_validate(hyeig_ctx* ctx, int64_t n, const int64_t* rowptr, const int32_t* colidx, int* flag) {
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, rowptr, colidx, flag);
  return hip_err(ctx, hipGetLastError(), "k_validate launch");
}

hyeig_status launch_rowstats(hyeig_ctx* ctx, int64_t n, const int64_t* rowptr, const int32_t* colidx,
                             const float* vals, float* rowabs, float* rownnz) {
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_rowstats, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, rowptr, colidx, vals, rowabs,
                     rownnz);
  return hip_err(ctx, hipGetLastError(), "k_rowstats launch");
}

hyeig_status launch_to_bf16(hyeig_ctx* ctx, int64_t nnz, const float* src, uint16_t* dst) {
  int64_t blocks = (nnz + 255) / 256;
  if (blocks == 0) return HYEIG_OK;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, nnz, src, dst);
  return hip_err(ctx, hipGetLastError(), "k_to_bf16 launch");
}

hyeig_status launch_spmm(hyeig_ctx* ctx, const hyeig_mat* H, int m, const void* X, int64_t ldx, hyeig_dtype xdt,
                         void* Y, int64_t ldy, hyeig_dtype acc, hyeig_dtype vdt) {
  if (vdt == HYEIG_BF16) {
    if (xdt == HYEIG_F32 && acc == HYEIG_F32)
      return spmm_width<float, float, uint16_t>(ctx, H, m, (const float*)X, ldx, (float*)Y, ldy, H->vals_bf16);
    return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: BF16 values need FP32 X and FP32 accumulation");
  }
  if (xdt == HYEIG_F32 && acc == HYEIG_F32)
    return spmm_width<float, float, float>(ctx, H, m, (const float*)X, ldx, (float*)Y, ldy, H->vals);
  if (xdt == HYEIG_F64 && acc == HYEIG_F64)
    return spmm_width<double, double, float>(ctx, H, m, (const double*)X, ldx, (double*)Y, ldy, H->vals);
  if (xdt == HYEIG_F32 && acc == HYEIG_F64)
    return spmm_width<float, double, float>(ctx, H, m, (const float*)X, ldx, (double*)Y, ldy, H->vals);
  return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: unsupported dtype combination");
}
