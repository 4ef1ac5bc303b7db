// Tall-skinny dense kernels of the block eigensolvers on gfx950:
//   gram          G = A^T B  (matrix cores; per-workgroup partials reduced in FP64)
//   block_update  Y = S C + beta Y, and a two-output form for the LOBPCG updates
//   residual + shifted-diagonal preconditioner with FP64 column norms
//   column dots / scaling / copies / fills
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "internal.h"

namespace {

constexpr int WAVE = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename T>
__device__ inline double to_d(T v) {
  return (double)v;
}

// ---------------------------------------------------------------------------
// reductions of per-block column partials:  out[c] = sum_b part[b * ncols + c]
// ---------------------------------------------------------------------------
__global__ void k_reduce_cols(int nblk, int ncols, const double* __restrict__ part, double* __restrict__ out) {
  int c = blockIdx.x * blockDim.y + threadIdx.y;
  if (c >= ncols) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[(int64_t)b * ncols + c];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, WAVE);
  if (threadIdx.x == 0) out[c] = s;
}


// ---------------------------------------------------------------------------
// fill / copy / scale
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(int64_t n, int m, T* __restrict__ Y, int64_t ld, T v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (i >= n) return;
  for (int j = threadIdx.x; j < m; j += blockDim.x) Y[i * ld + j] = v;
}

// Pseudo-random fill that does not depend on the launch shape: element (i, j)
// is the SplitMix64 output (Steele, Lea and Flood, OOPSLA 2014) for the
// counter i m + j + 1 of the stream seed, its top 53 bits mapped to [-1, 1).
template <typename T>
__global__ void k_fill_hash(int64_t n, int m, T* __restrict__ Y, int64_t ld, uint64_t seed) {
  int64_t i = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (i >= n) return;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    uint64_t z = seed + (uint64_t)(i * m + j + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    Y[i * ld + j] = (T)((double)(z >> 11) * 0x1.0p-52 - 1.0);
  }
}

template <typename TX, typename TY>
__global__ void k_copy(int64_t n, int m, const TX* __restrict__ X, int64_t ldx, TY* __restrict__ Y, int64_t ldy) {
  int64_t i = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (i >= n) return;
  for (int j = threadIdx.x; j < m; j += blockDim.x) Y[i * ldy + j] = (TY)X[i * ldx + j];
}

// Y (n x mp, contiguous) = [X(:, 0:m) 0]: columns gathered from wider rows, zero-padded
template <typename T>
__global__ void k_gather_pad(int64_t n, int m, int mp, const T* __restrict__ X, int64_t ldx, T* __restrict__ Y) {
  const int64_t tot = n * mp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / mp;
    const int c = (int)(e - i * mp);
    Y[e] = c < m ? X[i * ldx + c] : (T)0;
  }
}

// Y = a A + b B + g C (C optional), n x m blocks with their own leading
// dimensions, combined in FP64: the steps of the Chebyshev three-term recurrence
template <typename T>
__global__ void k_lincomb(int64_t n, int m, double a, const T* __restrict__ A, int64_t lda, double b,
                          const T* __restrict__ B, int64_t ldb, double g, const T* __restrict__ C, int64_t ldc,
                          T* __restrict__ Y, int64_t ldy) {
  int64_t i = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (i >= n) return;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double v = a * (double)A[i * lda + j] + b * (double)B[i * ldb + j];
    if (C) v += g * (double)C[i * ldc + j];
    Y[i * ldy + j] = (T)v;
  }
}

// Y[:, j] = X[:, idx[j]] for j < m (columns picked by a device index list)
template <typename T>
__global__ void k_gather_cols(int64_t n, int m, const int* __restrict__ idx, const T* __restrict__ X, int64_t ldx,
                              T* __restrict__ Y, int64_t ldy) {
  int64_t i = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (i >= n) return;
  for (int j = threadIdx.x; j < m; j += blockDim.x) Y[i * ldy + j] = X[i * ldx + idx[j]];
}

template <typename T>
__global__ void k_col_scale(int64_t n, int m, T* __restrict__ Y, int64_t ld, const double* __restrict__ s) {
  int64_t i = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (i >= n) return;
  for (int j = threadIdx.x; j < m; j += blockDim.x) Y[i * ld + j] = (T)((double)Y[i * ld + j] * s[j]);
}

// column dots with per-block partials; block = 32 columns x 8 rows
template <typename T>
__global__ void k_col_dots(int64_t n, int m, const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                           int64_t ldb, double* __restrict__ part) {
  __shared__ double red[8][33];
  const int j = threadIdx.x, ty = threadIdx.y;
  double s = 0.0;
  if (j < m)
    for (int64_t i = (int64_t)blockIdx.x * 8 + ty; i < n; i += (int64_t)gridDim.x * 8)
      s += (double)A[i * lda + j] * (double)B[i * ldb + j];
  red[ty][j] = s;
  __syncthreads();
  if (ty == 0 && j < m) {
    double t = 0.0;
    for (int q = 0; q < 8; ++q) t += red[q][j];
    part[(int64_t)blockIdx.x * m + j] = t;
  }
}

// ---------------------------------------------------------------------------
// Gram G = A^T B on matrix cores, and with SYM also A^T A in the same pass over
// A (the projected pair S^T H S, S^T S of the Rayleigh-Ritz step reads S and HS
// once).  The reduction index is the row: in a 16x16x4 MFMA lane l feeds
// A^T[i = l%16][k = l/16] and B[k = l/16][j = l%16], so the four lane groups
// take four consecutive rows.  Each wave walks its share of rows 16 at a time
// (four 4-row slices).  A and B are read through one buffer resource each that
// ends with the wave's rows; a lane's offset is its row part plus its column
// part (out of range past the width), so rows past the end and absent columns
// read zero without a branch.  A slice is reloaded for the next step as soon
// as its MFMAs are issued (the last step is peeled, so the steady loop has no
// condition).  A^T A is formed on its upper block triangle and mirrored.  The
// 4 waves of a workgroup add their tiles in LDS (FP64) and the workgroup writes
// one FP64 partial of ka x kb (then ka x ka).
// ---------------------------------------------------------------------------
template <typename T>
struct GBits;
template <>
struct GBits<float> {
  using V = uint32_t;
  static __device__ V load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
  }
  static __device__ float val(V v) { return __uint_as_float(v); }
};
template <>
struct GBits<double> {
  using V = __attribute__((ext_vector_type(2))) unsigned int;
  static __device__ V load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
  }
  static __device__ double val(V v) { return __builtin_bit_cast(double, v); }
};
constexpr uint32_t GRAM_OOB = 0x7FFFFFF0u;

template <typename T, bool F64MMA, int TA, int TB, bool SYM, bool PL>
__global__ __launch_bounds__(256) void k_gram(int64_t n, int ka, const T* __restrict__ A, int64_t lda, int kb,
                                              const T* __restrict__ B, int64_t ldb, int64_t bsa, int64_t bsb,
                                              int64_t rows_per_wave, double* __restrict__ part) {
  extern __shared__ double red[];
  using G = GBits<T>;
  using VT4 = typename std::conditional<F64MMA, f64x4, f32x4>::type;
  using MT = typename std::conditional<F64MMA, double, float>::type;
  constexpr uint32_t S = sizeof(T);
  constexpr int NS = SYM ? TA * (TA + 1) / 2 : 0;  // upper block triangle of A^T A
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i16 = lane & 15, k4 = lane >> 4;
  const int kt = SYM ? kb + ka : kb;  // columns of the partial
  for (int e = threadIdx.x; e < ka * kt; e += 256) red[e] = 0.0;
  __syncthreads();
  const int64_t wid = (int64_t)blockIdx.x * 4 + wv;
  const int64_t r0 = wid * rows_per_wave;
  const int64_t r1 = (r0 + rows_per_wave < n) ? r0 + rows_per_wave : n;
  VT4 acc[TA][TB], accs[NS > 0 ? NS : 1];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[a][b] = VT4{0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < (NS > 0 ? NS : 1); ++t) accs[t] = VT4{0, 0, 0, 0};

  if (r0 < r1) {
    const int64_t rows = r1 - r0;
    // PL: column block c of a matrix is its own n x 16 array, bs elements after
    // block c - 1 (one resource per block); otherwise one row-major array
    __amdgpu_buffer_rsrc_t ra[PL ? TA : 1], rb[PL ? TB : 1];
    uint32_t ca[TA], cb[TB];
#pragma unroll
    for (int a = 0; a < (PL ? TA : 1); ++a)
      ra[a] = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(A + a * bsa + r0 * lda), (short)0,
                                                (int)(rows * lda * S), 0x00020000);
#pragma unroll
    for (int b = 0; b < (PL ? TB : 1); ++b)
      rb[b] = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(B + b * bsb + r0 * ldb), (short)0,
                                                (int)(rows * ldb * S), 0x00020000);
#pragma unroll
    for (int a = 0; a < TA; ++a)
      ca[a] = 16 * a + i16 < ka ? (uint32_t)(((PL ? 0 : 16 * a) + i16) * S) : GRAM_OOB;
#pragma unroll
    for (int b = 0; b < TB; ++b)
      cb[b] = 16 * b + i16 < kb ? (uint32_t)(((PL ? 0 : 16 * b) + i16) * S) : GRAM_OOB;
    typename G::V va[4][TA], vb[4][TB];
    // slice u of the 16 rows from r: row r + 4 u + k4 of every block
    auto load_slice = [&](int64_t r, int u) {
      const int64_t row = r + 4 * u + k4;
      const uint32_t oa = (uint32_t)(row * lda * S), ob = (uint32_t)(row * ldb * S);
#pragma unroll
      for (int a = 0; a < TA; ++a) va[u][a] = G::load(ra[PL ? a : 0], oa + ca[a]);
#pragma unroll
      for (int b = 0; b < TB; ++b) vb[u][b] = G::load(rb[PL ? b : 0], ob + cb[b]);
    };
    auto mma_slice = [&](const MT(&xa)[TA], const MT(&xb)[TB]) {
#pragma unroll
      for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b) {
          if constexpr (F64MMA)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a], xb[b], acc[a][b], 0, 0, 0);
          else
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[a], xb[b], acc[a][b], 0, 0, 0);
        }
      if constexpr (SYM) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < TA; ++a)
#pragma unroll
          for (int a2 = a; a2 < TA; ++a2, ++t) {
            if constexpr (F64MMA)
              accs[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a], xa[a2], accs[t], 0, 0, 0);
            else
              accs[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[a], xa[a2], accs[t], 0, 0, 0);
          }
      }
    };
    auto step = [&](int64_t r, bool next) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        MT xa[TA], xb[TB];
#pragma unroll
        for (int a = 0; a < TA; ++a) xa[a] = (MT)G::val(va[u][a]);
#pragma unroll
        for (int b = 0; b < TB; ++b) xb[b] = (MT)G::val(vb[u][b]);
        if (next) load_slice(r + 16, u);
        mma_slice(xa, xb);
      }
    };
#pragma unroll
    for (int u = 0; u < 4; ++u) load_slice(0, u);
    int64_t r = 0;
    for (; r + 16 < rows; r += 16) step(r, true);
    step(r, false);
  }
  // FP64 16x16x4: element q of lane l holds row 4 q + l / 16;
  // FP32 16x16x4: element q of lane l holds row 4 (l / 16) + q
  auto row_of = [&](int q) { return F64MMA ? 4 * q + k4 : 4 * k4 + q; };
  for (int w = 0; w < 4; ++w) {
    if (w == wv) {
#pragma unroll
      for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int ii = a * 16 + row_of(q), jj = b * 16 + i16;
            if (ii < ka && jj < kb) red[ii + jj * ka] += (double)acc[a][b][q];
          }
      if constexpr (SYM) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < TA; ++a)
#pragma unroll
          for (int a2 = a; a2 < TA; ++a2, ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int ii = a * 16 + row_of(q), jj = a2 * 16 + i16;
              if (ii < ka && jj < ka) {
                const double v = (double)accs[t][q];
                red[ii + (kb + jj) * ka] += v;
                if (a2 > a) red[jj + (kb + ii) * ka] += v;
              }
            }
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < ka * kt; e += 256) part[(int64_t)blockIdx.x * ka * kt + e] = red[e];
}

// Split-BF16 Gram: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); A^T B is
// approximated by hi^T hi + hi^T lo + lo^T hi on 16x16x32 BF16 matrix cores
// (lane l feeds rows 8*(l/16) .. +7 of column l%16).
__device__ inline __bf16 f2bf(float x) { return (__bf16)x; }

template <int TA, int TB>
__global__ __launch_bounds__(256) void k_gram_split_bf16(int64_t n, int ka, const float* __restrict__ A, int64_t lda,
                                                         int kb, const float* __restrict__ B, int64_t ldb,
                                                         int64_t rows_per_wave, double* __restrict__ part) {
  __shared__ double red[64 * 64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int i16 = lane & 15, k8 = lane >> 4;
  for (int e = threadIdx.x; e < ka * kb; e += 256) red[e] = 0.0;
  __syncthreads();
  const int64_t wid = (int64_t)blockIdx.x * 4 + wv;
  int64_t r0 = wid * rows_per_wave;
  int64_t r1 = r0 + rows_per_wave;
  if (r1 > n) r1 = n;
  f32x4 acc[TA][TB];
#pragma unroll
  for (int a = 0; a < TA; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t r = r0; r < r1; r += 32) {
    bf16x8 ah[TA], al[TA], bh[TB], bl[TB];
#pragma unroll
    for (int a = 0; a < TA; ++a) {
      int col = a * 16 + i16;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        int64_t row = r + 8 * k8 + q;
        float x = (row < r1 && col < ka) ? A[row * lda + col] : 0.f;
        __bf16 h = f2bf(x);
        ah[a][q] = h;
        al[a][q] = f2bf(x - (float)h);
      }
    }
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      int col = b * 16 + i16;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        int64_t row = r + 8 * k8 + q;
        float x = (row < r1 && col < kb) ? B[row * ldb + col] : 0.f;
        __bf16 h = f2bf(x);
        bh[b][q] = h;
        bl[b][q] = f2bf(x - (float)h);
      }
    }
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
      for (int b = 0; b < TB; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
      }
  }
  for (int w = 0; w < 4; ++w) {
    if (w == wv) {
#pragma unroll
      for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            int ii = a * 16 + 4 * k8 + q, jj = b * 16 + i16;
            if (ii < ka && jj < kb) red[ii + jj * ka] += (double)acc[a][b][q];
          }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < ka * kb; e += 256) part[(int64_t)blockIdx.x * ka * kb + e] = red[e];
}

template <typename T, bool F64MMA, int TA, int TB, bool SYM, bool PL>
hyeig_status gram_launch(hyeig_ctx* ctx, int64_t n, int ka, const T* A, int64_t lda, int kb, const T* B, int64_t ldb,
                         int64_t bs, double* part, int nblk, int64_t rpw) {
  const size_t lds = (size_t)ka * (SYM ? kb + ka : kb) * sizeof(double);
  hipLaunchKernelGGL((k_gram<T, F64MMA, TA, TB, SYM, PL>), dim3(nblk), dim3(256), lds, ctx->stream, n, ka, A, lda, kb,
                     B, ldb, bs, bs, rpw, part);
  return hip_err(ctx, hipGetLastError(), "k_gram launch");
}

template <typename T, bool F64MMA>
hyeig_status gram_dispatch(hyeig_ctx* ctx, int64_t n, int ka, const T* A, int64_t lda, int kb, const T* B,
                           int64_t ldb, bool sym, int64_t bs, double* part, int nblk, int64_t rpw) {
  const int ta = (ka + 15) / 16, tb = (kb + 15) / 16;
  if (bs > 0) {
    // 16-column blocks stored apart (the solver's [X W P] for n_b = 16): the
    // Rayleigh-Ritz pair over all three blocks, and [X W]^T [X, [X W]] for the
    // orthonormalisation of W in the FP32 forms
    if (ta == 3 && tb == 3 && sym && lda == 16 && ldb == 16)
      return gram_launch<T, F64MMA, 3, 3, true, true>(ctx, n, ka, A, lda, kb, B, ldb, bs, part, nblk, rpw);
    if (ta == 2 && tb == 1 && sym && lda == 16 && ldb == 16)
      return gram_launch<T, F64MMA, 2, 1, true, true>(ctx, n, ka, A, lda, kb, B, ldb, bs, part, nblk, rpw);
    return set_err(ctx, HYEIG_EUNSUPPORTED, "gram: block-strided operands only for the 48- and 32-column pairs");
  }
#define GD(x, y)                                                                                              \
  if (ta == x && tb == y)                                                                                     \
    return sym ? gram_launch<T, F64MMA, x, y, true, false>(ctx, n, ka, A, lda, kb, B, ldb, 0, part, nblk, rpw)  \
               : gram_launch<T, F64MMA, x, y, false, false>(ctx, n, ka, A, lda, kb, B, ldb, 0, part, nblk, rpw);
  GD(1, 1) GD(1, 2) GD(1, 3) GD(1, 4) GD(2, 1) GD(2, 2) GD(2, 3) GD(2, 4)
  GD(3, 1) GD(3, 2) GD(3, 3) GD(3, 4) GD(4, 1) GD(4, 2) GD(4, 3) GD(4, 4)
#undef GD
  return set_err(ctx, HYEIG_EUNSUPPORTED, "gram: unsupported widths");
}

hyeig_status gram_split_dispatch(hyeig_ctx* ctx, int64_t n, int ka, const float* A, int64_t lda, int kb,
                                 const float* B, int64_t ldb, double* part, int nblk, int64_t rpw) {
  int ta = (ka + 15) / 16, tb = (kb + 15) / 16;
#define GS(x, y)                                                                                                   \
  if (ta == x && tb == y) {                                                                                        \
    hipLaunchKernelGGL((k_gram_split_bf16<x, y>), dim3(nblk), dim3(256), 0, ctx->stream, n, ka, A, lda, kb, B, ldb, \
                       rpw, part);                                                                                 \
    return hip_err(ctx, hipGetLastError(), "k_gram_split_bf16 launch");                                            \
  }
  GS(1, 1) GS(1, 2) GS(1, 3) GS(1, 4) GS(2, 1) GS(2, 2) GS(2, 3) GS(2, 4)
  GS(3, 1) GS(3, 2) GS(3, 3) GS(3, 4) GS(4, 1) GS(4, 2) GS(4, 3) GS(4, 4)
#undef GS
  return set_err(ctx, HYEIG_EUNSUPPORTED, "gram: widths above 64");
}

// ---------------------------------------------------------------------------
// block update on matrix cores: Y1 = alpha S C1 + beta Y1, optionally Y2 = S C2,
// with S n x k row-major and C k x m column-major FP64.  A wave forms 16 rows at
// a time with 16x16x4 MFMAs.  Lane group g = lane / 16 owns the contiguous
// slice [g KG, g KG + KG) of the inner index (MFMA step s takes k = g KG + s),
// so a lane's A operands are KG consecutive elements of one row of S (16-byte
// loads when the rows allow) and the 16 rows of a step are one contiguous
// span of S.  The coefficients a lane needs (k = g KG + s, column 16 cb + lane
// % 16) are loaded once per wave and stay in registers.
// ---------------------------------------------------------------------------
template <typename T, int KG, int NCB, bool VEC, bool TWO>
__global__ __launch_bounds__(256) void k_update(int64_t n, int k, int m, const T* __restrict__ S, int64_t lds,
                                                int64_t bss, const double* __restrict__ C1, double alpha, double beta,
                                                T* Y1, int64_t ld1, const double* __restrict__ C2, T* Y2, int64_t ld2,
                                                int yvec) {
  using VT4 = typename std::conditional<std::is_same<T, double>::value, f64x4, f32x4>::type;
  constexpr bool F64 = std::is_same<T, double>::value;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, i = lane & 15;
  T b1[NCB][KG], b2[NCB][KG];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int q = 0; q < KG; ++q) {
      const int kk = g * KG + q, j = cb * 16 + i;
      const bool ok = kk < k && j < m;
      b1[cb][q] = ok ? (T)C1[kk + (int64_t)j * k] : (T)0;
      if constexpr (TWO) b2[cb][q] = ok ? (T)C2[kk + (int64_t)j * k] : (T)0;
    }
  const int64_t ntiles = (n + 15) / 16;
  const int64_t wstride = (int64_t)gridDim.x * 4;
  // element kk of a row of S: at kk (one row-major array) or, with bss > 0, in
  // the n x 16 block kk / 16 stored bss elements after the previous one
  constexpr int EPC = VEC ? 16 / (int)sizeof(T) : 1;
  int64_t koff[KG / EPC];
#pragma unroll
  for (int q = 0; q < KG / EPC; ++q) {
    const int64_t kk = g * KG + q * EPC;
    koff[q] = bss > 0 ? (kk >> 4) * bss + (kk & 15) : kk;
  }
  // the KG elements of row t * 16 + i that lane group g contributes
  auto load = [&](int64_t t, T(&av)[KG]) {
    const int64_t row = t * 16 + i;
    const T* sr = S + row * lds;
    if constexpr (VEC) {
#pragma unroll
      for (int q = 0; q < KG / EPC; ++q) {
        uint4 u = make_uint4(0, 0, 0, 0);
        if (row < n) u = *reinterpret_cast<const uint4*>(sr + koff[q]);
        const T* e = reinterpret_cast<const T*>(&u);
#pragma unroll
        for (int w = 0; w < EPC; ++w) av[q * EPC + w] = e[w];
      }
    } else {
#pragma unroll
      for (int q = 0; q < KG; ++q) av[q] = (row < n && g * KG + q < k) ? sr[koff[q]] : (T)0;
    }
  };
  int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  T av[KG];
  load(t, av);
  for (; t < ntiles; t += wstride) {
    // the next tile's rows are requested before this tile's products (the last
    // request repeats the final tile and is not used)
    T an[KG];
    load(t + wstride < ntiles ? t + wstride : ntiles - 1, an);
    VT4 acc1[NCB], acc2[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      acc1[cb] = VT4{0, 0, 0, 0};
      acc2[cb] = VT4{0, 0, 0, 0};
    }
#pragma unroll
    for (int q = 0; q < KG; ++q)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        if constexpr (F64) {
          acc1[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], b1[cb][q], acc1[cb], 0, 0, 0);
          if constexpr (TWO) acc2[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], b2[cb][q], acc2[cb], 0, 0, 0);
        } else {
          // FP32: the transposed product C^T S^T, so that lane l ends with
          // columns 4 (l / 16) .. + 3 of row l % 16 (one 16-byte store)
          acc1[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b1[cb][q], av[q], acc1[cb], 0, 0, 0);
          if constexpr (TWO) acc2[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b2[cb][q], av[q], acc2[cb], 0, 0, 0);
        }
      }
    if constexpr (F64) {
      // element q of lane l: row 4 q + l / 16, column l % 16
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int j = cb * 16 + i;
        if (j >= m) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t r = t * 16 + 4 * q + g;
          if (r >= n) continue;
          T y = (T)alpha * acc1[cb][q];
          if (beta != 0.0) y += (T)beta * Y1[r * ld1 + j];
          Y1[r * ld1 + j] = y;
          if constexpr (TWO) Y2[r * ld2 + j] = acc2[cb][q];
        }
      }
    } else {
      // element q of lane l: row l % 16, column 4 (l / 16) + q
      const int64_t r = t * 16 + i;
      if (r < n) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const int j0 = cb * 16 + 4 * g;
          float4 y = make_float4(acc1[cb][0], acc1[cb][1], acc1[cb][2], acc1[cb][3]);
          y.x *= (float)alpha;
          y.y *= (float)alpha;
          y.z *= (float)alpha;
          y.w *= (float)alpha;
          if (yvec && j0 + 3 < m) {
            float4* yp = reinterpret_cast<float4*>(Y1 + r * ld1 + j0);
            if (beta != 0.0) {
              const float4 o = *yp;
              y.x += (float)beta * o.x;
              y.y += (float)beta * o.y;
              y.z += (float)beta * o.z;
              y.w += (float)beta * o.w;
            }
            *yp = y;
            if constexpr (TWO)
              *reinterpret_cast<float4*>(Y2 + r * ld2 + j0) =
                  make_float4(acc2[cb][0], acc2[cb][1], acc2[cb][2], acc2[cb][3]);
          } else {
            const float yv[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int j = j0 + q;
              if (j >= m) continue;
              float v = yv[q];
              if (beta != 0.0) v += (float)beta * Y1[r * ld1 + j];
              Y1[r * ld1 + j] = v;
              if constexpr (TWO) Y2[r * ld2 + j] = acc2[cb][q];
            }
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < KG; ++q) av[q] = an[q];
  }
}

template <typename T, int KG, int NCB, bool VEC, bool TWO>
hyeig_status update_launch(hyeig_ctx* ctx, int64_t n, int k, int m, const T* S, int64_t lds, int64_t bss, const double* C1,
                           double alpha, double beta, T* Y1, int64_t ld1, const double* C2, T* Y2, int64_t ld2) {
  const int64_t ntiles = (n + 15) / 16;
  int64_t blocks = (ntiles + 3) / 4;
  // as many workgroups as stay resident: the grid-stride loop gives every wave
  // the same number of tiles, so a second round of waves would run at low occupancy
  static const int per_cu = [] {
    int b = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void*)k_update<T, KG, NCB, VEC, TWO>, 256, 0) ==
                       hipSuccess &&
                   b > 0
               ? b
               : 2;
  }();
  const int64_t maxb = (int64_t)ctx->num_cu * per_cu;
  if (blocks > maxb) blocks = maxb;
  // 16-byte rows of Y (FP32): both outputs 16-byte aligned with ld % 4 == 0
  const bool yvec = ((uintptr_t)Y1 & 15) == 0 && ld1 % 4 == 0 && (!TWO || (((uintptr_t)Y2 & 15) == 0 && ld2 % 4 == 0));
  hipLaunchKernelGGL((k_update<T, KG, NCB, VEC, TWO>), dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, k, m, S,
                     lds, bss, C1, alpha, beta, Y1, ld1, C2, Y2, ld2, (int)yvec);
  return hip_err(ctx, hipGetLastError(), "k_update launch");
}

template <typename T, int KG, int NCB, bool TWO>
hyeig_status update_vec(hyeig_ctx* ctx, int64_t n, int k, int m, const T* S, int64_t lds, int64_t bss, const double* C1,
                        double alpha, double beta, T* Y1, int64_t ld1, const double* C2, T* Y2, int64_t ld2) {
  constexpr int EPC = 16 / (int)sizeof(T);
  if constexpr (KG % EPC == 0) {
    const bool vec = k == 4 * KG && (lds % EPC) == 0 && (bss % EPC) == 0 && ((uintptr_t)S & 15) == 0;
    if (vec)
      return update_launch<T, KG, NCB, true, TWO>(ctx, n, k, m, S, lds, bss, C1, alpha, beta, Y1, ld1, C2, Y2, ld2);
  }
  return update_launch<T, KG, NCB, false, TWO>(ctx, n, k, m, S, lds, bss, C1, alpha, beta, Y1, ld1, C2, Y2, ld2);
}

template <typename T, bool TWO>
hyeig_status update_dispatch(hyeig_ctx* ctx, int64_t n, int k, int m, const T* S, int64_t lds, int64_t bss, const double* C1,
                             double alpha, double beta, T* Y1, int64_t ld1, const double* C2, T* Y2, int64_t ld2) {
  const int kg = (k + 3) / 4;
#define UD(KG, NCB)                                                                                             \
  if (kg <= KG && (m + 15) / 16 == NCB)                                                                         \
    return update_vec<T, KG, NCB, TWO>(ctx, n, k, m, S, lds, bss, C1, alpha, beta, Y1, ld1, C2, Y2, ld2);
  UD(1, 1) UD(2, 1) UD(3, 1) UD(4, 1) UD(6, 1) UD(8, 1) UD(12, 1) UD(16, 1)
  UD(1, 2) UD(2, 2) UD(3, 2) UD(4, 2) UD(6, 2) UD(8, 2) UD(12, 2) UD(16, 2)
#undef UD
  return set_err(ctx, HYEIG_EUNSUPPORTED, "block_update: k > 64 or m > 32");
}

// ---------------------------------------------------------------------------
// The two LOBPCG updates of an iteration and the residual pass that opens the
// next one, in one sweep over the rows (nb <= 16 columns):
//   [X' P'] = S [C1 C2],  [HX' HP'] = HS [C1 C2]      (k_update's MFMA scheme)
// and from X', HX' as stored, the residual pass of k_resid_precond:
//   R = HX' - X' Theta (FP64, rounded to T),  part += R^2 per column,
//   W[:, pos[j]] = R[:, j] / max(|d - theta_j|, floor) (R if d is null),
//   columns na .. nb-1 of W cleared.
// A 16-row tile's S and HS rows are all requested before its products (no
// prefetch across tiles: the registers go to the two row sets, and the
// resident waves keep enough loads in flight); S and HS are read once and X',
// HX' are not read back.  The grid is resident (grid-stride over tiles); each
// workgroup writes one FP64 partial per column.
// ---------------------------------------------------------------------------
template <typename T, int KG, bool VEC>
__global__ __launch_bounds__(256) void k_update_resid(int64_t n, int k, int nb, const T* __restrict__ S,
                                                      const T* __restrict__ HS, int64_t lds, int64_t bss,
                                                      const double* __restrict__ C1, const double* __restrict__ C2,
                                                      T* X1, T* P1, T* HX1, T* HP1, int64_t ldy,
                                                      const double* __restrict__ theta, const float* __restrict__ d,
                                                      double floor, const int* __restrict__ pos, int na, T* W,
                                                      int64_t ldw, double* __restrict__ part) {
  using VT4 = typename std::conditional<std::is_same<T, double>::value, f64x4, f32x4>::type;
  constexpr bool F64 = std::is_same<T, double>::value;
  constexpr int RC = F64 ? 1 : 4;  // residual columns per lane
  __shared__ double red[4][64][RC];
  // the coefficients in LDS (element (kk, column i) at kk * 16 + i), read next
  // to their MFMAs: held in registers they would leave room for two waves per SIMD only
  __shared__ T cf[2][4 * KG * 16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, i = lane & 15;
  for (int e = threadIdx.x; e < 4 * KG * 16; e += 256) {
    const int kk = e >> 4, c = e & 15;
    const bool ok = kk < k && c < nb;
    cf[0][e] = ok ? (T)C1[kk + (int64_t)c * k] : (T)0;
    cf[1][e] = ok ? (T)C2[kk + (int64_t)c * k] : (T)0;
  }
  __syncthreads();
  // this lane's residual columns: i (FP64 layout) or 4 g .. 4 g + 3 (FP32)
  double th[RC], ss[RC];
  int pj[RC], jc[RC];
#pragma unroll
  for (int c = 0; c < RC; ++c) {
    jc[c] = F64 ? i : 4 * g + c;
    th[c] = jc[c] < nb ? theta[jc[c]] : 0.0;
    pj[c] = jc[c] < nb ? pos[jc[c]] : -1;
    ss[c] = 0.0;
  }
  const int64_t ntiles = (n + 15) / 16;
  const int64_t wstride = (int64_t)gridDim.x * 4;
  constexpr int EPC = VEC ? 16 / (int)sizeof(T) : 1;
  int64_t koff[KG / EPC];
#pragma unroll
  for (int q = 0; q < KG / EPC; ++q) {
    const int64_t kk = g * KG + q * EPC;
    koff[q] = bss > 0 ? (kk >> 4) * bss + (kk & 15) : kk;
  }
  auto load = [&](const T* __restrict__ A, int64_t t, T(&av)[KG]) {
    const int64_t row = t * 16 + i;
    const T* sr = A + row * lds;
    if constexpr (VEC) {
#pragma unroll
      for (int q = 0; q < KG / EPC; ++q) {
        uint4 u = make_uint4(0, 0, 0, 0);
        if (row < n) u = *reinterpret_cast<const uint4*>(sr + koff[q]);
        const T* e = reinterpret_cast<const T*>(&u);
#pragma unroll
        for (int w = 0; w < EPC; ++w) av[q * EPC + w] = e[w];
      }
    } else {
#pragma unroll
      for (int q = 0; q < KG; ++q) av[q] = (row < n && g * KG + q < k) ? sr[koff[q]] : (T)0;
    }
  };
  auto products = [&](const T(&av)[KG], VT4& a1, VT4& a2) {
    a1 = VT4{0, 0, 0, 0};
    a2 = VT4{0, 0, 0, 0};
    // (an index the compiler cannot see through, so the reads stay in the loop)
    int cb = g * KG * 16 + i;
    asm volatile("" : "+v"(cb));
#pragma unroll
    for (int q = 0; q < KG; ++q) {
      const T b1 = cf[0][cb + q * 16], b2 = cf[1][cb + q * 16];
      if constexpr (F64) {
        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], b1, a1, 0, 0, 0);
        a2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], b2, a2, 0, 0, 0);
      } else {
        a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(b1, av[q], a1, 0, 0, 0);
        a2 = __builtin_amdgcn_mfma_f32_16x16x4f32(b2, av[q], a2, 0, 0, 0);
      }
    }
  };
  // element e of a lane's accumulator: FP64 row 4 e + g, column i; FP32 row i,
  // column 4 g + e (16-byte rows: ldy % 4 == 0, aligned, checked by the host)
  auto store = [&](int64_t t, const VT4& a1, const VT4& a2, T* Y1, T* Y2) {
    if constexpr (F64) {
      if (i < nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t r = t * 16 + 4 * e + g;
          if (r < n) {
            Y1[r * ldy + i] = a1[e];
            Y2[r * ldy + i] = a2[e];
          }
        }
    } else {
      const int64_t r = t * 16 + i;
      if (r < n && 4 * g + 3 < nb) {
        *reinterpret_cast<float4*>(Y1 + r * ldy + 4 * g) = make_float4(a1[0], a1[1], a1[2], a1[3]);
        *reinterpret_cast<float4*>(Y2 + r * ldy + 4 * g) = make_float4(a2[0], a2[1], a2[2], a2[3]);
      } else if (r < n) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (4 * g + e < nb) {
            Y1[r * ldy + 4 * g + e] = a1[e];
            Y2[r * ldy + 4 * g + e] = a2[e];
          }
      }
    }
  };
  for (int64_t t = (int64_t)blockIdx.x * 4 + wv; t < ntiles; t += wstride) {
    {
      T av[KG], ah[KG];
      load(S, t, av);
      load(HS, t, ah);
      VT4 a1, a2;
      products(av, a1, a2);
      store(t, a1, a2, X1, P1);
      VT4 h1, h2;
      products(ah, h1, h2);
      store(t, h1, h2, HX1, HP1);
      // the residual pass on this tile's stored X' and HX'
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = F64 ? t * 16 + 4 * e + g : t * 16 + i;
        const int c = F64 ? 0 : e;
        if (r >= n || jc[c] >= nb) continue;
        const double x = (double)(T)a1[e], hx = (double)(T)h1[e];
        const T rt = (T)(hx - th[c] * x);
        ss[c] += (double)rt * (double)rt;
        T* wr = W + r * ldw;
        if (pj[c] >= 0) {
          double w = (double)rt;
          if (d) {
            const double den = fabs((double)d[r] - th[c]);
            w = w / (den > floor ? den : floor);
          }
          wr[pj[c]] = (T)w;
        }
        if (jc[c] >= na) wr[jc[c]] = (T)0;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < RC; ++c) red[wv][lane][c] = ss[c];
  __syncthreads();
  if (threadIdx.x < nb) {
    // column j: lanes 16 q + j (FP64 layout) or entry j % 4 of lanes 16 (j / 4) + i (FP32)
    const int j = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < 4; ++w) {
      if constexpr (F64) {
        for (int q = 0; q < 4; ++q) s += red[w][16 * q + j][0];
      } else {
        for (int r = 0; r < 16; ++r) s += red[w][16 * (j >> 2) + r][j & 3];
      }
    }
    part[(int64_t)blockIdx.x * nb + j] = s;
  }
}

template <typename T, int KG, bool VEC>
hyeig_status update_resid_launch(hyeig_ctx* ctx, int64_t n, int k, int nb, const T* S, const T* HS, int64_t lds,
                                 int64_t bss, const double* C1, const double* C2, T* X1, T* P1, T* HX1, T* HP1,
                                 int64_t ldy, const double* theta, const float* d, double floor, const int* pos, int na,
                                 T* W, int64_t ldw, double* part, int* nblk) {
  const int64_t ntiles = (n + 15) / 16;
  int64_t blocks = (ntiles + 3) / 4;
  static const int per_cu = [] {
    int b = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void*)k_update_resid<T, KG, VEC>, 256, 0) ==
                       hipSuccess &&
                   b > 0
               ? b
               : 2;
  }();
  const int64_t maxb = (int64_t)ctx->num_cu * std::min(per_cu, 8);
  if (blocks > maxb) blocks = maxb;
  *nblk = (int)blocks;
  hipLaunchKernelGGL((k_update_resid<T, KG, VEC>), dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, k, nb, S, HS,
                     lds, bss, C1, C2, X1, P1, HX1, HP1, ldy, theta, d, floor, pos, na, W, ldw, part);
  return hip_err(ctx, hipGetLastError(), "k_update_resid launch");
}

template <typename T>
hyeig_status update_resid_dispatch(hyeig_ctx* ctx, int64_t n, int k, int nb, const T* S, const T* HS, int64_t lds,
                                   int64_t bss, const double* C1, const double* C2, T* X1, T* P1, T* HX1, T* HP1,
                                   int64_t ldy, const double* theta, const float* d, double floor, const int* pos,
                                   int na, T* W, int64_t ldw, double* part, int* nblk) {
  constexpr int EPC = 16 / (int)sizeof(T);
  const int kg = (k + 3) / 4;
  const bool vec = (lds % EPC) == 0 && (bss % EPC) == 0 && ((uintptr_t)S & 15) == 0 && ((uintptr_t)HS & 15) == 0;
#define UR(KG)                                                                                                    \
  if (kg <= KG) {                                                                                                 \
    if constexpr (KG % EPC == 0) {                                                                                \
      if (vec && k == 4 * KG)                                                                                     \
        return update_resid_launch<T, KG, true>(ctx, n, k, nb, S, HS, lds, bss, C1, C2, X1, P1, HX1, HP1, ldy,    \
                                                theta, d, floor, pos, na, W, ldw, part, nblk);                    \
    }                                                                                                             \
    return update_resid_launch<T, KG, false>(ctx, n, k, nb, S, HS, lds, bss, C1, C2, X1, P1, HX1, HP1, ldy, theta, \
                                             d, floor, pos, na, W, ldw, part, nblk);                              \
  }
  UR(1) UR(2) UR(3) UR(4) UR(6) UR(8) UR(12)
#undef UR
  return set_err(ctx, HYEIG_EUNSUPPORTED, "update_resid: k > 48");
}

// ---------------------------------------------------------------------------
// residual + shifted-diagonal preconditioner.  Thread (row, j), j < nb:
//   r = HX[row, j] - theta[j] X[row, j];  norms2[j] += r^2
//   pos[j] >= 0:  W[row, pos[j]] = r / max(|d[row] - theta[j]|, floor)  (r if d == null)
//   columns na .. wcols_total-1 of W are cleared.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_resid_precond(int64_t n, int nb, const T* __restrict__ X, int64_t ldx,
                                                       const T* __restrict__ HX, int64_t ldhx,
                                                       const double* __restrict__ theta, const float* __restrict__ d,
                                                       double floor, const int* __restrict__ pos, int na, T* W,
                                                       int64_t ldw, int wtot, double* __restrict__ part,
                                                       const int* __restrict__ guard) {
  if (guard && *guard == 0) return;  // uniform over the grid, before any barrier
  __shared__ double red[8][33];
  const int j = threadIdx.x, ty = threadIdx.y;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 8 + ty; i < n; i += (int64_t)gridDim.x * 8) {
    if (j < nb) {
      double th = theta[j];
      double r = (double)HX[i * ldhx + j] - th * (double)X[i * ldx + j];
      T rt = (T)r;
      s += (double)rt * (double)rt;
      int p = pos[j];
      if (p >= 0) {
        double w = (double)rt;
        if (d) {
          double den = fabs((double)d[i] - th);
          w = w / (den > floor ? den : floor);
        }
        W[i * ldw + p] = (T)w;
      }
    }
    if (j >= na && j < wtot) W[i * ldw + j] = (T)0;
  }
  red[ty][j] = s;
  __syncthreads();
  if (ty == 0 && j < nb) {
    double t = 0.0;
    for (int q = 0; q < 8; ++q) t += red[q][j];
    part[(int64_t)blockIdx.x * nb + j] = t;
  }
}

// The same for blocks whose rows start on 16-byte boundaries and whose nb fills
// whole 16-byte pieces (nb % 4 == 0 in FP32, nb % 2 == 0 in FP64): thread
// (row, g) takes columns VW g .. VW g + VW - 1 (VW = 16 bytes / sizeof(T)) with
// 16-byte loads of X and HX, nb / VW threads per row, two rows in flight per
// thread.  The residual is formed in FP64 as above (HX - theta X cancels near
// convergence).
template <typename T>
struct alignas(16) Piece16 {
  static constexpr int VW = 16 / (int)sizeof(T);
  T v[VW];
};

template <typename T>
__global__ __launch_bounds__(256) void k_resid_precond_v(int64_t n, int nb, const T* __restrict__ X, int64_t ldx,
                                                         const T* __restrict__ HX, int64_t ldhx,
                                                         const double* __restrict__ theta,
                                                         const float* __restrict__ d, double floor,
                                                         const int* __restrict__ pos, int na, T* W, int64_t ldw,
                                                         int wtot, double* __restrict__ part,
                                                         const int* __restrict__ guard) {
  constexpr int VW = Piece16<T>::VW;
  if (guard && *guard == 0) return;  // uniform over the grid, before any barrier
  __shared__ double red[256][VW];
  const int tpr = nb / VW;     // threads per row
  const int rpb = 256 / tpr;   // rows per block step
  const int g = threadIdx.x % tpr, rl = threadIdx.x / tpr;
  const bool live = rl < rpb;
  double th[VW];
  int pj[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) {
    th[q] = theta[VW * g + q];
    pj[q] = pos[VW * g + q];
  }
  double s[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) s[q] = 0.0;
  auto row_out = [&](int64_t i, const Piece16<T>& x, const Piece16<T>& h) {
    const double di = d ? (double)d[i] : 0.0;
    T* wr = W + i * ldw;
#pragma unroll
    for (int q = 0; q < VW; ++q) {
      const double r = (double)h.v[q] - th[q] * (double)x.v[q];
      const T rt = (T)r;
      s[q] += (double)rt * (double)rt;
      if (pj[q] >= 0) {
        double w = (double)rt;
        if (d) {
          const double den = fabs(di - th[q]);
          w = w / (den > floor ? den : floor);
        }
        wr[pj[q]] = (T)w;
      }
      const int j = VW * g + q;
      if (j >= na && j < wtot) wr[j] = (T)0;
    }
    for (int j = nb + g; j < wtot; j += tpr) wr[j] = (T)0;
  };
  auto load = [](const T* p) { return *reinterpret_cast<const Piece16<T>*>(p); };
  if (live) {
    const int64_t step = (int64_t)gridDim.x * rpb;
    int64_t i = (int64_t)blockIdx.x * rpb + rl;
    for (; i + step < n; i += 2 * step) {
      const Piece16<T> x0 = load(X + i * ldx + VW * g);
      const Piece16<T> h0 = load(HX + i * ldhx + VW * g);
      const Piece16<T> x1 = load(X + (i + step) * ldx + VW * g);
      const Piece16<T> h1 = load(HX + (i + step) * ldhx + VW * g);
      row_out(i, x0, h0);
      row_out(i + step, x1, h1);
    }
    if (i < n) {
      const Piece16<T> x0 = load(X + i * ldx + VW * g);
      const Piece16<T> h0 = load(HX + i * ldhx + VW * g);
      row_out(i, x0, h0);
    }
  }
#pragma unroll
  for (int q = 0; q < VW; ++q) red[threadIdx.x][q] = live ? s[q] : 0.0;
  __syncthreads();
  if (threadIdx.x < nb) {
    const int gg = threadIdx.x / VW, q = threadIdx.x % VW;
    double t = 0.0;
    for (int r = 0; r < rpb; ++r) t += red[r * tpr + gg][q];
    part[(int64_t)blockIdx.x * nb + threadIdx.x] = t;
  }
}

int reduce_blocks(int64_t n) {
  int64_t b = (n + 7) / 8;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

}  // namespace

hyeig_status reduce_cols(hyeig_ctx* ctx, int nblk, int ncols, const double* part, double* out) {
  dim3 blk(64, 4);
  dim3 grd((ncols + 3) / 4);
  hipLaunchKernelGGL(k_reduce_cols, grd, blk, 0, ctx->stream, nblk, ncols, part, out);
  return hip_err(ctx, hipGetLastError(), "k_reduce_cols launch");
}

// row-wise element kernels: min(m, 32) lanes across a row and 256 / that many
// rows per workgroup, so that narrow blocks leave no lane idle
static dim3 row_block(int m) {
  const int x = m < 32 ? (m < 1 ? 1 : m) : 32;
  return dim3(x, 256 / x);
}
static dim3 row_grid(int64_t n, dim3 blk) { return dim3((unsigned)((n + blk.y - 1) / blk.y)); }

hyeig_status launch_fill(hyeig_ctx* ctx, int64_t n, int m, void* Y, int64_t ld, hyeig_dtype dt, double value) {
  if (n <= 0 || m <= 0) return HYEIG_OK;
  const dim3 blk = row_block(m), grd = row_grid(n, blk);
  if (dt == HYEIG_F64)
    hipLaunchKernelGGL(k_fill<double>, grd, blk, 0, ctx->stream, n, m, (double*)Y, ld, value);
  else
    hipLaunchKernelGGL(k_fill<float>, grd, blk, 0, ctx->stream, n, m, (float*)Y, ld, (float)value);
  return hip_err(ctx, hipGetLastError(), "k_fill launch");
}

hyeig_status launch_fill_hash(hyeig_ctx* ctx, int64_t n, int m, void* Y, int64_t ld, hyeig_dtype dt, uint64_t seed) {
  if (n <= 0 || m <= 0) return HYEIG_OK;
  const dim3 blk = row_block(m), grd = row_grid(n, blk);
  if (dt == HYEIG_F64)
    hipLaunchKernelGGL(k_fill_hash<double>, grd, blk, 0, ctx->stream, n, m, (double*)Y, ld, seed);
  else
    hipLaunchKernelGGL(k_fill_hash<float>, grd, blk, 0, ctx->stream, n, m, (float*)Y, ld, seed);
  return hip_err(ctx, hipGetLastError(), "k_fill_hash launch");
}

hyeig_status launch_copy(hyeig_ctx* ctx, int64_t n, int m, const void* X, int64_t ldx, hyeig_dtype xdt, void* Y,
                         int64_t ldy, hyeig_dtype ydt) {
  if (n <= 0 || m <= 0) return HYEIG_OK;
  const dim3 blk = row_block(m), grd = row_grid(n, blk);
  if (xdt == HYEIG_F32 && ydt == HYEIG_F32)
    hipLaunchKernelGGL((k_copy<float, float>), grd, blk, 0, ctx->stream, n, m, (const float*)X, ldx, (float*)Y, ldy);
  else if (xdt == HYEIG_F32 && ydt == HYEIG_F64)
    hipLaunchKernelGGL((k_copy<float, double>), grd, blk, 0, ctx->stream, n, m, (const float*)X, ldx, (double*)Y,
                       ldy);
  else if (xdt == HYEIG_F64 && ydt == HYEIG_F32)
    hipLaunchKernelGGL((k_copy<double, float>), grd, blk, 0, ctx->stream, n, m, (const double*)X, ldx, (float*)Y,
                       ldy);
  else
    hipLaunchKernelGGL((k_copy<double, double>), grd, blk, 0, ctx->stream, n, m, (const double*)X, ldx, (double*)Y,
                       ldy);
  return hip_err(ctx, hipGetLastError(), "k_copy launch");
}

hyeig_status launch_gather_pad(hyeig_ctx* ctx, int64_t n, int m, int mp, const void* X, int64_t ldx, void* Y,
                               hyeig_dtype dt) {
  if (n <= 0) return HYEIG_OK;
  int64_t blocks = (n * mp + 255) / 256;
  const int64_t maxb = (int64_t)ctx->num_cu * 16;
  if (blocks > maxb) blocks = maxb;
  if (dt == HYEIG_F64)
    hipLaunchKernelGGL(k_gather_pad<double>, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, m, mp,
                       (const double*)X, ldx, (double*)Y);
  else
    hipLaunchKernelGGL(k_gather_pad<float>, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, m, mp,
                       (const float*)X, ldx, (float*)Y);
  return hip_err(ctx, hipGetLastError(), "k_gather_pad launch");
}

hyeig_status launch_lincomb(hyeig_ctx* ctx, int64_t n, int m, double a, const void* A, int64_t lda, double b,
                            const void* B, int64_t ldb, double g, const void* C, int64_t ldc, void* Y, int64_t ldy,
                            hyeig_dtype dt) {
  if (n <= 0 || m <= 0) return HYEIG_OK;
  if (m > 32) return set_err(ctx, HYEIG_EUNSUPPORTED, "lincomb: more than 32 columns");
  const dim3 blk = row_block(m), grd = row_grid(n, blk);
  if (dt == HYEIG_F64)
    hipLaunchKernelGGL(k_lincomb<double>, grd, blk, 0, ctx->stream, n, m, a, (const double*)A, lda, b,
                       (const double*)B, ldb, g, (const double*)C, ldc, (double*)Y, ldy);
  else
    hipLaunchKernelGGL(k_lincomb<float>, grd, blk, 0, ctx->stream, n, m, a, (const float*)A, lda, b,
                       (const float*)B, ldb, g, (const float*)C, ldc, (float*)Y, ldy);
  return hip_err(ctx, hipGetLastError(), "k_lincomb launch");
}

hyeig_status launch_gather_cols(hyeig_ctx* ctx, int64_t n, int m, const int* idx, const void* X, int64_t ldx,
                                void* Y, int64_t ldy, hyeig_dtype dt) {
  if (n <= 0 || m <= 0) return HYEIG_OK;
  if (m > 32) return set_err(ctx, HYEIG_EUNSUPPORTED, "gather_cols: more than 32 columns");
  const dim3 blk = row_block(m), grd = row_grid(n, blk);
  if (dt == HYEIG_F64)
    hipLaunchKernelGGL(k_gather_cols<double>, grd, blk, 0, ctx->stream, n, m, idx, (const double*)X, ldx,
                       (double*)Y, ldy);
  else
    hipLaunchKernelGGL(k_gather_cols<float>, grd, blk, 0, ctx->stream, n, m, idx, (const float*)X, ldx,
                       (float*)Y, ldy);
  return hip_err(ctx, hipGetLastError(), "k_gather_cols launch");
}

hyeig_status launch_col_scale(hyeig_ctx* ctx, int64_t n, int m, void* Y, int64_t ld, const double* s,
                              hyeig_dtype dt) {
  if (n <= 0 || m <= 0) return HYEIG_OK;
  const dim3 blk = row_block(m), grd = row_grid(n, blk);
  if (dt == HYEIG_F64)
    hipLaunchKernelGGL(k_col_scale<double>, grd, blk, 0, ctx->stream, n, m, (double*)Y, ld, s);
  else
    hipLaunchKernelGGL(k_col_scale<float>, grd, blk, 0, ctx->stream, n, m, (float*)Y, ld, s);
  return hip_err(ctx, hipGetLastError(), "k_col_scale launch");
}

hyeig_status launch_col_dots(hyeig_ctx* ctx, int64_t n, int m, const void* A, int64_t lda, const void* B,
                             int64_t ldb, hyeig_dtype dt, double* dots) {
  if (m > 32) return set_err(ctx, HYEIG_EUNSUPPORTED, "col_dots: more than 32 columns");
  int nblk = reduce_blocks(n);
  hyeig_status st;
  double* part = (double*)ws_get(ctx, WS_REDUCE, (size_t)nblk * m * sizeof(double), &st);
  if (!part) return st;
  dim3 blk(32, 8);
  if (dt == HYEIG_F64)
    hipLaunchKernelGGL(k_col_dots<double>, dim3(nblk), blk, 0, ctx->stream, n, m, (const double*)A, lda,
                       (const double*)B, ldb, part);
  else
    hipLaunchKernelGGL(k_col_dots<float>, dim3(nblk), blk, 0, ctx->stream, n, m, (const float*)A, lda,
                       (const float*)B, ldb, part);
  HY_CHECK(hip_err(ctx, hipGetLastError(), "k_col_dots launch"));
  return reduce_cols(ctx, nblk, m, part, dots);
}

hyeig_status launch_gram2(hyeig_ctx* ctx, int64_t n, int ka, const void* A, int64_t lda, int kb1, const void* B1,
                          int64_t ldb1, int kb2, const void* B2, int64_t ldb2, hyeig_dtype dt, hyeig_mma_mode mode,
                          double* G, int64_t bs, double* fixed_part, int64_t fixed_cap) {
  // one pass for [A^T B1, A^T A] (the Rayleigh-Ritz pair); other pairs take two
  const bool sym = kb2 > 0 && B2 == A && ldb2 == lda && kb2 == ka && mode != HYEIG_MMA_SPLIT_BF16 &&
                   ka * (kb1 + ka) <= 6144;  // FP64 partial of the workgroup within 48 KB of LDS
  if (bs > 0 && !sym) return set_err(ctx, HYEIG_EUNSUPPORTED, "gram: block-strided operands need the fused pair");
  if (kb2 > 0 && !sym) {
    HY_CHECK(launch_gram2(ctx, n, ka, A, lda, kb1, B1, ldb1, 0, nullptr, 0, dt, mode, G, 0, fixed_part, fixed_cap));
    return launch_gram2(ctx, n, ka, A, lda, kb2, B2, ldb2, 0, nullptr, 0, dt, mode, G + (size_t)ka * kb1, 0,
                        fixed_part, fixed_cap);
  }
  const int kt = sym ? kb1 + ka : kb1;
  // rows per wave: enough workgroups to fill the chip (8 waves per CU), 16-row steps;
  // with a fixed partials buffer no more workgroups than it holds partials for
  int64_t waves = (n + 255) / 256;
  int64_t maxw = (int64_t)ctx->num_cu * 8;
  if (fixed_part) {
    const int64_t fit = 4 * (fixed_cap / ((int64_t)ka * kt));
    if (fit < 4) return set_err(ctx, HYEIG_EUNSUPPORTED, "gram: partials larger than the fixed buffer");
    if (maxw > fit) maxw = fit;
  }
  if (waves > maxw) waves = maxw;
  if (waves < 4) waves = 4;
  int64_t rpw = (n + waves - 1) / waves;
  rpw = (rpw + 31) / 32 * 32;
  // byte offsets inside a wave's rows are 32-bit
  const int64_t es = dt == HYEIG_F64 ? 8 : 4;
  if (rpw * (lda > ldb1 ? lda : ldb1) * es >= (int64_t)INT32_MAX)
    return set_err(ctx, HYEIG_EUNSUPPORTED, fixed_part ? "gram: n times the leading dimension too large for the "
                                                         "allocation-free form"
                                                       : "gram: leading dimension too large");
  int nblk = (int)((n + rpw * 4 - 1) / (rpw * 4));
  if (nblk < 1) nblk = 1;
  hyeig_status st;
  double* part = fixed_part;
  if (!part) part = (double*)ws_get(ctx, WS_GRAM, (size_t)nblk * ka * kt * sizeof(double), &st);
  if (!part) return st;
  if (mode == HYEIG_MMA_SPLIT_BF16) {
    HY_CHECK(gram_split_dispatch(ctx, n, ka, (const float*)A, lda, kb1, (const float*)B1, ldb1, part, nblk, rpw));
  } else if (mode == HYEIG_MMA_F64) {
    if (dt == HYEIG_F64)
      HY_CHECK((gram_dispatch<double, true>(ctx, n, ka, (const double*)A, lda, kb1, (const double*)B1, ldb1, sym,
                                            bs, part, nblk, rpw)));
    else
      HY_CHECK((gram_dispatch<float, true>(ctx, n, ka, (const float*)A, lda, kb1, (const float*)B1, ldb1, sym, bs,
                                           part, nblk, rpw)));
  } else {
    HY_CHECK((gram_dispatch<float, false>(ctx, n, ka, (const float*)A, lda, kb1, (const float*)B1, ldb1, sym, bs,
                                          part, nblk, rpw)));
  }
  return reduce_cols(ctx, nblk, ka * kt, part, G);
}

hyeig_status launch_gram(hyeig_ctx* ctx, int64_t n, int ka, const void* A, int64_t lda, int kb, const void* B,
                         int64_t ldb, hyeig_dtype dt, hyeig_mma_mode mode, double* G) {
  return launch_gram2(ctx, n, ka, A, lda, kb, B, ldb, 0, nullptr, 0, dt, mode, G, 0);
}

// ---------------------------------------------------------------------------
// Fixed device buffer for callers that cannot allocate (graph capture, serving
// loops): the Gram partials of hyeig_gram_noalloc live here.  Each device the
// library runs on holds its own copy until the process ends; host code never
// passes the array's name to a kernel (on the host it is only a stand-in), it
// passes the device address looked up once per device by scratch_init.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[HYEIG_MAX_DEVICES] = {};
}  // namespace

hyeig_status scratch_init(hyeig_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= HYEIG_MAX_DEVICES)
    return set_err(ctx, HYEIG_EUNSUPPORTED, "scratch: device index beyond the supported count");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* p = nullptr;
    HY_HIP(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_err(ctx, HYEIG_EDEVICE, "scratch: no device address");
    g_scratch_ptr[ctx->device] = (double*)p;
  }
  ctx->scratch = g_scratch_ptr[ctx->device];
  return HYEIG_OK;
}

hyeig_status launch_gram_noalloc(hyeig_ctx* ctx, int64_t n, int ka, const void* A, int64_t lda, int kb,
                                 const void* B, int64_t ldb, hyeig_dtype dt, hyeig_mma_mode mode, double* G) {
  if (!ctx->scratch) return set_err(ctx, HYEIG_EDEVICE, "gram_noalloc: fixed buffer not set up for this device");
  return launch_gram2(ctx, n, ka, A, lda, kb, B, ldb, 0, nullptr, 0, dt, mode, G, 0, ctx->scratch,
                      (int64_t)SCRATCH_DOUBLES);
}

hyeig_status launch_block_update_a(hyeig_ctx* ctx, int64_t n, int k, int m, const void* S, int64_t lds,
                                   const double* C, double alpha, double beta, void* Y, int64_t ldy, hyeig_dtype dt) {
  if (n <= 0) return HYEIG_OK;
  if (k > 64 || m > 32) return set_err(ctx, HYEIG_EUNSUPPORTED, "block_update: k > 64 or m > 32");
  if (dt == HYEIG_F64)
    return update_dispatch<double, false>(ctx, n, k, m, (const double*)S, lds, 0, C, alpha, beta, (double*)Y, ldy,
                                          nullptr, nullptr, 0);
  return update_dispatch<float, false>(ctx, n, k, m, (const float*)S, lds, 0, C, alpha, beta, (float*)Y, ldy, nullptr,
                                       nullptr, 0);
}

hyeig_status launch_block_update_bs(hyeig_ctx* ctx, int64_t n, int k, int m, const void* S, int64_t lds, int64_t bs,
                                    const double* C, void* Y, int64_t ldy, hyeig_dtype dt) {
  if (n <= 0) return HYEIG_OK;
  if (k > 64 || m > 32) return set_err(ctx, HYEIG_EUNSUPPORTED, "block_update: k > 64 or m > 32");
  if (bs > 0 && lds != 16) return set_err(ctx, HYEIG_EUNSUPPORTED, "block_update: block-strided S needs 16 columns");
  if (dt == HYEIG_F64)
    return update_dispatch<double, false>(ctx, n, k, m, (const double*)S, lds, bs, C, 1.0, 0.0, (double*)Y, ldy,
                                          nullptr, nullptr, 0);
  return update_dispatch<float, false>(ctx, n, k, m, (const float*)S, lds, bs, C, 1.0, 0.0, (float*)Y, ldy, nullptr,
                                       nullptr, 0);
}

hyeig_status launch_block_update(hyeig_ctx* ctx, int64_t n, int k, int m, const void* S, int64_t lds,
                                 const double* C, double beta, void* Y, int64_t ldy, hyeig_dtype dt) {
  return launch_block_update_a(ctx, n, k, m, S, lds, C, 1.0, beta, Y, ldy, dt);
}

hyeig_status launch_block_update2(hyeig_ctx* ctx, int64_t n, int k, int m, const void* S, int64_t lds,
                                  const double* C1, void* Y1, int64_t ld1, const double* C2, void* Y2, int64_t ld2,
                                  hyeig_dtype dt, int64_t bs) {
  if (n <= 0) return HYEIG_OK;
  if (k > 64 || m > 32) return set_err(ctx, HYEIG_EUNSUPPORTED, "block_update2: k > 64 or m > 32");
  if (bs > 0 && lds != 16) return set_err(ctx, HYEIG_EUNSUPPORTED, "block_update2: block-strided S needs 16 columns");
  if (dt == HYEIG_F64)
    return update_dispatch<double, true>(ctx, n, k, m, (const double*)S, lds, bs, C1, 1.0, 0.0, (double*)Y1, ld1, C2,
                                         (double*)Y2, ld2);
  return update_dispatch<float, true>(ctx, n, k, m, (const float*)S, lds, bs, C1, 1.0, 0.0, (float*)Y1, ld1, C2,
                                      (float*)Y2, ld2);
}

bool update_resid_fits(int64_t n, int k, int nb, int64_t ldy, const void* X1, const void* P1, const void* HX1,
                       const void* HP1, hyeig_dtype dt) {
  if (n <= 0 || nb < 1 || nb > 16 || k < 1 || k > 48) return false;
  if (dt == HYEIG_F64) return true;
  // FP32: 16-byte stores of four columns
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  return ldy % 4 == 0 && al(X1) && al(P1) && al(HX1) && al(HP1);
}

hyeig_status launch_update_resid(hyeig_ctx* ctx, int64_t n, int k, int nb, const void* S, const void* HS, int64_t lds,
                                 int64_t bss, const double* C1, const double* C2, void* X1, void* P1, void* HX1,
                                 void* HP1, int64_t ldy, const double* theta, const float* d, double floor,
                                 const int* pos, int na, void* W, int64_t ldw, hyeig_dtype dt, double* norms2) {
  if (!update_resid_fits(n, k, nb, ldy, X1, P1, HX1, HP1, dt))
    return set_err(ctx, HYEIG_EUNSUPPORTED, "update_resid: shape or alignment");
  const int64_t ntiles = (n + 15) / 16;
  const int64_t maxblk = std::min<int64_t>((ntiles + 3) / 4, (int64_t)ctx->num_cu * 8);
  hyeig_status st;
  double* part = (double*)ws_get(ctx, WS_REDUCE, (size_t)maxblk * nb * sizeof(double), &st);
  if (!part) return st;
  int nblk = 0;
  if (dt == HYEIG_F64)
    HY_CHECK(update_resid_dispatch<double>(ctx, n, k, nb, (const double*)S, (const double*)HS, lds, bss, C1, C2,
                                           (double*)X1, (double*)P1, (double*)HX1, (double*)HP1, ldy, theta, d, floor,
                                           pos, na, (double*)W, ldw, part, &nblk));
  else
    HY_CHECK(update_resid_dispatch<float>(ctx, n, k, nb, (const float*)S, (const float*)HS, lds, bss, C1, C2,
                                          (float*)X1, (float*)P1, (float*)HX1, (float*)HP1, ldy, theta, d, floor, pos,
                                          na, (float*)W, ldw, part, &nblk));
  return reduce_cols(ctx, nblk, nb, part, norms2);
}

hyeig_status launch_resid_precond(hyeig_ctx* ctx, int64_t n, int nb, const void* X, int64_t ldx, const void* HX,
                                  int64_t ldhx, const double* theta, const float* d, double floor, int na,
                                  const int* pos, void* W, int64_t ldw, int wtot, hyeig_dtype dt, double* norms2,
                                  const int* guard) {
  if (nb > 32 || wtot > 32) return set_err(ctx, HYEIG_EUNSUPPORTED, "resid_precond: more than 32 columns");
  int nblk = reduce_blocks(n);
  hyeig_status st;
  double* part = (double*)ws_get(ctx, WS_REDUCE, (size_t)nblk * nb * sizeof(double), &st);
  if (!part) return st;
  const int vw = dt == HYEIG_F32 ? 4 : 2;  // elements per 16-byte piece
  const bool vec = nb % vw == 0 && ldx % vw == 0 && ldhx % vw == 0 && ((uintptr_t)X & 15) == 0 &&
                   ((uintptr_t)HX & 15) == 0;
  if (vec) {
    if (dt == HYEIG_F32)
      hipLaunchKernelGGL(k_resid_precond_v<float>, dim3(nblk), dim3(256), 0, ctx->stream, n, nb, (const float*)X, ldx,
                         (const float*)HX, ldhx, theta, d, floor, pos, na, (float*)W, ldw, wtot, part, guard);
    else
      hipLaunchKernelGGL(k_resid_precond_v<double>, dim3(nblk), dim3(256), 0, ctx->stream, n, nb, (const double*)X,
                         ldx, (const double*)HX, ldhx, theta, d, floor, pos, na, (double*)W, ldw, wtot, part, guard);
    HY_CHECK(hip_err(ctx, hipGetLastError(), "k_resid_precond_v launch"));
    return norms2 ? reduce_cols(ctx, nblk, nb, part, norms2) : HYEIG_OK;
  }
  dim3 blk(32, 8);
  if (dt == HYEIG_F64)
    hipLaunchKernelGGL(k_resid_precond<double>, dim3(nblk), blk, 0, ctx->stream, n, nb, (const double*)X, ldx,
                       (const double*)HX, ldhx, theta, d, floor, pos, na, (double*)W, ldw, wtot, part, guard);
  else
    hipLaunchKernelGGL(k_resid_precond<float>, dim3(nblk), blk, 0, ctx->stream, n, nb, (const float*)X, ldx,
                       (const float*)HX, ldhx, theta, d, floor, pos, na, (float*)W, ldw, wtot, part, guard);
  HY_CHECK(hip_err(ctx, hipGetLastError(), "k_resid_precond launch"));
  return norms2 ? reduce_cols(ctx, nblk, nb, part, norms2) : HYEIG_OK;
}
