// Device kernels of batched RMM-DIIS (Algorithm 4, SpMVs batched into one
// product as in Section 4.2).  FP32 vectors, FP64 coefficients and dots.
// Layouts: blocks n x k row-major with ld = k; the history ring is
// [s_max][n][k]; per-column coefficients are [k][SMAX] FP64 on the device.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace {

constexpr int RB = 8;  // rows per workgroup step in the element-wise kernels
// Reduction kernels run k x rb threads per workgroup (rb = 256 / k rows), so no
// lane idles for k < 32; partial sums per column go through dynamic LDS.

struct SlotList {
  int w;
  int slot[RMM_SMAX];
};

// x~_j = sum_l alpha[j][l] Xh[slot_l][:, j];  H x~_j = sum_l alpha[j][l] (Rh + theta_h X h)[slot_l][:, j]
// dots: [blk][k][2] = (x~ . x~, x~ . Hx~)
template <typename T>
__global__ __launch_bounds__(256) void k_rmm_combine(int64_t n, int k, const T* __restrict__ Xh,
                                                     const T* __restrict__ Rh, SlotList sl,
                                                     const double* __restrict__ alpha,
                                                     const double* __restrict__ thetah,
                                                     const int* __restrict__ active, T* __restrict__ Xt,
                                                     T* __restrict__ HXt, double* __restrict__ part) {
  extern __shared__ double red[];
  const int j = threadIdx.x, ty = threadIdx.y, rb = blockDim.y;
  double sxx = 0.0, sxh = 0.0;
  if (active[j]) {
    double a[RMM_SMAX], th[RMM_SMAX];
#pragma unroll
    for (int l = 0; l < RMM_SMAX; ++l) {
      a[l] = l < sl.w ? alpha[j * RMM_SMAX + l] : 0.0;
      th[l] = l < sl.w ? thetah[j * RMM_SMAX + l] : 0.0;
    }
    for (int64_t i = (int64_t)blockIdx.x * rb + ty; i < n; i += (int64_t)gridDim.x * rb) {
      double x = 0.0, hx = 0.0;
      // the window in groups of four slots, every load of a group issued before
      // its sums (slots past w read slot 0 again and are not summed)
#pragma unroll
      for (int l0 = 0; l0 < RMM_SMAX; l0 += 4) {
        if (l0 < sl.w) {
          T xv[4], rv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int l = l0 + u;
            const int64_t off = (int64_t)(l < sl.w ? sl.slot[l] : sl.slot[0]) * n * k + i * k + j;
            xv[u] = Xh[off];
            rv[u] = Rh[off];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (l0 + u < sl.w) {
              x += a[l0 + u] * (double)xv[u];
              hx += a[l0 + u] * ((double)rv[u] + th[l0 + u] * (double)xv[u]);
            }
        }
      }
      const T xf = (T)x, hf = (T)hx;
      Xt[i * k + j] = xf;
      HXt[i * k + j] = hf;
      sxx += (double)xf * (double)xf;
      sxh += (double)xf * (double)hf;
    }
  }
  red[(ty * k + j) * 2 + 0] = sxx;
  red[(ty * k + j) * 2 + 1] = sxh;
  __syncthreads();
  if (ty == 0) {
    double a = 0, b = 0;
    for (int q = 0; q < rb; ++q) {
      a += red[(q * k + j) * 2 + 0];
      b += red[(q * k + j) * 2 + 1];
    }
    part[((int64_t)blockIdx.x * k + j) * 2 + 0] = a;
    part[((int64_t)blockIdx.x * k + j) * 2 + 1] = b;
  }
}

// x~ /= nrm, Hx~ /= nrm, r~ = Hx~ - theta~ x~, Z = r~ / max(|d - theta~|, floor) (or r~)
template <typename T>
__global__ __launch_bounds__(256) void k_rmm_scale(int64_t n, int k, const double* __restrict__ coef,
                                                   const int* __restrict__ active, T* __restrict__ Xt,
                                                   T* __restrict__ HXt, T* __restrict__ Zt,
                                                   const float* __restrict__ d, double floor) {
  // k x rb threads per workgroup (rb = 256 / k rows), as in the reductions
  const int j = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  if (j >= k || i >= n || !active[j]) return;
  const double inv = coef[2 * j], th = coef[2 * j + 1];
  const double x = (double)Xt[i * k + j] * inv;
  const double hx = (double)HXt[i * k + j] * inv;
  const T xf = (T)x, hf = (T)hx;
  Xt[i * k + j] = xf;
  HXt[i * k + j] = hf;
  double r = (double)hf - th * (double)xf;
  if (d) {
    double den = fabs((double)d[i] - th);
    r = r / (den > floor ? den : floor);
  }
  Zt[i * k + j] = (T)r;
}

// six dots per column for the 2x2 pencil: x.Hx, x.Hz, z.Hz, x.x, x.z, z.z
template <typename T>
__global__ __launch_bounds__(256) void k_rmm_gram6(int64_t n, int k, const T* __restrict__ Xt,
                                                   const T* __restrict__ Zt, const T* __restrict__ HXt,
                                                   const T* __restrict__ HZ, double* __restrict__ part) {
  extern __shared__ double red[];
  const int j = threadIdx.x, ty = threadIdx.y, rb = blockDim.y;
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * rb + ty; i < n; i += (int64_t)gridDim.x * rb) {
    const double x = Xt[i * k + j], z = Zt[i * k + j], hx = HXt[i * k + j], hz = HZ[i * k + j];
    s[0] += x * hx;
    s[1] += x * hz;
    s[2] += z * hz;
    s[3] += x * x;
    s[4] += x * z;
    s[5] += z * z;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) red[(ty * k + j) * 6 + q] = s[q];
  __syncthreads();
  if (ty == 0)
    for (int q = 0; q < 6; ++q) {
      double a = 0;
      for (int t = 0; t < rb; ++t) a += red[(t * k + j) * 6 + q];
      part[((int64_t)blockIdx.x * k + j) * 6 + q] = a;
    }
}

// x = g0 x~ + g1 z; Hx = g0 Hx~ + g1 Hz; r = Hx - theta x; push (x, r) into the ring at
// slot `push`; dots: [blk][k][1 + w] = (r.r, r.Rh[slot_l] for l < w) with the new entry.
template <typename T>
__global__ __launch_bounds__(256) void k_rmm_update(int64_t n, int k, const double* __restrict__ g,
                                                    const int* __restrict__ active, const T* __restrict__ Xt,
                                                    const T* __restrict__ Zt, const T* __restrict__ HXt,
                                                    const T* __restrict__ HZ, T* __restrict__ X,
                                                    T* __restrict__ HX, T* __restrict__ R,
                                                    T* __restrict__ Xh, T* __restrict__ Rh, int push,
                                                    SlotList sl, double* __restrict__ part) {
  extern __shared__ double red[];
  constexpr int W = RMM_SMAX + 1;
  const int j = threadIdx.x, ty = threadIdx.y, rb = blockDim.y;
  double s[W];
#pragma unroll
  for (int q = 0; q < W; ++q) s[q] = 0.0;
  if (active[j]) {
    const double g0 = g[3 * j], g1 = g[3 * j + 1], th = g[3 * j + 2];
    for (int64_t i = (int64_t)blockIdx.x * rb + ty; i < n; i += (int64_t)gridDim.x * rb) {
      const int64_t e = i * k + j;
      const double x = g0 * (double)Xt[e] + g1 * (double)Zt[e];
      const double hx = g0 * (double)HXt[e] + g1 * (double)HZ[e];
      const T xf = (T)x, hf = (T)hx;
      const T rf = (T)((double)hf - th * (double)xf);
      X[e] = xf;
      HX[e] = hf;
      R[e] = rf;
      const int64_t po = (int64_t)push * n * k + e;
      Xh[po] = xf;
      Rh[po] = rf;
      s[0] += (double)rf * (double)rf;
      // fully unrolled over the window so the sums stay in registers; history
      // loads in groups of four as in the combination
#pragma unroll
      for (int l0 = 0; l0 < RMM_SMAX; l0 += 4) {
        if (l0 < sl.w) {
          T rv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int l = l0 + u;
            const int sl_ = l < sl.w ? sl.slot[l] : sl.slot[0];
            rv[u] = Rh[(int64_t)sl_ * n * k + e];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (l0 + u < sl.w) s[1 + l0 + u] += (double)rf * (double)((sl.slot[l0 + u] == push) ? rf : rv[u]);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < W; ++q) red[(ty * k + j) * W + q] = s[q];
  __syncthreads();
  if (ty == 0)
    for (int q = 0; q <= sl.w; ++q) {
      double a = 0;
      for (int t = 0; t < rb; ++t) a += red[(t * k + j) * W + q];
      part[((int64_t)blockIdx.x * k + j) * W + q] = a;
    }
}

__global__ void k_reduce_parts(int nblk, int width, const double* __restrict__ part, double* __restrict__ out) {
  int c = blockIdx.x * blockDim.y + threadIdx.y;
  if (c >= width) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[(int64_t)b * width + c];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0) out[c] = s;
}

int nblocks_for(int64_t n) {
  int64_t b = (n + RB - 1) / RB;
  return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

hyeig_status reduce_parts(hyeig_ctx* ctx, int nblk, int width, const double* part, double* out) {
  dim3 blk(64, 4);
  hipLaunchKernelGGL(k_reduce_parts, dim3((width + 3) / 4), blk, 0, ctx->stream, nblk, width, part, out);
  return hip_err(ctx, hipGetLastError(), "k_reduce_parts launch");
}

SlotList make_slots(int w, const int* slots) {
  SlotList s;
  s.w = w;
  for (int l = 0; l < RMM_SMAX; ++l) s.slot[l] = l < w ? slots[l] : 0;
  return s;
}



template <typename T>
hyeig_status rmm_combine_t(hyeig_ctx* ctx, int64_t n, int k, const void* Xh, const void* Rh, int w, const int* slots,
                           const double* alpha, const double* thetah, const int* active, void* Xt, void* HXt,
                           double* dots2) {
  int nblk = nblocks_for(n);
  hyeig_status st;
  double* part = (double*)ws_get(ctx, WS_REDUCE, (size_t)nblk * k * 2 * sizeof(double), &st);
  if (!part) return st;
  const int rb = 256 / k;
  hipLaunchKernelGGL(k_rmm_combine<T>, dim3(nblk), dim3(k, rb), sizeof(double) * rb * k * 2, ctx->stream, n, k, (const T*)Xh, (const T*)Rh,
                     make_slots(w, slots), alpha, thetah, active, (T*)Xt, (T*)HXt, part);
  HY_CHECK(hip_err(ctx, hipGetLastError(), "k_rmm_combine launch"));
  return reduce_parts(ctx, nblk, k * 2, part, dots2);
}

template <typename T>
hyeig_status rmm_scale_t(hyeig_ctx* ctx, int64_t n, int k, const double* coef, const int* active, void* Xt, void* HXt,
                         void* Zt, const float* d, double floor) {
  const int rb = 256 / k;
  dim3 grd((unsigned)((n + rb - 1) / rb));
  hipLaunchKernelGGL(k_rmm_scale<T>, grd, dim3(k, rb), 0, ctx->stream, n, k, coef, active, (T*)Xt, (T*)HXt, (T*)Zt,
                     d, floor);
  return hip_err(ctx, hipGetLastError(), "k_rmm_scale launch");
}

template <typename T>
hyeig_status rmm_gram6_t(hyeig_ctx* ctx, int64_t n, int k, const void* Xt, const void* Zt, const void* HXt,
                         const void* HZ, double* g6) {
  int nblk = nblocks_for(n);
  hyeig_status st;
  double* part = (double*)ws_get(ctx, WS_REDUCE, (size_t)nblk * k * 6 * sizeof(double), &st);
  if (!part) return st;
  const int rb = 256 / k;
  hipLaunchKernelGGL(k_rmm_gram6<T>, dim3(nblk), dim3(k, rb), sizeof(double) * rb * k * 6, ctx->stream, n, k, (const T*)Xt, (const T*)Zt,
                     (const T*)HXt, (const T*)HZ, part);
  HY_CHECK(hip_err(ctx, hipGetLastError(), "k_rmm_gram6 launch"));
  return reduce_parts(ctx, nblk, k * 6, part, g6);
}

template <typename T>
hyeig_status rmm_update_t(hyeig_ctx* ctx, int64_t n, int k, const double* g, const int* active, const void* Xt,
                          const void* Zt, const void* HXt, const void* HZ, void* X, void* HX, void* R, void* Xh,
                          void* Rh, int push, int w, const int* slots, double* dots) {
  int nblk = nblocks_for(n);
  hyeig_status st;
  double* part = (double*)ws_get(ctx, WS_REDUCE, (size_t)nblk * k * (RMM_SMAX + 1) * sizeof(double), &st);
  if (!part) return st;
  const int rb = 256 / k;
  hipLaunchKernelGGL(k_rmm_update<T>, dim3(nblk), dim3(k, rb), sizeof(double) * rb * k * (RMM_SMAX + 1), ctx->stream, n, k, g, active, (const T*)Xt,
                     (const T*)Zt, (const T*)HXt, (const T*)HZ, (T*)X, (T*)HX, (T*)R, (T*)Xh, (T*)Rh, push,
                     make_slots(w, slots), part);
  HY_CHECK(hip_err(ctx, hipGetLastError(), "k_rmm_update launch"));
  return reduce_parts(ctx, nblk, k * (RMM_SMAX + 1), part, dots);
}

}  // namespace

hyeig_status launch_rmm_combine(hyeig_ctx* ctx, hyeig_dtype dt, int64_t n, int k, const void* Xh, const void* Rh,
                                int w, const int* slots, const double* alpha, const double* thetah,
                                const int* active, void* Xt, void* HXt, double* dots2) {
  if (dt == HYEIG_F64) return rmm_combine_t<double>(ctx, n, k, Xh, Rh, w, slots, alpha, thetah, active, Xt, HXt, dots2);
  return rmm_combine_t<float>(ctx, n, k, Xh, Rh, w, slots, alpha, thetah, active, Xt, HXt, dots2);
}

hyeig_status launch_rmm_scale(hyeig_ctx* ctx, hyeig_dtype dt, int64_t n, int k, const double* coef,
                              const int* active, void* Xt, void* HXt, void* Zt, const float* d, double floor) {
  if (dt == HYEIG_F64) return rmm_scale_t<double>(ctx, n, k, coef, active, Xt, HXt, Zt, d, floor);
  return rmm_scale_t<float>(ctx, n, k, coef, active, Xt, HXt, Zt, d, floor);
}

hyeig_status launch_rmm_gram6(hyeig_ctx* ctx, hyeig_dtype dt, int64_t n, int k, const void* Xt, const void* Zt,
                              const void* HXt, const void* HZ, double* g6) {
  if (dt == HYEIG_F64) return rmm_gram6_t<double>(ctx, n, k, Xt, Zt, HXt, HZ, g6);
  return rmm_gram6_t<float>(ctx, n, k, Xt, Zt, HXt, HZ, g6);
}

hyeig_status launch_rmm_update(hyeig_ctx* ctx, hyeig_dtype dt, int64_t n, int k, const double* g, const int* active,
                               const void* Xt, const void* Zt, const void* HXt, const void* HZ, void* X, void* HX,
                               void* R, void* Xh, void* Rh, int push, int w, const int* slots, double* dots) {
  if (dt == HYEIG_F64)
    return rmm_update_t<double>(ctx, n, k, g, active, Xt, Zt, HXt, HZ, X, HX, R, Xh, Rh, push, w, slots, dots);
  return rmm_update_t<float>(ctx, n, k, g, active, Xt, Zt, HXt, HZ, X, HX, R, Xh, Rh, push, w, slots, dots);
}
