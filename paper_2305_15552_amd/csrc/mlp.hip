// Learned per-row preconditioner: an MLP 4 -> 64 -> 1 (ReLU) evaluated on BF16
// matrix cores with FP32 accumulation, its MSE gradient, Adam on FP32 master
// weights, the residual features, and the correction-equation labels it is
// trained on (MINRES on the GPU through the library's own product).
//
// The preconditioner K of LOBPCG is left open by the paper (Section 2.3,
// eq. (wblock)); this learned K is a project addition.  Definitions:
//   out(f) = w2 . relu(W1 f + b1) + b2,  parameters W1[64][4], b1[64], w2[64], b2
//   features of residual entry (k, j): (d_k - theta_j)/||H||, r_kj/||r_j|| sqrt(n),
//     row 1-norm/||H||, row nnz / mean row nnz
//   apply: w_kj = out(f_kj) ||r_j|| / (||H|| sqrt(n))
//   target: t_j = 20 MINRES steps on (I - XX^T)(H - theta_j)(I - XX^T) t = -r_j,
//     scaled as t_kj ||H|| sqrt(n) / ||r_j||.
//
// Inference (the forward pass and the preconditioner apply) runs one sample per
// lane on 4x4x4 BF16 MFMAs with 16 blocks, 64 samples per wave step: block b,
// column j is the sample of lane 4 b + j, so the lane's own four features are
// its B operand (K = 4, no padding) and the instruction returns four hidden
// pre-activations of that sample in the lane's accumulator, which starts from
// b1.  Sixteen such products give all 64; after ReLU and rounding to BF16 they
// are the B operand of layer 2, whose A rows all hold the matching four w2
// entries, so register 0 of the accumulator ends with w2 . relu(h) for the
// lane's sample.
//
// Training evaluates on 16x16x32 BF16 MFMAs, 16 samples per wave step:
//   layer 1:  H^T (64 x 16) = W1' (64 x 32) F'^T (32 x 16), four 16-row blocks;
//             F' = (f0..f3, 1, 0, 0, 0) carries the bias b1 in W1' column 4
//   layer 2:  out^T (16 x 16, row 0 used) = w2'^T (16 x 64) H^T, two K=32 steps.
// Lane (g = lane / 16, i = lane % 16) receives layer-1 rows 4 g + q of each
// block for sample i; the layer-2 inner index is permuted so that exactly
// these values form its B operand (slot (g, e) <-> hidden 32 c + 4 g + e for
// e < 4 and 32 c + 16 + 4 g + e - 4 otherwise), with w2 permuted alike.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace {

constexpr int NH = HYEIG_MLP_HIDDEN;
constexpr int NF = HYEIG_MLP_FEATURES;
constexpr int NP = HYEIG_MLP_NPARAM;
constexpr int NPART = NP + 1;  // gradient partials plus the loss

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// device image of the weights
struct MlpDev {
  float master[NP];
  float m[NP], v[NP];
  uint16_t w1b[NH * 8];  // row h: bf16 W1[h][0..3], b1[h], 0, 0, 0
  uint16_t w2b[NH];
  float b2;
};

__device__ inline uint16_t bf16_bits(float x) {
  const __bf16 b = (__bf16)x;
  return __builtin_bit_cast(uint16_t, b);
}
__device__ inline float bf16_val(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }

// weights -> BF16 kernel operands
__device__ void pack_weights(MlpDev* W, int h) {
  if (h < NH) {
#pragma unroll
    for (int f = 0; f < NF; ++f) W->w1b[h * 8 + f] = bf16_bits(W->master[h * NF + f]);
    W->w1b[h * 8 + 4] = bf16_bits(W->master[NH * NF + h]);
    W->w1b[h * 8 + 5] = W->w1b[h * 8 + 6] = W->w1b[h * 8 + 7] = 0;
    W->w2b[h] = bf16_bits(W->master[NH * NF + NH + h]);
  }
  if (h == 0) W->b2 = W->master[NP - 1];
}

__global__ void k_mlp_pack(MlpDev* W) { pack_weights(W, threadIdx.x); }

// Two MLP layers for the 16 samples of a wave step.  f: features of sample i
// (lanes with g = 0 use them).  pre[hb][q] = layer-1 value of hidden 16 hb +
// 4 g + q for sample i (bias included); the return value is out for sample i
// on lanes with g = 0.
__device__ inline float mlp_eval16(const MlpDev* __restrict__ W, int g, int i, const float (&f)[NF],
                                   f32x4 (&pre)[4]) {
  bf16x8 bfe;
#pragma unroll
  for (int e = 0; e < 8; ++e) bfe[e] = (__bf16)0.0f;
  if (g == 0) {
#pragma unroll
    for (int e = 0; e < NF; ++e) bfe[e] = (__bf16)f[e];
    bfe[4] = (__bf16)1.0f;
  }
#pragma unroll
  for (int hb = 0; hb < 4; ++hb) {
    bf16x8 a;
    if (g == 0) {
      a = *reinterpret_cast<const bf16x8*>(W->w1b + (16 * hb + i) * 8);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] = (__bf16)0.0f;
    }
    pre[hb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfe, f32x4{0, 0, 0, 0}, 0, 0, 0);
  }
  f32x4 acc = {0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    bf16x8 b, a;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      b[e] = (__bf16)fmaxf(pre[2 * c][e], 0.0f);
      b[e + 4] = (__bf16)fmaxf(pre[2 * c + 1][e], 0.0f);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int h = 32 * c + (e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4));
      a[e] = (i == 0) ? __builtin_bit_cast(__bf16, W->w2b[h]) : (__bf16)0.0f;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  return acc[0] + W->b2;
}

__device__ inline void load_feat(const float* __restrict__ F, int64_t s, int64_t N, float (&f)[NF]) {
  if (s < N) {
    const float4 u = *reinterpret_cast<const float4*>(F + s * NF);
    f[0] = u.x, f[1] = u.y, f[2] = u.z, f[3] = u.w;
  } else {
    f[0] = f[1] = f[2] = f[3] = 0.f;
  }
}

typedef short s16x4 __attribute__((ext_vector_type(4)));

// Per-lane operands of the one-sample-per-lane evaluation: layer-1 A rows
// W1[4 hg + lane % 4][0..3], the accumulator start (b1 of hidden 4 hg .. 4 hg +
// 3), layer-2 A rows w2[4 hg .. 4 hg + 3] (all BF16 values; BF16 bit patterns as
// shorts, the builtin's operand type).
struct MlpLane {
  s16x4 a1[NH / 4];
  f32x4 c1[NH / 4];
  s16x4 a2[NH / 4];
  float b2;
};

__device__ inline void mlp_lane_load(const MlpDev* __restrict__ W, int lane, MlpLane& L) {
  const int i = lane & 3;
#pragma unroll
  for (int hg = 0; hg < NH / 4; ++hg) {
    L.a1[hg] = *reinterpret_cast<const s16x4*>(W->w1b + (4 * hg + i) * 8);
    L.a2[hg] = *reinterpret_cast<const s16x4*>(W->w2b + 4 * hg);
#pragma unroll
    for (int q = 0; q < 4; ++q) L.c1[hg][q] = bf16_val(W->w1b[(4 * hg + q) * 8 + 4]);
  }
  L.b2 = W->b2;
}

__device__ inline short bf16_short(float x) { return __builtin_bit_cast(short, (__bf16)x); }

// out(f) for the lane's own sample; every lane of the wave must call it
__device__ inline float mlp_eval64(const MlpLane& L, const float (&f)[NF]) {
  const s16x4 b = {bf16_short(f[0]), bf16_short(f[1]), bf16_short(f[2]), bf16_short(f[3])};
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int hg = 0; hg < NH / 4; ++hg) {
    const f32x4 h = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(L.a1[hg], b, L.c1[hg], 0, 0, 0);
    // ReLU on the BF16 bit patterns: a negative value (or -0) is a negative short
    s16x4 r = {bf16_short(h[0]), bf16_short(h[1]), bf16_short(h[2]), bf16_short(h[3])};
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = r[q] > 0 ? r[q] : (short)0;
    acc = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(L.a2[hg], r, acc, 0, 0, 0);
  }
  return acc[0] + L.b2;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const MlpDev* __restrict__ W, int64_t N,
                                                     const float* __restrict__ F, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  MlpLane L;
  mlp_lane_load(W, lane, L);
  const int64_t step = (int64_t)gridDim.x * 256;
  int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x - lane;
  float f[NF];
  load_feat(F, s + lane, N, f);
  for (; s < N; s += step) {
    const int64_t t = s + lane;
    float fn[NF];
    load_feat(F, t + step, N, fn);  // the next step's features, in flight during this one
    const float o = mlp_eval64(L, f);
    if (t < N) out[t] = o;
#pragma unroll
    for (int e = 0; e < NF; ++e) f[e] = fn[e];
  }
}

// inclusive sum over the 16 lanes of a DPP row; lane 15 of each row ends with the total
__device__ inline float row_sum16(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x112, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x118, 0xf, 0xf, false));
  return x;
}

// MSE loss and gradient: per-wave partials part[w][0..NP) (gradient, parameter
// layout) and part[w][NP] (sum of squared errors).  Lane (g, i) keeps the
// gradient terms of its 16 hidden units for the samples i it sees.
__global__ __launch_bounds__(256) void k_mlp_backward(const MlpDev* __restrict__ W, int64_t N,
                                                      const float* __restrict__ F, const float* __restrict__ T,
                                                      double* __restrict__ part) {
  const int lane = threadIdx.x & 63, g = lane >> 4, i = lane & 15;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t groups = (N + 15) / 16;
  const float scale = 2.0f / (float)N;
  float w2h[16];
#pragma unroll
  for (int hb = 0; hb < 4; ++hb)
#pragma unroll
    for (int q = 0; q < 4; ++q) w2h[hb * 4 + q] = bf16_val(W->w2b[16 * hb + 4 * g + q]);
  float gW1[16][NF], gb1[16], gw2[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    gb1[u] = gw2[u] = 0.f;
#pragma unroll
    for (int e = 0; e < NF; ++e) gW1[u][e] = 0.f;
  }
  float gb2 = 0.f;
  double sse = 0.0;
  for (int64_t gr = wave; gr < groups; gr += (int64_t)gridDim.x * 4) {
    const int64_t s = gr * 16 + i;
    float f[NF];
    load_feat(F, s, N, f);
    f32x4 pre[4];
    const float o = mlp_eval16(W, g, i, f, pre);
    float go = 0.f;
    if (g == 0 && s < N) {
      const float e = o - T[s];
      sse += (double)e * (double)e;
      go = scale * e;
      gb2 += go;
    }
    go = __shfl(go, i, 64);  // the output gradient of sample i, on every lane of column i
#pragma unroll
    for (int hb = 0; hb < 4; ++hb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int u = hb * 4 + q;
        const float p = pre[hb][q];
        gw2[u] += go * fmaxf(p, 0.f);
        const float dp = p > 0.f ? go * w2h[u] : 0.f;
        gb1[u] += dp;
#pragma unroll
        for (int e = 0; e < NF; ++e) gW1[u][e] += dp * f[e];
      }
  }
  // sum over the 16 samples columns of each row; lane 15 of row g writes
  double* out = part + wave * NPART;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int h = 16 * (u >> 2) + 4 * g + (u & 3);
    const float a = row_sum16(gb1[u]), b = row_sum16(gw2[u]);
    float c[NF];
#pragma unroll
    for (int e = 0; e < NF; ++e) c[e] = row_sum16(gW1[u][e]);
    if (i == 15) {
#pragma unroll
      for (int e = 0; e < NF; ++e) out[h * NF + e] = c[e];
      out[NH * NF + h] = a;
      out[NH * NF + NH + h] = b;
    }
  }
  const float tb2 = row_sum16(gb2);
  for (int off = 1; off < 16; off <<= 1) sse += __shfl_xor(sse, off, 64);
  if (lane == 15) {
    out[NP - 1] = tb2;
    out[NP] = sse;
  }
}

// Adam (Kingma and Ba, bias-corrected) on the FP32 master weights, then the
// BF16 operand copies
__global__ void k_mlp_adam(MlpDev* W, const double* __restrict__ grad, int step, float lr, float beta1, float beta2,
                           float eps) {
  const int q = threadIdx.x;
  if (q < NP) {
    const float gq = (float)grad[q];
    const float m = beta1 * W->m[q] + (1.f - beta1) * gq;
    const float v = beta2 * W->v[q] + (1.f - beta2) * gq * gq;
    W->m[q] = m;
    W->v[q] = v;
    const float mh = m / (1.f - powf(beta1, (float)step));
    const float vh = v / (1.f - powf(beta2, (float)step));
    W->master[q] -= lr * mh / (sqrtf(vh) + eps);
  }
  __syncthreads();
  pack_weights(W, q);
}

// features of a residual block (sample k * ncol + j)
template <typename T>
__device__ inline void entry_features(int64_t k, int j, const float* __restrict__ d, const double* __restrict__ theta,
                                      T r, const double* __restrict__ rnorm, const float* __restrict__ rowabs,
                                      const float* __restrict__ rownnz, double inv_h, double sqrt_n, double inv_mnz,
                                      float (&f)[NF]) {
  const double rn = rnorm[j] > 0 ? rnorm[j] : 1.0;
  f[0] = (float)(((double)d[k] - theta[j]) * inv_h);
  f[1] = (float)((double)r / rn * sqrt_n);
  f[2] = (float)((double)rowabs[k] * inv_h);
  f[3] = (float)((double)rownnz[k] * inv_mnz);
}

template <typename T>
__global__ void k_mlp_features(int64_t n, int ncol, const T* __restrict__ R, int64_t ldr, const float* __restrict__ d,
                               const double* __restrict__ theta, const double* __restrict__ rnorm,
                               const float* __restrict__ rowabs, const float* __restrict__ rownnz, double inv_h,
                               double sqrt_n, double inv_mnz, float* __restrict__ F) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n * ncol) return;
  const int64_t k = s / ncol;
  const int j = (int)(s % ncol);
  float f[NF];
  entry_features<T>(k, j, d, theta, R[k * ldr + j], rnorm, rowabs, rownnz, inv_h, sqrt_n, inv_mnz, f);
  *reinterpret_cast<float4*>(F + s * NF) = make_float4(f[0], f[1], f[2], f[3]);
}

// targets tau_kj = t_kj ||H|| sqrt(n) / ||r_j||
__global__ void k_mlp_targets(int64_t n, int ncol, const double* __restrict__ Tm, int64_t ldt,
                              const double* __restrict__ rnorm, double hs, float* __restrict__ tau) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n * ncol) return;
  const int64_t k = s / ncol;
  const int j = (int)(s % ncol);
  const double rn = rnorm[j] > 0 ? rnorm[j] : 1.0;
  tau[s] = (float)(Tm[k * ldt + j] * hs / rn);
}

// W[k, a] <- out(features of R[k, a]) ||r_a|| / (||H|| sqrt(n)) in place (W holds R
// on entry); a non-finite output sets *bad.  Column a of W is column j of the
// caller's block with pos[j] = a (pos null: j = a); theta and nrm2 (squared
// residual norms) are indexed by j.  Sample s = k na + a sits on lane s % 64 of
// its wave step; (k, a) advance by the grid stride without a division.
template <typename T>
__global__ __launch_bounds__(256) void k_mlp_precond(const MlpDev* __restrict__ W, int64_t n, int na, T* Wm,
                                                     int64_t ldw, const float* __restrict__ d,
                                                     const double* __restrict__ theta,
                                                     const double* __restrict__ nrm2, const int* __restrict__ pos,
                                                     int ncol, const float* __restrict__ rowabs,
                                                     const float* __restrict__ rownnz, double hnorm, double inv_mnz,
                                                     int* bad) {
  // per W column: theta / ||H|| split into FP32 head and tail, sqrt(n) / ||r||,
  // ||r|| / (||H|| sqrt(n))
  __shared__ float4 colc[32];
  const double sqrt_n = sqrt((double)n);
  if (threadIdx.x < ncol) {
    const int j = threadIdx.x;
    const int a = pos ? pos[j] : j;
    if (a >= 0 && a < na) {
      const double rn0 = sqrt(fmax(nrm2[j], 0.0));
      const double rn = rn0 > 0.0 ? rn0 : 1.0;
      const double th = theta[j] / hnorm;
      const float hi = (float)th;
      colc[a] = make_float4(hi, (float)(th - (double)hi), (float)(sqrt_n / rn), (float)(rn / (hnorm * sqrt_n)));
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  MlpLane L;
  mlp_lane_load(W, lane, L);
  const float inv_h = (float)(1.0 / hnorm), mnz = (float)inv_mnz;
  const int64_t N = n * na;
  const int64_t step = (int64_t)gridDim.x * 256;
  const int64_t qstep = step / na;
  const int rstep = (int)(step % na);
  int64_t base = (int64_t)blockIdx.x * 256 + threadIdx.x - lane;
  int64_t k = (base + lane) / na;
  int a = (int)((base + lane) % na);
  // the inputs of one wave step; the next step's are loaded before this one's
  // network runs, so their latency hides behind it
  struct In {
    float r, dk, ra, rz;
  };
  auto fetch = [&](int64_t kk, int aa, bool live) {
    In v = {0.f, 0.f, 0.f, 0.f};
    if (live) {
      v.r = (float)Wm[kk * ldw + aa];
      v.dk = d[kk];
      v.ra = rowabs[kk];
      v.rz = rownnz[kk];
    }
    return v;
  };
  In cur = fetch(k, a, base + lane < N);
  for (; base < N; base += step) {
    const bool live = base + lane < N;
    int64_t kn = k + qstep;
    int an = a + rstep;
    if (an >= na) {
      an -= na;
      ++kn;
    }
    const In nxt = fetch(kn, an, base + step + lane < N);
    const float4 cc = live ? colc[a] : make_float4(0.f, 0.f, 0.f, 0.f);
    // (d_k - theta_a) / ||H||: d_k / ||H|| - head - tail, exact to FP32 rounding
    // of the result when d_k is close to theta_a
    const float f[NF] = {(cur.dk * inv_h - cc.x) - cc.y, cur.r * cc.z, cur.ra * inv_h, cur.rz * mnz};
    const float o = mlp_eval64(L, f);
    if (live) {
      const float w = o * cc.w;
      if (!isfinite(w)) atomicOr(bad, 1);
      Wm[k * ldw + a] = (T)w;
    }
    cur = nxt;
    k = kn;
    a = an;
  }
}

// flags[1] += (flags[0] != 0); flags[0] = 0: counts the iterations whose learned
// preconditioner fell back, without a host round trip
__global__ void k_mlp_flag_count(int* flags) {
  if (threadIdx.x == 0) {
    if (flags[0]) flags[1] += 1;
    flags[0] = 0;
  }
}

// out[:, j] = a_j X1[:, j] + b_j X2[:, j] + c_j X3[:, j]   (FP64 blocks, X2/X3 nullable;
// out may alias an input)
__global__ void k_lincomb(int64_t n, int k, double* out, int64_t ld, const double* __restrict__ a, const double* X1,
                          const double* __restrict__ b, const double* X2, const double* __restrict__ c,
                          const double* X3) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t r = e / k;
  const int j = (int)(e % k);
  const int64_t o = r * ld + j;
  double v = a[j] * X1[o];
  if (X2) v += b[j] * X2[o];
  if (X3) v += c[j] * X3[o];
  out[o] = v;
}

// a grid of one-sample-per-lane kernels: as many 256-thread blocks as the chip
// holds at once (every wave stays resident for the grid-stride loop), fewer when
// N samples fill fewer; the occupancy is asked once per kernel
template <const void* (*K)()>
int64_t resident_blocks(hyeig_ctx* ctx, int64_t N) {
  static const int per_cu = [] {
    int b = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, K(), 256, 0) == hipSuccess && b > 0 ? b : 1;
  }();
  const int64_t need = (N + 255) / 256;
  const int64_t maxb = (int64_t)ctx->num_cu * per_cu;
  return need < 1 ? 1 : (need < maxb ? need : maxb);
}

const void* kp_forward() { return (const void*)k_mlp_forward; }
const void* kp_precond_f32() { return (const void*)k_mlp_precond<float>; }
const void* kp_precond_f64() { return (const void*)k_mlp_precond<double>; }

int mlp_blocks(hyeig_ctx* ctx, int64_t N) {
  int64_t groups = (N + 15) / 16;
  int64_t b = (groups + 3) / 4;
  const int64_t maxb = (int64_t)ctx->num_cu * 8;
  if (b > maxb) b = maxb;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

struct hyeig_mlp {
  hyeig_ctx* ctx = nullptr;
  MlpDev* d = nullptr;
  int step = 0;
};

hyeig_status launch_mlp_precond(hyeig_ctx* ctx, const hyeig_mlp* mlp, const hyeig_mat* H, int64_t n, int na,
                                void* W, int64_t ldw, hyeig_dtype dt, const double* theta, const double* nrm2,
                                const int* pos, int ncol, double hnorm, int* d_bad) {
  if (!H->rowabs || !H->rownnz)
    return set_err(ctx, HYEIG_EINVAL, "MLP preconditioner: the matrix was prepared without HYEIG_MAT_ROWSTATS");
  if (na > 32 || ncol > 32 || (!pos && ncol != na))
    return set_err(ctx, HYEIG_EINVAL, "MLP preconditioner: at most 32 columns");
  if (n <= 0 || na <= 0) return HYEIG_OK;
  const double inv_mnz = 1.0 / H->rownnz_mean;
  const int64_t blocks = dt == HYEIG_F64 ? resident_blocks<kp_precond_f64>(ctx, n * na)
                                          : resident_blocks<kp_precond_f32>(ctx, n * na);
  if (dt == HYEIG_F64)
    hipLaunchKernelGGL(k_mlp_precond<double>, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, mlp->d, n, na,
                       (double*)W, ldw, H->diag, theta, nrm2, pos, ncol, H->rowabs, H->rownnz, hnorm, inv_mnz, d_bad);
  else
    hipLaunchKernelGGL(k_mlp_precond<float>, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, mlp->d, n, na,
                       (float*)W, ldw, H->diag, theta, nrm2, pos, ncol, H->rowabs, H->rownnz, hnorm, inv_mnz, d_bad);
  return hip_err(ctx, hipGetLastError(), "k_mlp_precond launch");
}

hyeig_status launch_mlp_flag_count(hyeig_ctx* ctx, int* flags) {
  hipLaunchKernelGGL(k_mlp_flag_count, dim3(1), dim3(64), 0, ctx->stream, flags);
  return hip_err(ctx, hipGetLastError(), "k_mlp_flag_count launch");
}

namespace {

hyeig_status mlp_backward_dev(hyeig_ctx* ctx, const hyeig_mlp* mlp, int64_t N, const float* F, const float* T,
                              double* d_grad_loss /* NPART, device */) {
  const int blocks = mlp_blocks(ctx, N);
  const int waves = blocks * 4;
  hyeig_status st;
  double* part = (double*)ws_get(ctx, WS_MLP, (size_t)waves * NPART * sizeof(double), &st);
  if (!part) return st;
  HY_HIP(ctx, hipMemsetAsync(part, 0, (size_t)waves * NPART * sizeof(double), ctx->stream));
  hipLaunchKernelGGL(k_mlp_backward, dim3(blocks), dim3(256), 0, ctx->stream, mlp->d, N, F, T, part);
  HY_CHECK(hip_err(ctx, hipGetLastError(), "k_mlp_backward launch"));
  return reduce_cols(ctx, waves, NPART, part, d_grad_loss);
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hyeig_status alloc(hyeig_ctx* ctx, size_t bytes) {
    hipError_t e = hipMalloc(&p, bytes < 64 ? 64 : bytes);
    if (e != hipSuccess) {
      p = nullptr;
      return set_err(ctx, HYEIG_ENOMEM, "mlp: device allocation failed");
    }
    return HYEIG_OK;
  }
  double* d() const { return (double*)p; }
};

hyeig_status lincomb(hyeig_ctx* ctx, int64_t n, int k, double* out, int64_t ld, const double* a, const double* X1,
                     const double* b, const double* X2, const double* c, const double* X3) {
  const int64_t tot = n * k;
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, n, k, out, ld, a, X1,
                     b, X2, c, X3);
  return hip_err(ctx, hipGetLastError(), "k_lincomb launch");
}

}  // namespace

extern "C" {

hyeig_status hyeig_mlp_create(hyeig_ctx* ctx, const float* h_params, hyeig_mlp** out) {
  if (!ctx || !h_params || !out) return ctx ? set_err(ctx, HYEIG_EINVAL, "mlp_create: null argument") : HYEIG_EINVAL;
  *out = nullptr;
  for (int q = 0; q < NP; ++q)
    if (!std::isfinite(h_params[q])) return set_err(ctx, HYEIG_EINVAL, "mlp_create: non-finite parameter");
  hyeig_mlp* m = new hyeig_mlp();
  m->ctx = ctx;
  hipError_t e = hipMalloc((void**)&m->d, sizeof(MlpDev));
  if (e != hipSuccess) {
    delete m;
    return set_err(ctx, HYEIG_ENOMEM, "mlp_create: device allocation failed");
  }
  MlpDev host{};
  for (int q = 0; q < NP; ++q) host.master[q] = h_params[q];
  e = hipMemcpyAsync(m->d, &host, sizeof(MlpDev), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(64), 0, ctx->stream, m->d);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(m->d);
    delete m;
    return hip_err(ctx, e, "mlp_create");
  }
  *out = m;
  return HYEIG_OK;
}

hyeig_status hyeig_mlp_get(hyeig_ctx* ctx, const hyeig_mlp* mlp, float* h_params) {
  if (!ctx || !mlp || !h_params) return ctx ? set_err(ctx, HYEIG_EINVAL, "mlp_get: null argument") : HYEIG_EINVAL;
  HY_HIP(ctx, hipMemcpyAsync(h_params, mlp->d->master, sizeof(float) * NP, hipMemcpyDeviceToHost, ctx->stream));
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return HYEIG_OK;
}

void hyeig_mlp_destroy(hyeig_mlp* mlp) {
  if (!mlp) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(mlp->d);
  delete mlp;
}

hyeig_status hyeig_mlp_forward(hyeig_ctx* ctx, const hyeig_mlp* mlp, int64_t N, const float* d_feat, float* d_out) {
  if (!ctx || !mlp || N < 0 || (N > 0 && (!d_feat || !d_out)))
    return ctx ? set_err(ctx, HYEIG_EINVAL, "mlp_forward: bad argument") : HYEIG_EINVAL;
  if (((uintptr_t)d_feat & 15) != 0) return set_err(ctx, HYEIG_EINVAL, "mlp_forward: features must be 16-byte aligned");
  if (N == 0) return HYEIG_OK;
  const int64_t blocks = resident_blocks<kp_forward>(ctx, N);
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, mlp->d, N, d_feat, d_out);
  return hip_err(ctx, hipGetLastError(), "k_mlp_forward launch");
}

hyeig_status hyeig_mlp_precond(hyeig_ctx* ctx, const hyeig_mlp* mlp, const hyeig_mat* H, int k, void* d_W,
                               int64_t ldw, hyeig_dtype dt, const double* h_theta, double hnorm) {
  if (!ctx) return HYEIG_EINVAL;
  if (!mlp || !H || !d_W || !h_theta || k < 1 || k > 32 || ldw < k || !(hnorm > 0.0))
    return set_err(ctx, HYEIG_EINVAL, "mlp_precond: bad argument (1 <= k <= 32, ldw >= k, hnorm > 0, non-null)");
  if (dt != HYEIG_F32 && dt != HYEIG_F64) return set_err(ctx, HYEIG_EUNSUPPORTED, "mlp_precond: dtype");
  if (!H->rowabs || !H->rownnz)
    return set_err(ctx, HYEIG_EINVAL, "mlp_precond: the matrix was prepared without HYEIG_MAT_ROWSTATS");
  const int64_t n = H->n;
  if (n == 0) return HYEIG_OK;
  hyeig_status st;
  // device: squared column norms (k), theta (k), the non-finite flag
  double* dw = (double*)ws_get(ctx, WS_MLP2, sizeof(double) * (2 * (size_t)k + 1), &st);
  if (!dw) return st;
  int* bad = reinterpret_cast<int*>(dw + 2 * k);
  HY_CHECK(launch_col_dots(ctx, n, k, d_W, ldw, d_W, ldw, dt, dw));
  HY_CHECK(h2d_queued(ctx, dw + k, h_theta, sizeof(double) * k));
  HY_CHECK(launch_fill(ctx, 1, 1, bad, 1, HYEIG_F32, 0.0));  // integer zero (all bits clear)
  HY_CHECK(launch_mlp_precond(ctx, mlp, H, n, k, d_W, ldw, dt, dw + k, dw, nullptr, k, hnorm, bad));
  int hb = 0;
  HY_HIP(ctx, hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (hb) return set_err(ctx, HYEIG_ENUMERIC, "mlp_precond: non-finite network output");
  return HYEIG_OK;
}

hyeig_status hyeig_mlp_backward(hyeig_ctx* ctx, const hyeig_mlp* mlp, int64_t N, const float* d_feat,
                                const float* d_target, float* d_grad, double* h_loss) {
  if (!ctx || !mlp || N <= 0 || !d_feat || !d_target || !d_grad)
    return ctx ? set_err(ctx, HYEIG_EINVAL, "mlp_backward: bad argument") : HYEIG_EINVAL;
  if (((uintptr_t)d_feat & 15) != 0) return set_err(ctx, HYEIG_EINVAL, "mlp_backward: features must be 16-byte aligned");
  hyeig_status st;
  double* gl = (double*)ws_get(ctx, WS_MLP2, NPART * sizeof(double), &st);
  if (!gl) return st;
  HY_CHECK(mlp_backward_dev(ctx, mlp, N, d_feat, d_target, gl));
  std::vector<double> h(NPART);
  HY_HIP(ctx, hipMemcpyAsync(h.data(), gl, sizeof(double) * NPART, hipMemcpyDeviceToHost, ctx->stream));
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<float> g(NP);
  for (int q = 0; q < NP; ++q) g[q] = (float)h[q];
  HY_HIP(ctx, hipMemcpyAsync(d_grad, g.data(), sizeof(float) * NP, hipMemcpyHostToDevice, ctx->stream));
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h_loss) *h_loss = h[NP] / (double)N;
  return HYEIG_OK;
}

hyeig_status hyeig_mlp_train(hyeig_ctx* ctx, hyeig_mlp* mlp, int64_t N, const float* d_feat, const float* d_target,
                             const hyeig_train_params* tp, double* h_loss_per_epoch) {
  if (!ctx || !mlp || N <= 0 || !d_feat || !d_target || !tp || tp->epochs < 0 || tp->batch <= 0)
    return ctx ? set_err(ctx, HYEIG_EINVAL, "mlp_train: bad argument") : HYEIG_EINVAL;
  if (((uintptr_t)d_feat & 15) != 0) return set_err(ctx, HYEIG_EINVAL, "mlp_train: features must be 16-byte aligned");
  hyeig_status st;
  double* gl = (double*)ws_get(ctx, WS_MLP2, NPART * sizeof(double), &st);
  if (!gl) return st;
  const int64_t nb = (N + tp->batch - 1) / tp->batch;
  // batches are contiguous ranges; their order is shuffled every epoch
  std::vector<int64_t> order(nb);
  for (int64_t b = 0; b < nb; ++b) order[b] = b;
  uint64_t rs = tp->seed * 0x9E3779B97F4A7C15ull + 1;
  std::vector<double> loss(NPART);
  for (int ep = 0; ep < tp->epochs; ++ep) {
    for (int64_t b = nb - 1; b > 0; --b) {
      rs ^= rs << 13, rs ^= rs >> 7, rs ^= rs << 17;
      std::swap(order[b], order[(int64_t)(rs % (uint64_t)(b + 1))]);
    }
    double sse = 0.0;
    for (int64_t bi = 0; bi < nb; ++bi) {
      const int64_t s0 = order[bi] * tp->batch;
      const int64_t cnt = std::min<int64_t>(tp->batch, N - s0);
      HY_CHECK(mlp_backward_dev(ctx, mlp, cnt, d_feat + s0 * NF, d_target + s0, gl));
      ++mlp->step;
      hipLaunchKernelGGL(k_mlp_adam, dim3(1), dim3(NP), 0, ctx->stream, mlp->d, gl, mlp->step, (float)tp->lr,
                         (float)tp->beta1, (float)tp->beta2, (float)tp->eps);
      HY_CHECK(hip_err(ctx, hipGetLastError(), "k_mlp_adam launch"));
      if (h_loss_per_epoch) {
        HY_HIP(ctx, hipMemcpyAsync(loss.data() + NP, gl + NP, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
        sse += loss[NP];
      }
    }
    if (h_loss_per_epoch) h_loss_per_epoch[ep] = sse / (double)N;
  }
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return HYEIG_OK;
}

hyeig_status hyeig_mlp_labels(hyeig_ctx* ctx, const hyeig_mat* H, int k, const void* d_X, int64_t ldx,
                              hyeig_dtype dt, double hnorm, int steps, float* d_feat, float* d_target,
                              double* h_theta) {
  if (!ctx || !H || !d_X || !d_feat || !d_target || k < 1 || k > 32 || ldx < k || hnorm <= 0 || steps < 1 ||
      (dt != HYEIG_F32 && dt != HYEIG_F64))
    return ctx ? set_err(ctx, HYEIG_EINVAL, "mlp_labels: bad argument") : HYEIG_EINVAL;
  if (!H->rowabs || !H->rownnz)
    return set_err(ctx, HYEIG_EINVAL, "mlp_labels: the matrix was prepared without HYEIG_MAT_ROWSTATS");
  if (((uintptr_t)d_feat & 15) != 0) return set_err(ctx, HYEIG_EINVAL, "mlp_labels: features must be 16-byte aligned");
  const int64_t n = H->n;
  const size_t blk = (size_t)n * k * sizeof(double);
  DevBuf X, R, v, pv, xs, b0, b1, b2, c0, c1, c2, sc;
  for (DevBuf* b : {&X, &R, &v, &pv, &xs, &b0, &b1, &b2, &c0, &c1, &c2}) HY_CHECK(b->alloc(ctx, blk));
  HY_CHECK(sc.alloc(ctx, sizeof(double) * (8 * 32 + 32 * 32)));
  double* s_a = sc.d();
  double* s_b = s_a + 32;
  double* s_c = s_b + 32;
  double* s_dot = s_c + 32;
  double* s_th = s_dot + 32;
  double* s_rn = s_th + 32;
  double* G = s_a + 8 * 32;
  auto coef = [&](const std::vector<double>& a, const std::vector<double>& b,
                  const std::vector<double>& c) -> hyeig_status {
    std::vector<double> h(3 * 32, 0.0);
    for (int j = 0; j < k; ++j) h[j] = a[j], h[32 + j] = b[j], h[64 + j] = c[j];
    HY_HIP(ctx, hipMemcpyAsync(s_a, h.data(), sizeof(double) * 96, hipMemcpyHostToDevice, ctx->stream));
    HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return HYEIG_OK;
  };
  auto dots = [&](const double* A, const double* B, std::vector<double>& out) -> hyeig_status {
    HY_CHECK(launch_col_dots(ctx, n, k, A, k, B, k, HYEIG_F64, s_dot));
    HY_HIP(ctx, hipMemcpyAsync(out.data(), s_dot, sizeof(double) * k, hipMemcpyDeviceToHost, ctx->stream));
    HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return HYEIG_OK;
  };
  // vv <- (I - X X^T) vv
  auto proj = [&](double* vv) -> hyeig_status {
    HY_CHECK(launch_gram(ctx, n, k, X.p, k, k, vv, k, HYEIG_F64, HYEIG_MMA_F64, G));
    return launch_block_update_a(ctx, n, k, k, X.p, k, G, -1.0, 1.0, vv, k, HYEIG_F64);
  };
  const std::vector<double> one(k, 1.0), zero(k, 0.0);
  // orthonormal Ritz block, Ritz values, residuals and their norms (FP64)
  HY_CHECK(launch_copy(ctx, n, k, d_X, ldx, dt, X.p, k, HYEIG_F64));
  HY_CHECK(hyeig_cholqr(ctx, n, k, X.p, k, HYEIG_F64, 2, nullptr));
  HY_CHECK(launch_spmm(ctx, H, k, X.p, k, HYEIG_F64, R.p, k, HYEIG_F64, HYEIG_F32));
  std::vector<double> th(k), rn(k), negth(k);
  HY_CHECK(dots(X.d(), R.d(), th));
  for (int j = 0; j < k; ++j) negth[j] = -th[j];
  HY_CHECK(coef(one, negth, zero));
  HY_CHECK(lincomb(ctx, n, k, R.d(), k, s_a, R.d(), s_b, X.d(), nullptr, nullptr));
  HY_CHECK(dots(R.d(), R.d(), rn));
  for (int j = 0; j < k; ++j) rn[j] = std::sqrt(rn[j]);
  HY_HIP(ctx, hipMemcpyAsync(s_th, th.data(), sizeof(double) * k, hipMemcpyHostToDevice, ctx->stream));
  HY_HIP(ctx, hipMemcpyAsync(s_rn, rn.data(), sizeof(double) * k, hipMemcpyHostToDevice, ctx->stream));
  // MINRES (Paige and Saunders) on P (H - theta_j) P t = -P r_j for all columns at
  // once: Lanczos vectors in three rotating buffers (r1, r2, next), direction
  // vectors w in three (w1, w2, w), scalar recurrences per column on the host
  double *r1 = b0.d(), *r2 = b1.d(), *ny = b2.d();
  double *w1 = c0.d(), *w2 = c1.d(), *w = c2.d();
  std::vector<double> negone(k, -1.0);
  HY_CHECK(coef(negone, zero, zero));
  HY_CHECK(lincomb(ctx, n, k, r2, k, s_a, R.d(), nullptr, nullptr, nullptr, nullptr));
  HY_CHECK(proj(r2));
  HY_HIP(ctx, hipMemsetAsync(xs.p, 0, blk, ctx->stream));
  HY_HIP(ctx, hipMemsetAsync(w, 0, blk, ctx->stream));
  HY_HIP(ctx, hipMemsetAsync(w2, 0, blk, ctx->stream));
  HY_HIP(ctx, hipMemsetAsync(r1, 0, blk, ctx->stream));
  std::vector<double> beta(k), oldb(k, 0.0), dbar(k, 0.0), epsln(k, 0.0), phibar(k), cs(k, -1.0), sn(k, 0.0),
      alfa(k), ca(k), cb(k), cc(k);
  HY_CHECK(dots(r2, r2, beta));
  std::vector<char> live(k);
  for (int j = 0; j < k; ++j) {
    beta[j] = std::sqrt(beta[j]);
    phibar[j] = beta[j];
    live[j] = beta[j] > 0.0;
  }
  for (int it = 0; it < steps; ++it) {
    // v = y / beta with y = r2
    for (int j = 0; j < k; ++j) ca[j] = live[j] ? 1.0 / beta[j] : 0.0;
    HY_CHECK(coef(ca, zero, zero));
    HY_CHECK(lincomb(ctx, n, k, v.d(), k, s_a, r2, nullptr, nullptr, nullptr, nullptr));
    // next = P (H - theta) P v - (beta / oldb) r1
    HY_HIP(ctx, hipMemcpyAsync(pv.p, v.p, blk, hipMemcpyDeviceToDevice, ctx->stream));
    HY_CHECK(proj(pv.d()));
    HY_CHECK(launch_spmm(ctx, H, k, pv.p, k, HYEIG_F64, ny, k, HYEIG_F64, HYEIG_F32));
    HY_CHECK(coef(one, negth, zero));
    HY_CHECK(lincomb(ctx, n, k, ny, k, s_a, ny, s_b, pv.d(), nullptr, nullptr));
    HY_CHECK(proj(ny));
    for (int j = 0; j < k; ++j) cb[j] = (it > 0 && live[j]) ? -beta[j] / oldb[j] : 0.0;
    HY_CHECK(coef(one, cb, zero));
    HY_CHECK(lincomb(ctx, n, k, ny, k, s_a, ny, s_b, r1, nullptr, nullptr));
    HY_CHECK(dots(v.d(), ny, alfa));
    // next -= (alfa / beta) r2
    for (int j = 0; j < k; ++j) cb[j] = live[j] ? -alfa[j] / beta[j] : 0.0;
    HY_CHECK(coef(one, cb, zero));
    HY_CHECK(lincomb(ctx, n, k, ny, k, s_a, ny, s_b, r2, nullptr, nullptr));
    // r1 <- r2, r2 <- next; the old r1 becomes the next scratch
    double* t = r1;
    r1 = r2;
    r2 = ny;
    ny = t;
    std::vector<double> nb(k);
    HY_CHECK(dots(r2, r2, nb));
    std::vector<double> phi(k), gam(k), oldeps(k), delta(k);
    for (int j = 0; j < k; ++j) {
      if (!live[j]) {
        phi[j] = 0.0, gam[j] = 1.0, oldeps[j] = delta[j] = 0.0;
        continue;
      }
      oldb[j] = beta[j];
      beta[j] = std::sqrt(nb[j]);
      oldeps[j] = epsln[j];
      delta[j] = cs[j] * dbar[j] + sn[j] * alfa[j];
      const double gbar = sn[j] * dbar[j] - cs[j] * alfa[j];
      epsln[j] = sn[j] * beta[j];
      dbar[j] = -cs[j] * beta[j];
      gam[j] = std::max(std::hypot(gbar, beta[j]), 1e-300);
      cs[j] = gbar / gam[j];
      sn[j] = beta[j] / gam[j];
      phi[j] = cs[j] * phibar[j];
      phibar[j] = sn[j] * phibar[j];
    }
    // w <- (v - oldeps w1 - delta w2) / gamma with (w1, w2) <- (w2, w), into the old w1
    for (int j = 0; j < k; ++j) {
      ca[j] = live[j] ? 1.0 / gam[j] : 0.0;
      cb[j] = live[j] ? -oldeps[j] / gam[j] : 0.0;
      cc[j] = live[j] ? -delta[j] / gam[j] : 0.0;
    }
    HY_CHECK(coef(ca, cb, cc));
    HY_CHECK(lincomb(ctx, n, k, w1, k, s_a, v.d(), s_b, w2, s_c, w));
    t = w1;
    w1 = w2;
    w2 = w;
    w = t;
    // x += phi w
    HY_CHECK(coef(one, phi, zero));
    HY_CHECK(lincomb(ctx, n, k, xs.d(), k, s_a, xs.d(), s_b, w, nullptr, nullptr));
    for (int j = 0; j < k; ++j)
      if (beta[j] == 0.0) live[j] = 0;
  }
  // features of R and targets of the MINRES solutions
  const double inv_h = 1.0 / hnorm, sqrt_n = std::sqrt((double)n), inv_mnz = 1.0 / H->rownnz_mean;
  const int64_t tot = n * k;
  hipLaunchKernelGGL(k_mlp_features<double>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, n, k,
                     R.d(), (int64_t)k, H->diag, s_th, s_rn, H->rowabs, H->rownnz, inv_h, sqrt_n, inv_mnz, d_feat);
  HY_CHECK(hip_err(ctx, hipGetLastError(), "k_mlp_features launch"));
  hipLaunchKernelGGL(k_mlp_targets, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream, n, k, xs.d(),
                     (int64_t)k, s_rn, hnorm * sqrt_n, d_target);
  HY_CHECK(hip_err(ctx, hipGetLastError(), "k_mlp_targets launch"));
  HY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (h_theta)
    for (int j = 0; j < k; ++j) h_theta[j] = th[j];
  return HYEIG_OK;
}

}  // extern "C"
