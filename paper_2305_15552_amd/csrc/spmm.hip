// Half-stored symmetric block product Y = H X, H = U + U^T - diag(U), for gfx950.
//
// The prepared form groups the upper triangle U in 32 x 32 tiles.  For tile
// (I, J) (block row I, block column J >= I) it keeps the 32 row bitmasks, the 32
// column bitmasks (the diagonal excluded, so each diagonal entry is applied
// once) and the tile's values packed row-major, each tile starting on an
// 8-value boundary; a column index lists the tiles of each block column.
// The product kernel is "owner computes": the wavefront owning block row J
// applies both halves of H for y_J (the tiles of row J directly, the tiles of
// column J transposed) and writes y_J once.  No atomics, no clearing of Y.
// Every tile is read twice, once by its row owner and once by its column
// owner; the second read comes at most a band width of block rows later.
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
__device__ inline int64_t wave_sum_i64(int64_t v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// tiles per block row and their value storage (each tile rounded up to 8 values)
__global__ void k_tile_count(int64_t n, int64_t nbr, const int64_t* __restrict__ rowptr,
                             const int32_t* __restrict__ colidx, int64_t* __restrict__ counts,
                             int64_t* __restrict__ pvals) {
  const int lane = threadIdx.x & 63;
  const int64_t br = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (br >= nbr) return;
  const int64_t row = br * 32 + lane;
  const bool own = lane < 32 && row < n;
  int64_t p = own ? rowptr[row] : 0, e = own ? rowptr[row + 1] : 0;
  int64_t cnt = 0, pv = 0;
  for (;;) {
    int cur = (p < e) ? (colidx[p] >> 5) : INT_MAX;
    int J = wave_min_i32(cur);
    if (J == INT_MAX) break;
    ++cnt;
    int64_t p0 = p;
    while (p < e && (colidx[p] >> 5) == J) ++p;
    int64_t tn = wave_sum_i64(p - p0);
    pv += (tn + 7) & ~(int64_t)7;
  }
  if (lane == 0) {
    counts[br] = cnt;
    pvals[br] = pv;
  }
}

__global__ void k_tile_fill(int64_t n, int64_t nbr, const int64_t* __restrict__ rowptr,
                            const int32_t* __restrict__ colidx, const float* __restrict__ vin,
                            const int64_t* __restrict__ tile_ptr, int32_t* __restrict__ tile_col,
                            int64_t* __restrict__ tile_val, uint32_t* __restrict__ tile_mask,
                            uint32_t* __restrict__ tile_cmask, float* __restrict__ vout, float* __restrict__ diag,
                            const int64_t* __restrict__ vbase_br) {
  const int lane = threadIdx.x & 63;
  const int64_t br = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (br >= nbr) return;
  const int64_t row = br * 32 + lane;
  const bool own = lane < 32 && row < n;
  int64_t p = own ? rowptr[row] : 0, e = own ? rowptr[row + 1] : 0;
  int64_t vbase = vbase_br[br];
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
    vbase += (total + 7) & ~7u;
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
// the product ("owner computes")
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

// Inclusive prefix sum inside each 32-lane half of the wave, by DPP row shifts
// (within rows of 16 lanes) and a row broadcast of lane 15 / 47 into rows 1 / 3.
template <int CTRL, int ROWMASK>
__device__ inline uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xf, false);
}
__device__ inline uint32_t incl_scan32(uint32_t x) {
  x += dpp_u32<0x111, 0xf>(x);  // row_shr:1
  x += dpp_u32<0x112, 0xf>(x);  // row_shr:2
  x += dpp_u32<0x114, 0xf>(x);  // row_shr:4
  x += dpp_u32<0x118, 0xf>(x);  // row_shr:8
  x += dpp_u32<0x142, 0xa>(x);  // row_bcast:15, rows 1 and 3
  return x;
}

__device__ inline int rl(int v, int q) { return __builtin_amdgcn_readlane(v, q); }

// LDS pointers keep their 32-bit address arithmetic
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T*;

// Row stride (elements) of a staged 32 x M block of x in LDS: a whole number of
// 16-byte slots, odd, so that rows taken at random by different lanes spread
// over the LDS banks (an even slot count maps many rows onto the same banks).
template <int M, typename AT>
struct XStride {
  static constexpr int RB = M * (int)sizeof(AT);
  static constexpr int SLOTS = (RB + 15) / 16;
  static constexpr int ODD = (SLOTS % 2 == 0) ? SLOTS + 1 : SLOTS;
  static constexpr int VALUE = (RB < 16) ? M : ODD * 16 / (int)sizeof(AT);
};

// Per-wave LDS: the staged x blocks of the two halves (the first one reused to
// combine the halves at the end), the packed values of the two tiles in flight
// and the (row offset, row mask) table of the transposed tile.
template <int M, typename AT>
struct SpmmLds {
  static constexpr int XS = XStride<M, AT>::VALUE;
  static constexpr int XB = 32 * XS;  // elements of one staged x block
  static constexpr int BYTES = 2 * XB * (int)sizeof(AT) + 2 * 1024 * 4 + 64 * 8;
  static constexpr int WAVES = 1;  // one wave per workgroup: LDS in the finest grain for occupancy
};

// Values of one tile half, staged by 32 lanes in chunks of 16 bytes (4 FP32 or
// 8 BF16 values): chunk c = lane + 32 q.  Tiles start on 8-value boundaries.
template <typename VT>
struct VChunk {
  static constexpr int PER = 16 / (int)sizeof(VT);  // values per chunk
  static constexpr int QV = 4;                        // chunks per lane held in registers
};

// x block of one half: 32 rows of M elements.  With 16-byte rows pieces
// (VEC) lane `self` holds pieces self + 32 q; otherwise elements self + 32 q.
// Either way a lane holds M elements.
template <int M, typename XT>
struct XBlk {
  static constexpr int EPC = 16 / (int)sizeof(XT);                     // elements per piece
  static constexpr bool VEC = (M * (int)sizeof(XT)) % 16 == 0;
  static constexpr int CPR = VEC ? M / EPC : 1;                        // pieces per row
  static constexpr int NQ = VEC ? CPR : M;                             // loads per lane
};

template <int M, typename XT, typename VT>
struct Pref {
  uint32_t rowm, cm;
  uint4 v[VChunk<VT>::QV];
  XT x[M];
};

template <int M, bool XV, typename XT, typename VT>
__device__ inline void prefetch(Pref<M, XT, VT>& pf, bool has, bool dir, int self, int t, int64_t vb, int nv,
                                int xblk, const uint32_t* __restrict__ tile_mask,
                                const uint32_t* __restrict__ tile_cmask, const VT* __restrict__ vals,
                                const XT* __restrict__ X, int64_t n, int m, int64_t ldx) {
  using XB_ = XBlk<M, XT>;
  pf.rowm = has ? tile_mask[(int64_t)t * 32 + self] : 0u;
  pf.cm = (has && !dir) ? tile_cmask[(int64_t)t * 32 + self] : 0u;
  const uint4* vc = reinterpret_cast<const uint4*>(vals + vb);
  const int nch = has ? nv / VChunk<VT>::PER : 0;
#pragma unroll
  for (int q = 0; q < VChunk<VT>::QV; ++q) {
    const int c = self + 32 * q;
    pf.v[q] = c < nch ? vc[c] : make_uint4(0, 0, 0, 0);
  }
  const int64_t row0 = (int64_t)xblk * 32;
  const XT* xb = X + row0 * ldx;
  if constexpr (XV) {
#pragma unroll
    for (int q = 0; q < XB_::NQ; ++q) {
      const int ch = self + 32 * q;
      const int r = ch / XB_::CPR, cc = ch % XB_::CPR;
      uint4 u = make_uint4(0, 0, 0, 0);
      if (has && row0 + r < n) u = *reinterpret_cast<const uint4*>(xb + (int64_t)r * ldx + cc * XB_::EPC);
      const XT* e = reinterpret_cast<const XT*>(&u);
#pragma unroll
      for (int i = 0; i < XB_::EPC; ++i) pf.x[q * XB_::EPC + i] = e[i];
    }
  } else {
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const int e = self + 32 * q;  // element e of the block: row e / M, column e % M
      const int r = e / M, j = e % M;
      pf.x[q] = (has && row0 + r < n && j < m) ? xb[(int64_t)r * ldx + j] : (XT)0;
    }
  }
}

// stage the prefetched x block of one half into LDS (row stride XS)
template <int M, bool XV, typename XT, typename AT, int XS>
__device__ inline void stage_x(const XT (&x)[M], AT* Xs, int self) {
  using XB_ = XBlk<M, XT>;
  if constexpr (XV) {
#pragma unroll
    for (int q = 0; q < XB_::NQ; ++q) {
      const int ch = self + 32 * q;
      const int r = ch / XB_::CPR, cc = ch % XB_::CPR;
#pragma unroll
      for (int i = 0; i < XB_::EPC; ++i) Xs[r * XS + cc * XB_::EPC + i] = (AT)x[q * XB_::EPC + i];
    }
  } else {
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const int e = self + 32 * q;
      Xs[(e / M) * XS + (e % M)] = (AT)x[q];
    }
  }
}

template <typename VT>
__device__ inline float chunk_val(const uint4& u, int i);
template <>
__device__ inline float chunk_val<float>(const uint4& u, int i) {
  const uint32_t w = i == 0 ? u.x : i == 1 ? u.y : i == 2 ? u.z : u.w;
  return __uint_as_float(w);
}
template <>
__device__ inline float chunk_val<uint16_t>(const uint4& u, int i) {
  const uint32_t w = (i >> 1) == 0 ? u.x : (i >> 1) == 1 ? u.y : (i >> 1) == 2 ? u.z : u.w;
  return __uint_as_float((i & 1) ? (w & 0xFFFF0000u) : (w << 16));
}

__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave w owns block row J and forms y_J completely:
//   lanes  0..31 (direct half):     the tiles (J, J') of block row J,
//                                   y_J[r] += sum_c u_rc x_J'[c]        (r = lane)
//   lanes 32..63 (transposed half): the tiles (I, J) of block column J, I <= J,
//                                   y_J[c] += sum_r u_rc x_I[r]        (c = lane - 32)
// The halves walk their tile lists in step.  Per step: lane q of the wave holds
// the metadata of step s0 + q (read out with readlane); the masks, values and x
// block of the next step are loaded into registers while the current step
// computes.  Each lane walks the set bits of its row (direct) or column
// (transposed) bitmask; the value of entry (r, c) sits at the tile's row
// offset of r plus the number of set bits of row r left of c.  The walk is a
// three-stage pipeline: bit and row-table lookup of entry k + 2, value and x
// row loads of entry k + 1, FMAs of entry k, unrolled twice so that the x
// rows alternate between two register sets.  y_J, the sum of both halves, is
// written once with plain stores: no atomics and no clearing of Y.
template <int M, bool XV, typename XT, typename AT, typename VT>
__global__ __launch_bounds__(256) void k_spmm_sym(int64_t n, int64_t nbr, int per_xcd,
                                                  const int64_t* __restrict__ tile_ptr,
                                                  const int64_t* __restrict__ col_ptr,
                                                  const int32_t* __restrict__ col_tiles,
                                                  const int32_t* __restrict__ col_brow,
                                                  const int32_t* __restrict__ tile_col,
                                                  const int64_t* __restrict__ tile_val,
                                                  const uint32_t* __restrict__ tile_mask,
                                                  const uint32_t* __restrict__ tile_cmask,
                                                  const VT* __restrict__ vals, int m, const XT* __restrict__ X,
                                                  int64_t ldx, AT* __restrict__ Y, int64_t ldy, int yvec) {
  using L = SpmmLds<M, AT>;
  constexpr int XS = L::XS;
  constexpr int WAVES = L::WAVES;
  constexpr int PER = VChunk<VT>::PER;
  constexpr int QV = VChunk<VT>::QV;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // workgroups are dealt to the 8 XCDs in turn: give each XCD a contiguous range of block rows
  const int64_t blk = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  const int64_t J = blk * WAVES + wv;
  if (J >= nbr) return;  // wave-uniform

  unsigned char* base = lds_raw + (size_t)wv * L::BYTES;
  AT* XD = reinterpret_cast<AT*>(base);  // x of the direct half's tile; y staging at the end
  AT* XT_ = XD + L::XB;                  // x of the transposed half's tile
  float* PD = reinterpret_cast<float*>(XT_ + L::XB);
  float* PT = PD + 1024;
  uint2* RI = reinterpret_cast<uint2*>(PT + 1024);  // (row offset, row mask) of both tiles, 32 each

  const bool dir = lane < 32;
  const int self = lane & 31;
  AT* const Xs = dir ? XD : XT_;
  float* const P = dir ? PD : PT;
  const int64_t r0 = tile_ptr[J], r1 = tile_ptr[J + 1];
  const int64_t c0 = col_ptr[J], c1 = col_ptr[J + 1];
  const int64_t nr = r1 - r0, nc = c1 - c0;
  const int64_t steps = nr > nc ? nr : nc;

  AT a[M];
#pragma unroll
  for (int j = 0; j < M; ++j) a[j] = (AT)0;

  for (int64_t s0 = 0; s0 < steps; s0 += 64) {
    // lane q: metadata of step s0 + q for both halves
    const int64_t sq = s0 + lane;
    const int td = (sq < nr) ? (int)(r0 + sq) : -1;
    const int tt = (sq < nc) ? col_tiles[c0 + sq] : -1;
    const int xd = (td >= 0) ? tile_col[td] : 0;
    const int xt = (tt >= 0) ? col_brow[c0 + sq] : 0;
    int64_t lo = (td >= 0) ? tile_val[td] : 0, hi = (td >= 0) ? tile_val[td + 1] : 0;
    const int vd8 = (int)(lo >> 3), nd = (int)(hi - lo);
    lo = (tt >= 0) ? tile_val[tt] : 0;
    hi = (tt >= 0) ? tile_val[tt + 1] : 0;
    const int vt8 = (int)(lo >> 3), nt = (int)(hi - lo);
    const int cnt = (int)((steps - s0) < 64 ? (steps - s0) : 64);

    Pref<M, XT, VT> pf;
    auto fetch = [&](int q) -> bool {
      const int t0 = rl(td, q), t1 = rl(tt, q), b0 = rl(vd8, q), b1 = rl(vt8, q);
      const int n0 = rl(nd, q), n1 = rl(nt, q), x0 = rl(xd, q), x1 = rl(xt, q);
      const int t = dir ? t0 : t1;
      const bool has = t >= 0;
      const int64_t vb = (int64_t)(uint32_t)(dir ? b0 : b1) << 3;
      const int nv = dir ? n0 : n1;
      const int xblk = dir ? x0 : x1;
      prefetch<M, XV, XT, VT>(pf, has, dir, self, t, vb, nv, xblk, tile_mask, tile_cmask, vals, X, n, m, ldx);
      return has;
    };
    bool has_n = fetch(0);

    for (int q = 0; q < cnt; ++q) {
      const bool has = has_n;
      const int vb0 = rl(vd8, q), vb1 = rl(vt8, q);
      const int64_t vb = (int64_t)(uint32_t)(dir ? vb0 : vb1) << 3;
      const uint32_t rowm = pf.rowm;
      uint32_t bits = dir ? rowm : pf.cm;
      const uint32_t v0 = (uint32_t)__popc(rowm);
      const uint32_t inc = incl_scan32(v0);
      const uint32_t off = inc - v0;
      const uint32_t tot0 = (uint32_t)rl((int)inc, 31), tot1 = (uint32_t)rl((int)inc, 63);
      const uint32_t total = dir ? tot0 : tot1;
      // stage the prefetched step in LDS
      RI[lane] = make_uint2(off, rowm);
      const int nch = has ? (int)((total + PER - 1) / PER) : 0;
#pragma unroll
      for (int qq = 0; qq < QV; ++qq) {
        const int c = self + 32 * qq;
        if (c < nch)
#pragma unroll
          for (int i = 0; i < PER; ++i) P[c * PER + i] = chunk_val<VT>(pf.v[qq], i);
      }
      if (nch > 32 * QV) {
        // values beyond the chunks held in registers (tiles with more than 32 QV PER entries)
        const uint4* vc = reinterpret_cast<const uint4*>(vals + vb);
        for (int c = self + 32 * QV; c < nch; c += 32) {
          const uint4 u = vc[c];
#pragma unroll
          for (int i = 0; i < PER; ++i) P[c * PER + i] = chunk_val<VT>(u, i);
        }
      }
      stage_x<M, XV, XT, AT, XS>(pf.x, Xs, self);
      // prefetch the next step
      if (q + 1 < cnt) has_n = fetch(q + 1);
      wave_sync_lds();

      // walk the entries: lanes without entries skip; a lane past its last
      // entry re-reads its previous one (a valid address) before leaving
      if (bits) {
        // direct lanes look up their own row, transposed lanes row idx of their tile
        const uint2* RIh = RI + (dir ? 0 : 32);
        auto pos_of = [&](int idx, uint2 ri) -> uint32_t {
          const int c = dir ? idx : self;
          return ri.x + (uint32_t)__popc(ri.y & ((1u << c) - 1u));
        };
        auto row_info = [&](int idx) -> uint2 { return RIh[dir ? self : idx]; };
        // x row idx of the staged block, addressed in 32-bit LDS bytes
        const uint32_t x3 = (uint32_t)(uintptr_t)(lds_ptr<const AT>)Xs;
        auto xrow = [&](int idx) -> lds_ptr<const AT> {
          return (lds_ptr<const AT>)(uintptr_t)(x3 + __umul24((unsigned)idx, (unsigned)(XS * sizeof(AT))));
        };
        auto take = [&](int prev, bool& has) -> int {
          has = bits != 0u;
          const int i = has ? __builtin_ctz(bits) : prev;
          bits &= bits - 1u;
          return i;
        };
        auto fma_row = [&](float v, const AT(&xr)[M]) {
          const AT w = (AT)v;
#pragma unroll
          for (int j = 0; j < M; ++j) a[j] += w * xr[j];
        };
        bool hB, hC, hD;
        const int iA = __builtin_ctz(bits);
        bits &= bits - 1u;
        const uint2 rA = row_info(iA);
        int iB = take(iA, hB);
        uint2 rB = row_info(iB);
        float vA = P[pos_of(iA, rA)];
        AT xA[M];
#pragma unroll
        for (int j = 0; j < M; ++j) xA[j] = xrow(iA)[j];
        for (;;) {
          // loads: row table of entry C, value and x row of entry B; then the FMAs of entry A
          const int iC = take(iB, hC);
          const uint2 rC = row_info(iC);
          const float vB = P[pos_of(iB, rB)];
          AT xB[M];
#pragma unroll
          for (int j = 0; j < M; ++j) xB[j] = xrow(iB)[j];
          __builtin_amdgcn_sched_barrier(0);
          fma_row(vA, xA);
          __builtin_amdgcn_sched_barrier(0);
          if (!hB) break;
          const int iD = take(iC, hD);
          const uint2 rD = row_info(iD);
          vA = P[pos_of(iC, rC)];
#pragma unroll
          for (int j = 0; j < M; ++j) xA[j] = xrow(iC)[j];
          __builtin_amdgcn_sched_barrier(0);
          fma_row(vB, xB);
          __builtin_amdgcn_sched_barrier(0);
          if (!hC) break;
          iB = iD;
          rB = rD;
          hB = hD;
        }
      }
      wave_sync_lds();
    }
  }
  // y_J = direct half + transposed half: the transposed lanes hand their sums
  // over through LDS and the direct lanes store the rows
  if (!dir) {
#pragma unroll
    for (int j = 0; j < M; ++j) XD[self * XS + j] = a[j];
  }
  wave_sync_lds();
  if (dir) {
#pragma unroll
    for (int j = 0; j < M; ++j) a[j] += XD[self * XS + j];
    const int64_t row = J * 32 + self;
    if (row < n) {
      AT* yr = Y + row * ldy;
      constexpr bool YV = (M * (int)sizeof(AT)) % 16 == 0;
      if (YV && yvec) {
        constexpr int EPC = 16 / (int)sizeof(AT);
#pragma unroll
        for (int q = 0; q < M / EPC; ++q) {
          uint4 u;
          AT* e = reinterpret_cast<AT*>(&u);
#pragma unroll
          for (int i = 0; i < EPC; ++i) e[i] = a[q * EPC + i];
          *reinterpret_cast<uint4*>(yr + q * EPC) = u;
        }
      } else {
#pragma unroll
        for (int j = 0; j < M; ++j)
          if (j < m) yr[j] = a[j];
      }
    }
  }
}

template <int M, bool XV, typename XT, typename AT, typename VT>
hyeig_status launch_kernel(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                           const VT* vals, int64_t blocks, int per_xcd, size_t lds, int waves, bool yvec) {
  auto kern = k_spmm_sym<M, XV, XT, AT, VT>;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), lds, ctx->stream, H->n, H->nbr, per_xcd,
                     H->tile_ptr, H->col_ptr, H->col_tiles, H->col_brow, H->tile_col, H->tile_val, H->tile_mask,
                     H->tile_cmask, vals, m, X, ldx, Y, ldy, (int)yvec);
  return hip_err(ctx, hipGetLastError(), "k_spmm_sym launch");
}

template <int M, typename XT, typename AT, typename VT>
hyeig_status run_spmm(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                      const VT* vals) {
  using L = SpmmLds<M, AT>;
  const int waves = L::WAVES;
  const int64_t groups = (H->nbr + waves - 1) / waves;
  if (groups == 0) return HYEIG_OK;
  const int64_t per_xcd = (groups + 7) / 8;
  const int64_t blocks = per_xcd * 8;
  if (blocks > (int64_t)INT_MAX) return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: matrix too large");
  const size_t lds = (size_t)L::BYTES * waves;
  // 16-byte pieces of x and y rows when the rows are whole, aligned and unpadded
  const bool xvec = m == M && (ldx * (int64_t)sizeof(XT)) % 16 == 0 && ((uintptr_t)X & 15) == 0;
  const bool yvec = m == M && (ldy * (int64_t)sizeof(AT)) % 16 == 0 && ((uintptr_t)Y & 15) == 0;
  if constexpr (XBlk<M, XT>::VEC) {
    if (xvec) return launch_kernel<M, true>(ctx, H, m, X, ldx, Y, ldy, vals, blocks, (int)per_xcd, lds, waves, yvec);
  }
  return launch_kernel<M, false>(ctx, H, m, X, ldx, Y, ldy, vals, blocks, (int)per_xcd, lds, waves, yvec);
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
                               int64_t* counts, int64_t* pvals) {
  int64_t blocks = (nbr * 64 + 255) / 256;
  hipLaunchKernelGGL(k_tile_count, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, n, nbr, rowptr, colidx,
                     counts, pvals);
  return hip_err(ctx, hipGetLastError(), "k_tile_count launch");
}

hyeig_status launch_tile_fill(hyeig_ctx* ctx, hyeig_mat* M, const int64_t* rowptr, const int32_t* colidx,
                              const float* vals, const int64_t* vbase) {
  int64_t blocks = (M->nbr * 64 + 255) / 256;
  hipLaunchKernelGGL(k_tile_fill, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, M->n, M->nbr, rowptr, colidx,
                     vals, M->tile_ptr, M->tile_col, M->tile_val, M->tile_mask, M->tile_cmask, M->vals, M->diag,
                     vbase);
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
