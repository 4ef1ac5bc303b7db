// Half-stored symmetric block product Y = H X, H = U + U^T - diag(U), for gfx950.
//
// The prepared form groups the upper triangle U in 32 x 32 tiles.  For tile
// (I, J) (block row I, block column J >= I) it keeps the 32 row bitmasks, the 32
// column bitmasks (the diagonal excluded, so each diagonal entry is applied
// once), the tile's values packed row-major, each tile starting on an 8-value
// boundary, and a second copy of them packed column-major in the same range
// (memory traded for a sequential walk of the transposed half); a column index
// lists the tiles of each block column.  For the matrix-core products every
// stored value also gets its slot in a dense operand tile (uint16, built on
// first use).
// The product kernels are "owner computes": the workgroup owning block row J
// applies both halves of H for y_J (the tiles of row J directly, the tiles of
// column J transposed) and writes y_J once.  No atomics, no clearing of Y.
// Every tile is read twice, once by its row owner and once by its column
// owner; the second read comes at most a band width of block rows later.
// Kernels: k_spmm_sym walks the set bits on vector units (widths up to 8, and
// BF16 values); k_spmm_sym_mma2 applies each tile as a dense 32 x 32 product
// on matrix cores (widths 9-16, FP32 or FP64 sums); k_spmm_sym_mma is the same
// with operands picked from the masks, used when the slots cannot be stored.
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

// Column-major copy of each tile's values in the tile's own value range: the
// entries of column c (rows ascending; the diagonal left out of diagonal
// tiles, as in the column masks) one after another, columns in order.  One
// wave per tile; lane c < 32 fills column c, reading entry (r, c) at row r's
// offset plus the set bits of row r left of c.
__global__ __launch_bounds__(256) void k_tile_tvals(int64_t ntiles, const int64_t* __restrict__ tile_val,
                                                    const uint32_t* __restrict__ tile_mask,
                                                    const uint32_t* __restrict__ tile_cmask,
                                                    const float* __restrict__ vals, float* __restrict__ tvals) {
  __shared__ uint32_t srm[4][32], sro[4][32];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, c = lane & 31;
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const bool live = t < ntiles;
  const uint32_t rm = live ? tile_mask[t * 32 + c] : 0u;
  const uint32_t cm = live ? tile_cmask[t * 32 + c] : 0u;
  uint32_t tot;
  const uint32_t ro = excl_scan32((uint32_t)__popc(rm), lane, &tot);
  const uint32_t co = excl_scan32((uint32_t)__popc(cm), lane, &tot);
  if (lane < 32) {
    srm[w][c] = rm;
    sro[w][c] = ro;
  }
  __syncthreads();
  if (live && lane < 32) {
    const int64_t vb = tile_val[t];
    const uint32_t below = (1u << c) - 1u;
    uint32_t bits = cm, k = 0;
    while (bits) {
      const int r = __builtin_ctz(bits);
      bits &= bits - 1u;
      tvals[vb + co + k] = vals[vb + sro[w][r] + (uint32_t)__popc(srm[w][r] & below)];
      ++k;
    }
  }
}

// ---------------------------------------------------------------------------
// the product ("owner computes")
// ---------------------------------------------------------------------------
using v4u = __attribute__((ext_vector_type(4))) unsigned int;
using v2u = __attribute__((ext_vector_type(2))) unsigned int;

// Raw buffer resource over [base, base + bytes): a load at an offset at or past
// `bytes` returns zero and reads no memory.  Word 3 is the raw 32-bit data
// format of the gfx9 family.
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ inline v4u buf_ld16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
}
// the same with the non-temporal hint (cache policy bit 1 on gfx950): for the
// tile values and masks, which stream through once per half, so that they do
// not push the x blocks (re-read by other tiles) out of the caches
__device__ inline v4u buf_ld16_nt(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 2);
}
// one element of X (4 or 8 bytes) as raw bits
template <typename XT>
struct XBits;
template <>
struct XBits<float> {
  using T = uint32_t;
  static __device__ T load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
  }
};
template <>
struct XBits<double> {
  using T = v2u;
  static __device__ T load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
  }
};
// an offset that every resource here treats as out of range
constexpr uint32_t OOB = 0x7FFFFFF0u;

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

__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS pointers keep 32-bit address arithmetic
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T*;

// Row stride (bytes) of a staged 32-row block in LDS: a whole, odd number of
// 16-byte slots, so that rows picked at random by different lanes spread over
// the LDS banks; rows under 16 bytes are packed.
template <int RB>
struct OddStride {
  static constexpr int SLOTS = (RB + 15) / 16;
  static constexpr int VALUE = (RB < 16) ? RB : ((SLOTS % 2 == 0) ? SLOTS + 1 : SLOTS) * 16;
};

// Per-wave LDS of the product: the values (2 KB: every BF16 tile, FP32 tiles of
// up to 512 entries) and the x blocks of the two tiles of a step, reused at the
// end for the wave's partial sums.  2 KB rather than the 4 KB of a full FP32
// tile keeps four waves per SIMD resident, so that one wave's LDS gathers
// overlap another's FMAs.
template <int M, typename XT, typename AT, typename VT>
struct Lay {
  static constexpr int VS = (int)sizeof(VT);
  static constexpr int PT = 2048;                       // value bytes staged per tile (512 FP32, 1024 BF16)
  static constexpr int XRB = M * (int)sizeof(XT);       // bytes of one x row
  static constexpr int XSB = OddStride<XRB>::VALUE;     // staged x row stride
  static constexpr int XBB = 33 * XSB;                  // staged x block after one zero row
  static constexpr int CSB = OddStride<M * (int)sizeof(AT)>::VALUE;  // partial-sum row stride
  static constexpr int STAGE = 2 * PT + 2 * XBB;
  static constexpr int COMB = 64 * CSB;
  static constexpr int WAVE = ((STAGE > COMB ? STAGE : COMB) + 15) / 16 * 16;
  static constexpr int BYTES = 2 * WAVE;
  // x block loads: 16-byte pieces (vector form) or single elements
  static constexpr bool VEC = XRB % 16 == 0;
  static constexpr int CPR = VEC ? XRB / 16 : 1;        // pieces per row
  static constexpr int NXV = (32 * CPR + 63) / 64;      // vector loads per tile
  static constexpr int NXS = (32 * M + 63) / 64;        // element loads per tile
};

template <typename VT>
__device__ inline float lds_val(uint32_t addr);
template <>
__device__ inline float lds_val<float>(uint32_t addr) {
  return *(lds_ptr<const float>)(uintptr_t)addr;
}
template <>
__device__ inline float lds_val<uint16_t>(uint32_t addr) {
  return __uint_as_float((uint32_t)*(lds_ptr<const uint16_t>)(uintptr_t)addr << 16);
}

template <int M, typename XT, typename AT>
__device__ inline void lds_xrow(uint32_t addr, AT (&xr)[M]) {
  if constexpr ((M * sizeof(XT)) % 16 == 0) {
    constexpr int EPC = 16 / (int)sizeof(XT);
#pragma unroll
    for (int p = 0; p < M / EPC; ++p) {
      const v4u u = *(lds_ptr<const v4u>)(uintptr_t)(addr + 16 * p);
      const XT* e = reinterpret_cast<const XT*>(&u);
#pragma unroll
      for (int i = 0; i < EPC; ++i) xr[p * EPC + i] = (AT)e[i];
    }
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) xr[j] = (AT)((lds_ptr<const XT>)(uintptr_t)addr)[j];
  }
}

// One lane's walk over one half-tile: the set bits of `bits` in ascending order;
// the k-th value is va.get(k) and the x row of bit i sits at LDS byte address
// xb + i XSB.  The wave runs until its longest walk ends: a lane past its last
// entry finds no bit (index -1), reads the zero row kept just before the x
// block and the next value slot, and adds zero.  One entry of loads is in
// flight while the previous one is accumulated.
// where a lane's values come from: the staged copy in LDS (byte address of its
// first value) or, for tiles over the staged size, memory
template <typename VT>
struct LdsVals {
  uint32_t a;
  __device__ float get(int k) const { return lds_val<VT>(a + (uint32_t)k * (uint32_t)sizeof(VT)); }
  __device__ void adv(int k) { a += (uint32_t)k * (uint32_t)sizeof(VT); }
};
template <typename VT>
struct MemVals {
  const VT* p;
  __device__ float get(int k) const;
  __device__ void adv(int k) { p += k; }
};
template <>
__device__ inline float MemVals<float>::get(int k) const {
  return p[k];
}
template <>
__device__ inline float MemVals<uint16_t>::get(int k) const {
  return __uint_as_float((uint32_t)p[k] << 16);
}

template <int M, typename XT, typename AT, int XSB, typename Src>
__device__ inline void walk(uint32_t bits, Src va, uint32_t xb, AT (&a)[M]) {
  auto fma_row = [&](float v, const AT(&xr)[M]) {
    const AT w = (AT)v;
#pragma unroll
    for (int j = 0; j < M; ++j) a[j] += w * xr[j];
  };
  // index of the lowest set bit, -1 for none (the hardware's find-first-bit);
  // kept opaque so that the -1 is not folded into the address arithmetic
  auto first = [](uint32_t b) -> int {
    int i = __builtin_ctzg(b, -1);
    __asm__("" : "+v"(i));
    return i;
  };
  auto xaddr = [&](int i) -> uint32_t { return xb + (uint32_t)__mul24(i, XSB); };
  bool hA = bits != 0;
  if (!__builtin_amdgcn_ballot_w64(hA)) return;
  int i = first(bits);
  bits &= bits - 1u;
  float vA = va.get(0);
  AT xA[M];
  lds_xrow<M, XT, AT>(xaddr(i), xA);
  // two entries per trip and one exit test at the bottom (a wave whose longest
  // walk is odd accumulates one all-zero entry)
  bool more;
  do {
    const bool hB = bits != 0;
    i = first(bits);
    bits &= bits - 1u;
    const float vB = va.get(1);
    AT xB[M];
    lds_xrow<M, XT, AT>(xaddr(i), xB);
    __builtin_amdgcn_sched_barrier(0);
    fma_row(hA ? vA : 0.0f, xA);
    __builtin_amdgcn_sched_barrier(0);
    hA = bits != 0;
    i = first(bits);
    bits &= bits - 1u;
    vA = va.get(2);
    lds_xrow<M, XT, AT>(xaddr(i), xA);
    va.adv(2);
    __builtin_amdgcn_sched_barrier(0);
    fma_row(hB ? vB : 0.0f, xB);
    __builtin_amdgcn_sched_barrier(0);
    more = __builtin_amdgcn_ballot_w64(hA) != 0;
  } while (more);
}

// Registers holding the next step's data while the current step is walked.
template <int M, typename XT, typename AT, typename VT>
struct Stage {
  using L = Lay<M, XT, AT, VT>;
  uint32_t mask;                    // this lane's row (or column) mask
  v4u v[2][2];                      // [tile][first two 1 KB pieces of its values]
  v4u xv[2][L::NXV];                // [tile][x pieces] (vector form)
  typename XBits<XT>::T xs[2][L::NXS];  // [tile][x elements] (element form)
};

// The workgroup of block row J forms y_J completely with two waves:
//   wave 0 (direct):     the tiles (J, J') of block row J,
//                        y_J[r] += sum_c u_rc x_J'[c]        (lane r of its tile)
//   wave 1 (transposed): the tiles (I, J) of block column J, I <= J,
//                        y_J[c] += sum_r u_rc x_I[r]        (lane c of its tile)
// Both walk a bitmask with the values in the same order: the direct wave a row
// mask over the row-major values, the transposed wave a column mask over the
// column-major copy.  Each wave takes two tiles of its list per step, one per
// 32-lane half.  Lane q holds the metadata of list entry s0 + q (read out with
// readlane).  The values, masks and x blocks of the step after next are loaded
// into registers (buffer loads whose range is the tile or the x block, so that
// no load needs a branch) while the current step is walked from LDS.  The four
// partial sums of each row meet in LDS and y_J is written once with plain
// stores: no atomics and no clearing of Y.
template <int M, bool XV, typename XT, typename AT, typename VT>
__global__ __launch_bounds__(128) void k_spmm_sym(int64_t n, int64_t nbr,
                                                  const int64_t* __restrict__ tile_ptr,
                                                  const int64_t* __restrict__ col_ptr,
                                                  const int32_t* __restrict__ col_tiles,
                                                  const int32_t* __restrict__ col_brow,
                                                  const int32_t* __restrict__ tile_col,
                                                  const int64_t* __restrict__ tile_val,
                                                  const uint32_t* __restrict__ tile_mask,
                                                  const uint32_t* __restrict__ tile_cmask,
                                                  const VT* __restrict__ vals, const VT* __restrict__ tvals, int m,
                                                  int xlast, const XT* __restrict__ X, int64_t ldx,
                                                  AT* __restrict__ Y, int64_t ldy, int yvec) {
  using L = Lay<M, XT, AT, VT>;
  constexpr int VS = L::VS;
  constexpr int XS_ = (int)sizeof(XT);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool tr = wv == 1;
  // Workgroup i takes block row i, so that the 8 XCDs (dealt workgroups in turn)
  // stream neighbouring parts of the matrix.  An XCD-contiguous assignment buys
  // no L2 reuse here (an x block comes back only after ~170 block rows, tens of
  // MB of traffic) and measured ~10% slower.
  const int64_t J = blockIdx.x;
  if (J >= nbr) return;  // uniform over the workgroup

  const int half = lane >> 5, self = lane & 31;
  const uint32_t lds0 = (uint32_t)(uintptr_t)(lds_ptr<unsigned char>)lds_raw;
  const uint32_t wbase = lds0 + (uint32_t)wv * L::WAVE;
  const uint32_t P0 = wbase, X0 = wbase + 2 * L::PT;

  const uint32_t* __restrict__ mk = tr ? tile_cmask : tile_mask;
  const VT* __restrict__ vv = tr ? tvals : vals;
  const int64_t l0 = tr ? col_ptr[J] : tile_ptr[J];
  const int64_t len = (tr ? col_ptr[J + 1] : tile_ptr[J + 1]) - l0;
  const uint32_t xrow_bytes = (uint32_t)(ldx * XS_);

  // per-lane byte offsets of the x pieces (vector form): in the x block in
  // memory, and in the staged block (negative: no piece for this lane)
  uint32_t xo[L::NXV];
  int xl[L::NXV];
#pragma unroll
  for (int k = 0; k < L::NXV; ++k) {
    const int ch = 64 * k + lane;
    const bool ok = ch < 32 * L::CPR;
    xo[k] = ok ? (uint32_t)(ch / L::CPR) * xrow_bytes + (uint32_t)(ch % L::CPR) * 16 : OOB;
    xl[k] = ok ? (ch / L::CPR) * L::XSB + (ch % L::CPR) * 16 : -1;
  }
  // the zero row before each staged x block (read by lanes past their last entry)
  for (int i = lane; i < 2 * L::XSB / 4; i += 64)
    *(lds_ptr<uint32_t>)(uintptr_t)(X0 + (i < L::XSB / 4 ? 4 * i : L::XBB + 4 * (i - L::XSB / 4))) = 0u;

  AT a[M];
#pragma unroll
  for (int j = 0; j < M; ++j) a[j] = (AT)0;

  for (int64_t s0 = 0; s0 < len; s0 += 64) {
    // lane q: metadata of list entry s0 + q
    const int64_t e = s0 + lane;
    const int te = (e < len) ? (tr ? col_tiles[l0 + e] : (int)(l0 + e)) : -1;
    const int xe = (te >= 0) ? (tr ? col_brow[l0 + e] : tile_col[te]) : 0;
    const int64_t lo = (te >= 0) ? tile_val[te] : 0, hi = (te >= 0) ? tile_val[te + 1] : 0;
    const int v8 = (int)(lo >> 3);                 // value offset in units of 8 values
    const int nb = (int)(hi - lo) * VS;            // value bytes (a multiple of 16)
    const int cnt = (int)((len - s0) < 64 ? (len - s0) : 64);
    const int nsteps = (cnt + 1) / 2;

    // tile t (0, 1) of step q: list entry 2 q + t of this chunk
    struct Meta {
      int t[2], x[2], nb[2];
      int64_t vb[2];
    };
    auto meta = [&](int q) {
      Meta md;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        // entries past this chunk of 64 (read-ahead at its end) are absent
        const int qi = 2 * q + u;
        const bool in = qi < 64;
        md.t[u] = in ? rl(te, qi & 63) : -1;
        md.x[u] = in ? rl(xe, qi & 63) : 0;
        md.nb[u] = md.t[u] >= 0 ? rl(nb, qi & 63) : 0;
        md.vb[u] = in ? (int64_t)(uint32_t)rl(v8, qi & 63) << 3 : 0;
      }
      return md;
    };
    // Loads of one step into registers.  Nothing here consumes a loaded value,
    // so no wait follows the loads; for an absent tile the mask is read from
    // tile 0 and dropped when staged, and the other loads have an empty range.
    auto fetch = [&](Stage<M, XT, AT, VT>& sg, const Meta& md) {
      const int tm = half ? md.t[1] : md.t[0];
      sg.mask = __builtin_nontemporal_load(&mk[(int64_t)(tm >= 0 ? tm : 0) * 32 + self]);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const auto rv = buf_rsrc(vv + md.vb[u], (uint32_t)md.nb[u]);
        sg.v[u][0] = buf_ld16_nt(rv, (uint32_t)lane * 16);
        sg.v[u][1] = buf_ld16_nt(rv, (uint32_t)lane * 16 + 1024);
        // x block: rows up to n; in the last row the first xlast elements (m,
        // or the full width M when the caller guarantees whole rows)
        const int64_t row0 = (int64_t)md.x[u] * 32;
        const int64_t rows = md.t[u] >= 0 ? (n - row0 < 32 ? n - row0 : 32) : 0;
        const uint32_t xbytes = rows > 0 ? (uint32_t)(((rows - 1) * ldx + xlast) * XS_) : 0u;
        const auto rx = buf_rsrc(X + row0 * ldx, xbytes);
        if constexpr (XV) {
#pragma unroll
          for (int k = 0; k < L::NXV; ++k) sg.xv[u][k] = buf_ld16(rx, xo[k]);
        } else {
#pragma unroll
          for (int k = 0; k < L::NXS; ++k) {
            const int el = 64 * k + lane;
            const int r = el / M, c = el % M;
            const uint32_t off = (el < 32 * M && c < m) ? (uint32_t)r * xrow_bytes + (uint32_t)(c * XS_) : OOB;
            sg.xs[u][k] = XBits<XT>::load(rx, off);
          }
        }
      }
    };
    // One step: stage the registers into LDS, refill them with step q + 2 (two
    // steps of walking cover the memory latency), walk.  Refills and steps past
    // the end of the list are issued anyway, as empty ones: with no branch
    // around them, each wait for a step's loads leaves the other step's loads
    // in flight.
    auto step = [&](Stage<M, XT, AT, VT>& sg, Meta& md, int q) {
      const uint32_t bits = (half ? md.t[1] : md.t[0]) >= 0 ? sg.mask : 0u;
      const int nb0 = md.nb[0], nb1 = md.nb[1];
      const int64_t vb0 = md.vb[0], vb1 = md.vb[1];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const uint32_t pt = P0 + u * L::PT;
        *(lds_ptr<v4u>)(uintptr_t)(pt + lane * 16) = sg.v[u][0];
        *(lds_ptr<v4u>)(uintptr_t)(pt + 1024 + lane * 16) = sg.v[u][1];
        const uint32_t xt = X0 + u * L::XBB + L::XSB;
        if constexpr (XV) {
#pragma unroll
          for (int k = 0; k < L::NXV; ++k)
            if (32 * L::CPR % 64 == 0 || xl[k] >= 0) *(lds_ptr<v4u>)(uintptr_t)(xt + xl[k]) = sg.xv[u][k];
        } else {
#pragma unroll
          for (int k = 0; k < L::NXS; ++k) {
            const int el = 64 * k + lane;
            if (32 * M % 64 == 0 || el < 32 * M)
              *(lds_ptr<typename XBits<XT>::T>)(uintptr_t)(xt + (el / M) * L::XSB + (el % M) * XS_) = sg.xs[u][k];
          }
        }
      }
      md = meta(q + 2);
      fetch(sg, md);
      wave_sync_lds();
      // this lane's first value: exclusive prefix of the mask popcounts in its half
      const uint32_t c0 = (uint32_t)__popc(bits);
      const uint32_t off = incl_scan32(c0) - c0;
      const uint32_t xb = X0 + half * L::XBB + L::XSB;
      if (nb0 > L::PT || nb1 > L::PT) {
        // a tile over the staged size in this step: values from memory.  The
        // walk's last read-ahead is never used; waiting for every load here
        // keeps it from holding up the next step (vmcnt(0), other counters free)
        walk<M, XT, AT, L::XSB>(bits, MemVals<VT>{vv + (half ? vb1 : vb0) + off}, xb, a);
        __builtin_amdgcn_s_waitcnt(0x0F70);
      } else {
        walk<M, XT, AT, L::XSB>(bits, LdsVals<VT>{P0 + half * L::PT + off * VS}, xb, a);
      }
      wave_sync_lds();
    };

    Stage<M, XT, AT, VT> sgA, sgB;
    Meta mA = meta(0), mB = meta(1);
    fetch(sgA, mA);
    fetch(sgB, mB);
    for (int q = 0; q < nsteps; q += 2) {
      step(sgA, mA, q);
      step(sgB, mB, q + 1);
    }
  }
  // y_J: the four partial sums of each row (two halves of each wave) meet in LDS
  {
    const uint32_t cb = wbase + (uint32_t)(half * 32 + self) * L::CSB;
#pragma unroll
    for (int j = 0; j < M; ++j) ((lds_ptr<AT>)(uintptr_t)cb)[j] = a[j];
  }
  __syncthreads();
  if (threadIdx.x < 32) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
      AT s[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
        s[p] = ((lds_ptr<const AT>)(uintptr_t)(lds0 + (p >> 1) * L::WAVE + ((p & 1) * 32 + self) * L::CSB))[j];
      a[j] = (s[0] + s[1]) + (s[2] + s[3]);
    }
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

// ---------------------------------------------------------------------------
// the product on matrix cores (FP32 values; FP32 x and FP32 sums on
// v_mfma_f32_16x16x4f32, or FP64 / FP32 x and FP64 sums on v_mfma_f64_16x16x4f64)
// ---------------------------------------------------------------------------
// The walk above gathers a whole x row from LDS for every stored entry (m * 4
// bytes per entry and lane, twice that for FP64 x).  At m = 16 that kept LDS
// busy for ~90% of the kernel, a third of those cycles bank conflicts, while
// its memory traffic (4.7 TB/s) stayed below what random 2 KB block reads
// sustain (6.2 TB/s from HBM, 7.6 TB/s from the 256 MB MALL).  Here each
// tile (one wave, 64 lanes) is applied as a dense 32 x 32 by 32 x 16 product on
// 16 MFMAs of shape 16x16x4: the tile's packed values are staged in LDS, each
// lane picks the (at most) 16 entries of the dense tile that it feeds to the
// matrix core, and the x block goes from memory straight into the B operands.
// Lane l (i = l % 16, kq = l / 16) feeds, in step s of half h, the entry
// (16 h + i, 4 s + kq) of the tile and the x element (4 s + kq, i); the
// accumulator element q of lane l is then y row 16 h + 4 kq + q (FP32 MFMA) or
// 16 h + 4 q + kq (FP64 MFMA), column i.
// Workgroup J has two waves, which share out the direct tiles of block row J
// and the transposed tiles of block column J; their sums meet in LDS at the end.
using f32x4 = __attribute__((ext_vector_type(4))) float;
using f64x4 = __attribute__((ext_vector_type(4))) double;

constexpr int MMA_STAGE = 4096 + 16;  // one tile's values (up to 1024) and a read-past slot
// Narrowest FP32 block applied on matrix cores; narrower ones walk the tiles.
// Measured at n = 2,097,152 (24 tiles of density 0.3 per block row), medians
// of one run: the walk takes 1.58 / 1.97 / 2.00 / 1.81 / 1.87 ms at
// m = 8 / 9 / 10 / 12 / 16 and this kernel 1.74 / 1.81 / 1.82 / 1.74 / 1.86 ms;
// its time hardly depends on m (each tile costs 16 MFMAs and 16 operand picks
// per lane whatever the width).
constexpr int MMA_MIN_WIDTH = 9;
// the same for FP64 sums (FP64 x, or FP32 x widened exactly)
constexpr int MMA64_MIN_WIDTH = 9;

__device__ inline uint32_t scan16(uint32_t x) {  // inclusive prefix sum in each row of 16 lanes
  x += dpp_u32<0x111, 0xf>(x);
  x += dpp_u32<0x112, 0xf>(x);
  x += dpp_u32<0x114, 0xf>(x);
  x += dpp_u32<0x118, 0xf>(x);
  return x;
}

template <typename XT>
struct MmaStage {
  uint32_t mlo, mhi;                 // masks of rows i and 16 + i
  v4u v[2];                          // the first 2 KB of the tile's packed values (512 FP32)
  typename XBits<XT>::T x[8];        // x elements (4 s + kq, i), raw bits
};

template <typename AT>
struct Mma;
template <>
struct Mma<float> {
  using V = f32x4;
  static __device__ V op(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ int row(int kq, int q) { return 4 * kq + q; }
};
template <>
struct Mma<double> {
  using V = f64x4;
  static __device__ V op(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ int row(int kq, int q) { return 4 * q + kq; }
};
template <typename XT>
__device__ inline XT xval(typename XBits<XT>::T b);
template <>
__device__ inline float xval<float>(uint32_t b) {
  return __uint_as_float(b);
}
template <>
__device__ inline double xval<double>(v2u b) {
  return __builtin_bit_cast(double, b);
}

template <typename XT, typename AT>
__global__ __launch_bounds__(128) void k_spmm_sym_mma(int64_t n, const int64_t* __restrict__ tile_ptr,
                                                      const int64_t* __restrict__ col_ptr,
                                                      const int32_t* __restrict__ col_tiles,
                                                      const int32_t* __restrict__ col_brow,
                                                      const int32_t* __restrict__ tile_col,
                                                      const int64_t* __restrict__ tile_val,
                                                      const uint32_t* __restrict__ tile_mask,
                                                      const uint32_t* __restrict__ tile_cmask,
                                                      const float* __restrict__ vals, const float* __restrict__ tvals,
                                                      int m, int xlast, const XT* __restrict__ X, int64_t ldx,
                                                      AT* __restrict__ Y, int64_t ldy) {
  using MM = Mma<AT>;
  using Acc = typename MM::V;
  constexpr int XS_ = (int)sizeof(XT);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool tr = wv == 1;
  const int64_t J = blockIdx.x;
  const int i16 = lane & 15, kq = lane >> 4;
  const uint32_t lds0 = (uint32_t)(uintptr_t)(lds_ptr<unsigned char>)lds_raw;
  const uint32_t P = lds0 + (uint32_t)wv * MMA_STAGE;

  // Both waves take entries of one list, the direct tiles of block row J and
  // then the transposed tiles of block column J, wave w the entries w, w + 2, ...
  // (the two parts differ in length from row to row; split this way the waves
  // finish together).
  const int64_t d0 = tile_ptr[J], dlen = tile_ptr[J + 1] - d0;
  const int64_t t0 = col_ptr[J], tlen = col_ptr[J + 1] - t0;
  const int64_t len = (dlen + tlen - wv + 1) / 2;  // entries of this wave
  // byte offsets of this lane's x elements in a block: rows 4 s + kq, column i
  // (columns at or past m read nothing)
  uint32_t xo[8];
#pragma unroll
  for (int s = 0; s < 8; ++s)
    xo[s] = i16 < m ? (uint32_t)(((int64_t)(4 * s + kq) * ldx + i16) * XS_) : OOB;

  Acc acc[2] = {Acc{0, 0, 0, 0}, Acc{0, 0, 0, 0}};

  for (int64_t s0 = 0; s0 < len; s0 += 64) {
    const int64_t e = s0 + lane;               // this wave's entry
    const int64_t g = 2 * e + wv;              // its place in the joint list
    const bool kt = g >= dlen;                 // a transposed tile
    const int te = (e < len) ? (kt ? col_tiles[t0 + g - dlen] : (int)(d0 + g)) : -1;
    const int xe = (te >= 0) ? (kt ? col_brow[t0 + g - dlen] : tile_col[te]) : 0;
    const int64_t lo = (te >= 0) ? tile_val[te] : 0, hi = (te >= 0) ? tile_val[te + 1] : 0;
    const int v8 = (int)(lo >> 3);
    const int nb = (int)(hi - lo) * 4;
    const int ktr = kt ? 1 : 0;
    const int cnt = (int)((len - s0) < 64 ? (len - s0) : 64);

    struct Meta {
      int t, x, nb;
      bool tr;
      int64_t vb;
    };
    auto meta = [&](int q) {
      Meta md;
      const bool in = q < 64;
      md.t = in ? rl(te, q & 63) : -1;
      md.x = in ? rl(xe, q & 63) : 0;
      md.nb = md.t >= 0 ? rl(nb, q & 63) : 0;
      md.tr = in ? rl(ktr, q & 63) != 0 : false;
      md.vb = in ? (int64_t)(uint32_t)rl(v8, q & 63) << 3 : 0;
      return md;
    };
    // loads of one tile into registers (an absent tile: masks of tile 0, dropped
    // later, and empty ranges for the values and the x block)
    auto fetch = [&](MmaStage<XT>& sg, const Meta& md) {
      // row masks and row-major values, or column masks and the column-major copy
      const uint32_t* __restrict__ mk = md.tr ? tile_cmask : tile_mask;
      const float* __restrict__ vv = md.tr ? tvals : vals;
      const int64_t tm = (int64_t)(md.t >= 0 ? md.t : 0) * 32;
      sg.mlo = __builtin_nontemporal_load(&mk[tm + i16]);
      sg.mhi = __builtin_nontemporal_load(&mk[tm + 16 + i16]);
      const auto rv = buf_rsrc(vv + md.vb, (uint32_t)md.nb);
#pragma unroll
      for (int u = 0; u < 2; ++u) sg.v[u] = buf_ld16_nt(rv, (uint32_t)lane * 16 + 1024 * u);
      const int64_t row0 = (int64_t)md.x * 32;
      const int64_t rows = md.t >= 0 ? (n - row0 < 32 ? n - row0 : 32) : 0;
      const uint32_t xbytes = rows > 0 ? (uint32_t)(((rows - 1) * ldx + xlast) * XS_) : 0u;
      const auto rx = buf_rsrc(X + row0 * ldx, xbytes);
#pragma unroll
      for (int s = 0; s < 8; ++s) sg.x[s] = XBits<XT>::load(rx, xo[s]);
    };
    // One tile: stage its values, build the A operands, multiply, and only then
    // refill the registers with tile q + 2 (the MFMAs read the x block straight
    // from them; a refill before would need a copy, and a copy waits for the
    // loads in flight).
    auto step = [&](MmaStage<XT>& sg, Meta& md, int q) {
      const bool live = md.t >= 0;
      const uint32_t mlo = live ? sg.mlo : 0u, mhi = live ? sg.mhi : 0u;
#pragma unroll
      for (int u = 0; u < 2; ++u) *(lds_ptr<v4u>)(uintptr_t)(P + 1024 * u + lane * 16) = sg.v[u];
      if (md.nb > 2048) {
        // a tile of more than 512 entries: the rest of its values straight from
        // memory (this waits for every load in flight; such tiles are rare where
        // the product is bandwidth-bound)
        const auto rv = buf_rsrc((md.tr ? tvals : vals) + md.vb, (uint32_t)md.nb);
#pragma unroll
        for (int u = 2; u < 4; ++u)
          *(lds_ptr<v4u>)(uintptr_t)(P + 1024 * u + lane * 16) = buf_ld16_nt(rv, (uint32_t)lane * 16 + 1024 * u);
      }
      wave_sync_lds();
      // first packed value of rows i and 16 + i: exclusive prefix of the row popcounts
      const uint32_t clo = (uint32_t)__popc(mlo), chi = (uint32_t)__popc(mhi);
      const uint32_t slo = scan16(clo), shi = scan16(chi);
      const uint32_t tot = (uint32_t)rl((int)slo, 15);
      uint32_t idx[2] = {slo - clo, tot + shi - chi};
      const uint32_t mh[2] = {mlo, mhi};
      const uint32_t below = (1u << kq) - 1u;
      float a[2][8];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        idx[h] += (uint32_t)__popc(mh[h] & below);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          // bits of columns 4 s + kq .. + 3; the value slot is read either way
          // and kept under an all-ones mask when the first of them is set
          const uint32_t nib = __builtin_amdgcn_ubfe(mh[h], (uint32_t)(4 * s + kq), 4u);
          const uint32_t keep = (uint32_t)__builtin_amdgcn_sbfe((int)nib, 0u, 1u);
          const uint32_t v = *(lds_ptr<const uint32_t>)(uintptr_t)(P + idx[h] * 4);
          a[h][s] = __uint_as_float(v & keep);
          idx[h] += (uint32_t)__popc(nib);
        }
      }
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const AT xs = (AT)xval<XT>(sg.x[s]);
        acc[0] = MM::op((AT)a[0][s], xs, acc[0]);
        acc[1] = MM::op((AT)a[1][s], xs, acc[1]);
      }
      wave_sync_lds();
      md = meta(q + 2);
      fetch(sg, md);
    };

    MmaStage<XT> sgA, sgB;
    Meta mA = meta(0), mB = meta(1);
    fetch(sgA, mA);
    fetch(sgB, mB);
    for (int q = 0; q < cnt; q += 2) {
      step(sgA, mA, q);
      step(sgB, mB, q + 1);
    }
  }
  // y_J = direct + transposed partial sums
  lds_ptr<AT> cb = (lds_ptr<AT>)(uintptr_t)(lds0 + MMA_STAGE);
  if (tr) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) cb[(h * 4 + q) * 64 + lane] = acc[h][q];
  }
  __syncthreads();
  if (!tr && i16 < m) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = J * 32 + 16 * h + MM::row(kq, q);
        if (row < n) Y[row * ldy + i16] = acc[h][q] + cb[(h * 4 + q) * 64 + lane];
      }
  }
}

template <typename XT, typename AT>
hyeig_status launch_mma(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                        int xlast) {
  static_assert(8 * 64 * sizeof(AT) <= MMA_STAGE, "partial sums fit the second wave's staging area");
  if (H->nbr > (int64_t)INT_MAX) return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: matrix too large");
  if (ldx > (int64_t)(INT_MAX / 64) / (int64_t)sizeof(XT))
    return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: leading dimension of X too large");
  hipLaunchKernelGGL((k_spmm_sym_mma<XT, AT>), dim3((unsigned)H->nbr), dim3(128), (size_t)2 * MMA_STAGE,
                     ctx->stream, H->n, H->tile_ptr, H->col_ptr, H->col_tiles, H->col_brow, H->tile_col, H->tile_val,
                     H->tile_mask, H->tile_cmask, H->vals, H->tvals, m, xlast, X, ldx, Y, ldy);
  return hip_err(ctx, hipGetLastError(), "k_spmm_sym_mma launch");
}

// ---------------------------------------------------------------------------
// the product on matrix cores with the operands scattered from stored slots
// ---------------------------------------------------------------------------
// k_spmm_sym_mma above spends about 80 VALU instructions per tile and lane on
// picking its 16 operands out of the packed values with the row masks, and on
// gfx950 VALU and matrix-core cycles add up (they do not overlap, within a
// wave or across waves).  Here every stored value carries its slot in a dense
// operand layout (pos for vals, tpos for the column-major copy tvals; built
// once from the masks by k_tile_pos): the wave clears a dense 32 x 32 tile in
// LDS, writes each value to its slot (two VALU instructions per value), and
// reads its MFMA operands back with 16-byte loads.  The masks are not read.
// Dense layout: entry (row, col) of the operand tile (row = 16 h + i, the MFMA
// row; col = 4 s + kq, its k index) sits at element
//   h * 576 + i * 36 + kq * 8 + s,
// so that lane (i, kq) finds its eight operands of half h consecutive; rows
// are 36 elements apart so that the 16-byte reads of a wave spread over the
// LDS banks.  A stored slot is that element + 4; slot 0 is a dummy element
// (padding values between tiles write their zero there).
constexpr int MMA2_RS = 36;                    // row stride of the dense operand tile (elements)
constexpr int MMA2_HALF = 16 * MMA2_RS;        // elements of one 16-row half
constexpr int MMA2_ELEMS = 2 * MMA2_HALF;      // 1152
constexpr int MMA2_DUMMY = 4;                  // slot offset: slots 0..3 lie before the tile

__device__ inline uint32_t mma2_slot(int row, int col) {
  return (uint32_t)(MMA2_DUMMY + (row >> 4) * MMA2_HALF + (row & 15) * MMA2_RS + (col & 3) * 8 + (col >> 2));
}

// Slots of every stored value, one wave per tile: lane r < 32 walks row r of the
// row masks (values packed row-major: row r's values from the exclusive prefix
// of the row popcounts, columns ascending) and lane c < 32 column c of the
// column masks (the column-major copy, diagonal excluded like the masks; as
// operand of the transposed half, entry (r, c) of U is entry (c, r)).
// Entries not written (padding between tiles) keep slot 0.
__global__ __launch_bounds__(256) void k_tile_pos(int64_t ntiles, const int64_t* __restrict__ tile_val,
                                                  const uint32_t* __restrict__ tile_mask,
                                                  const uint32_t* __restrict__ tile_cmask, uint16_t* __restrict__ pos,
                                                  uint16_t* __restrict__ tpos) {
  const int lane = threadIdx.x & 63, c = lane & 31;
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const bool live = t < ntiles;
  const uint32_t rm = live ? tile_mask[t * 32 + c] : 0u;
  const uint32_t cm = live ? tile_cmask[t * 32 + c] : 0u;
  uint32_t tot;
  const uint32_t ro = excl_scan32((uint32_t)__popc(rm), lane, &tot);
  const uint32_t co = excl_scan32((uint32_t)__popc(cm), lane, &tot);
  if (!live || lane >= 32) return;
  const int64_t vb = tile_val[t];
  uint32_t bits = rm, k = 0;
  while (bits) {
    const int col = __builtin_ctz(bits);
    bits &= bits - 1u;
    pos[vb + ro + k] = (uint16_t)mma2_slot(c, col);
    ++k;
  }
  bits = cm;
  k = 0;
  while (bits) {
    const int row = __builtin_ctz(bits);
    bits &= bits - 1u;
    tpos[vb + co + k] = (uint16_t)mma2_slot(c, row);
    ++k;
  }
}

__device__ inline v2u buf_ld8_nt(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 2);
}

template <typename XT>
struct Mma2Stage {
  v4u v[2];                          // values 4 l .. 4 l + 3 and 256 + 4 l .. (the first 512)
  v2u p[2];                          // their slots (uint16 pairs)
  typename XBits<XT>::T x[8];        // x elements (4 s + kq, i), raw bits
};

template <typename AT>
struct Mma2Lay {
  static constexpr int ES = (int)sizeof(AT);
  static constexpr int TILE = ((MMA2_DUMMY + MMA2_ELEMS) * ES + 15) / 16 * 16;  // LDS bytes per wave
  static constexpr int ZCH = MMA2_ELEMS * ES / 16;                              // 16-byte chunks to clear
};

// one value into its slot of the dense tile (FP32 bits, or widened to FP64)
template <typename AT>
__device__ inline void put_slot(uint32_t P, uint32_t slot, uint32_t bits);
template <>
__device__ inline void put_slot<float>(uint32_t P, uint32_t slot, uint32_t bits) {
  *(lds_ptr<uint32_t>)(uintptr_t)(P + slot * 4u) = bits;
}
template <>
__device__ inline void put_slot<double>(uint32_t P, uint32_t slot, uint32_t bits) {
  *(lds_ptr<double>)(uintptr_t)(P + slot * 8u) = (double)__uint_as_float(bits);
}

template <typename AT>
__device__ inline void scatter4(uint32_t P, const v4u& v, const v2u& p) {
  put_slot<AT>(P, p[0] & 0xFFFFu, v[0]);
  put_slot<AT>(P, p[0] >> 16, v[1]);
  put_slot<AT>(P, p[1] & 0xFFFFu, v[2]);
  put_slot<AT>(P, p[1] >> 16, v[3]);
}

template <typename XT, typename AT>
__global__ __launch_bounds__(128) void k_spmm_sym_mma2(int64_t n, const int64_t* __restrict__ tile_ptr,
                                                       const int64_t* __restrict__ col_ptr,
                                                       const int32_t* __restrict__ col_tiles,
                                                       const int32_t* __restrict__ col_brow,
                                                       const int32_t* __restrict__ tile_col,
                                                       const int64_t* __restrict__ tile_val,
                                                       const float* __restrict__ vals, const float* __restrict__ tvals,
                                                       const uint16_t* __restrict__ pos,
                                                       const uint16_t* __restrict__ tpos, int m, int xlast,
                                                       const XT* __restrict__ X, int64_t ldx, AT* __restrict__ Y,
                                                       int64_t ldy) {
  using MM = Mma<AT>;
  using Acc = typename MM::V;
  using L = Mma2Lay<AT>;
  constexpr int ES = L::ES;
  constexpr int XS_ = (int)sizeof(XT);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool tr = wv == 1;
  const int64_t J = blockIdx.x;
  const int i16 = lane & 15, kq = lane >> 4;
  const uint32_t lds0 = (uint32_t)(uintptr_t)(lds_ptr<unsigned char>)lds_raw;
  const uint32_t P = lds0 + (uint32_t)wv * L::TILE;        // slot 0 (dummy)
  const uint32_t D = P + MMA2_DUMMY * ES;                  // the dense tile
  // this lane's operands of half h: 8 consecutive elements from here
  const uint32_t opnd = D + (uint32_t)(i16 * MMA2_RS + kq * 8) * ES;

  // the joint list of block row J (direct tiles, then transposed ones), wave w
  // taking entries w, w + 2, ... (see k_spmm_sym_mma)
  const int64_t d0 = tile_ptr[J], dlen = tile_ptr[J + 1] - d0;
  const int64_t t0 = col_ptr[J], tlen = col_ptr[J + 1] - t0;
  const int64_t len = (dlen + tlen - wv + 1) / 2;
  uint32_t xo[8];
#pragma unroll
  for (int s = 0; s < 8; ++s)
    xo[s] = i16 < m ? (uint32_t)(((int64_t)(4 * s + kq) * ldx + i16) * XS_) : OOB;

  Acc acc[2] = {Acc{0, 0, 0, 0}, Acc{0, 0, 0, 0}};

  for (int64_t s0 = 0; s0 < len; s0 += 64) {
    const int64_t e = s0 + lane;
    const int64_t g = 2 * e + wv;
    const bool kt = g >= dlen;
    const int te = (e < len) ? (kt ? col_tiles[t0 + g - dlen] : (int)(d0 + g)) : -1;
    const int xe = (te >= 0) ? (kt ? col_brow[t0 + g - dlen] : tile_col[te]) : 0;
    const int64_t lo = (te >= 0) ? tile_val[te] : 0, hi = (te >= 0) ? tile_val[te + 1] : 0;
    const int v8 = (int)(lo >> 3);
    const int nb = (int)(hi - lo) * 4;
    const int ktr = kt ? 1 : 0;
    const int cnt = (int)((len - s0) < 64 ? (len - s0) : 64);

    struct Meta {
      int t, x, nb;
      bool tr;
      int64_t vb;
    };
    auto meta = [&](int q) {
      Meta md;
      const bool in = q < 64;
      md.t = in ? rl(te, q & 63) : -1;
      md.x = in ? rl(xe, q & 63) : 0;
      md.nb = md.t >= 0 ? rl(nb, q & 63) : 0;
      md.tr = in ? rl(ktr, q & 63) != 0 : false;
      md.vb = in ? (int64_t)(uint32_t)rl(v8, q & 63) << 3 : 0;
      return md;
    };
    // loads of one tile: its first 512 values and their slots, and its x block
    // (an absent tile: empty ranges, so zeros into the dummy slot)
    auto fetch = [&](Mma2Stage<XT>& sg, const Meta& md) {
      const float* __restrict__ vv = md.tr ? tvals : vals;
      const uint16_t* __restrict__ pp = md.tr ? tpos : pos;
      const auto rv = buf_rsrc(vv + md.vb, (uint32_t)md.nb);
      const auto rp = buf_rsrc(pp + md.vb, (uint32_t)md.nb / 2u);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        sg.v[u] = buf_ld16_nt(rv, (uint32_t)lane * 16 + 1024 * u);
        sg.p[u] = buf_ld8_nt(rp, (uint32_t)lane * 8 + 512 * u);
      }
      const int64_t row0 = (int64_t)md.x * 32;
      const int64_t rows = md.t >= 0 ? (n - row0 < 32 ? n - row0 : 32) : 0;
      const uint32_t xbytes = rows > 0 ? (uint32_t)(((rows - 1) * ldx + xlast) * XS_) : 0u;
      const auto rx = buf_rsrc(X + row0 * ldx, xbytes);
#pragma unroll
      for (int s = 0; s < 8; ++s) sg.x[s] = XBits<XT>::load(rx, xo[s]);
    };
    auto step = [&](Mma2Stage<XT>& sg, Meta& md, int q) {
      // clear the dense tile, write the values to their slots
#pragma unroll
      for (int j = 0; j < (L::ZCH + 63) / 64; ++j)
        if ((L::ZCH % 64) == 0 || lane + 64 * j < L::ZCH)
          *(lds_ptr<v4u>)(uintptr_t)(D + 16u * (uint32_t)(lane + 64 * j)) = v4u{0u, 0u, 0u, 0u};
#pragma unroll
      for (int u = 0; u < 2; ++u) scatter4<AT>(P, sg.v[u], sg.p[u]);
      if (md.nb > 2048) {
        // values 512 .. 1023 of a tile of more than 512 entries, straight from
        // memory (this waits for every load in flight; such tiles are rare)
        const auto rv = buf_rsrc((md.tr ? tvals : vals) + md.vb, (uint32_t)md.nb);
        const auto rp = buf_rsrc((md.tr ? tpos : pos) + md.vb, (uint32_t)md.nb / 2u);
#pragma unroll
        for (int u = 2; u < 4; ++u)
          scatter4<AT>(P, buf_ld16_nt(rv, (uint32_t)lane * 16 + 1024 * u), buf_ld8_nt(rp, (uint32_t)lane * 8 + 512 * u));
      }
      wave_sync_lds();
      AT a[2][8];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < 8 * ES / 16; ++c) {
          const v4u w = *(lds_ptr<const v4u>)(uintptr_t)(opnd + (uint32_t)(h * MMA2_HALF * ES + 16 * c));
          const AT* e4 = reinterpret_cast<const AT*>(&w);
#pragma unroll
          for (int z = 0; z < 16 / ES; ++z) a[h][c * (16 / ES) + z] = e4[z];
        }
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const AT xs = (AT)xval<XT>(sg.x[s]);
        acc[0] = MM::op(a[0][s], xs, acc[0]);
        acc[1] = MM::op(a[1][s], xs, acc[1]);
      }
      wave_sync_lds();
      md = meta(q + 2);
      fetch(sg, md);
    };

    Mma2Stage<XT> sgA, sgB;
    Meta mA = meta(0), mB = meta(1);
    fetch(sgA, mA);
    fetch(sgB, mB);
    for (int q = 0; q < cnt; q += 2) {
      step(sgA, mA, q);
      step(sgB, mB, q + 1);
    }
  }
  // y_J = direct + transposed partial sums
  lds_ptr<AT> cb = (lds_ptr<AT>)(uintptr_t)(lds0 + L::TILE);
  if (tr) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) cb[(h * 4 + q) * 64 + lane] = acc[h][q];
  }
  __syncthreads();
  if (!tr && i16 < m) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = J * 32 + 16 * h + MM::row(kq, q);
        if (row < n) Y[row * ldy + i16] = acc[h][q] + cb[(h * 4 + q) * 64 + lane];
      }
  }
}

// the slots of the matrix-core product, built once per matrix (false when they
// cannot be allocated: the mask-based kernel runs instead)
bool mma2_ready(hyeig_ctx* ctx, const hyeig_mat* Hc) {
  hyeig_mat* H = const_cast<hyeig_mat*>(Hc);
  if (H->pos) return true;
  if (H->pos_tried) return false;
  H->pos_tried = true;
  const size_t bytes = sizeof(uint16_t) * (size_t)(H->nvals + VAL_PAD);
  if (hipMalloc((void**)&H->pos, bytes) != hipSuccess) {
    H->pos = nullptr;
    (void)hipGetLastError();
    return false;
  }
  if (hipMalloc((void**)&H->tpos, bytes) != hipSuccess) {
    (void)hipFree(H->pos);
    H->pos = H->tpos = nullptr;
    (void)hipGetLastError();
    return false;
  }
  if (hipMemsetAsync(H->pos, 0, bytes, ctx->stream) != hipSuccess ||
      hipMemsetAsync(H->tpos, 0, bytes, ctx->stream) != hipSuccess)
    return false;
  const int64_t blocks = (H->ntiles + 3) / 4;
  if (blocks > 0)
    hipLaunchKernelGGL(k_tile_pos, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, H->ntiles, H->tile_val,
                       H->tile_mask, H->tile_cmask, H->pos, H->tpos);
  return hipGetLastError() == hipSuccess;
}

template <typename XT, typename AT>
hyeig_status launch_mma2(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                         int xlast) {
  using L = Mma2Lay<AT>;
  static_assert(8 * 64 * sizeof(AT) <= L::TILE, "partial sums fit the second wave's tile");
  if (H->nbr > (int64_t)INT_MAX) return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: matrix too large");
  if (ldx > (int64_t)(INT_MAX / 64) / (int64_t)sizeof(XT))
    return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: leading dimension of X too large");
  hipLaunchKernelGGL((k_spmm_sym_mma2<XT, AT>), dim3((unsigned)H->nbr), dim3(128), (size_t)2 * L::TILE, ctx->stream,
                     H->n, H->tile_ptr, H->col_ptr, H->col_tiles, H->col_brow, H->tile_col, H->tile_val, H->vals,
                     H->tvals, H->pos, H->tpos, m, xlast, X, ldx, Y, ldy);
  return hip_err(ctx, hipGetLastError(), "k_spmm_sym_mma2 launch");
}

template <typename XT, typename AT>
hyeig_status launch_mma_any(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                            int xlast) {
  if (mma2_ready(ctx, H)) return launch_mma2<XT, AT>(ctx, H, m, X, ldx, Y, ldy, xlast);
  return launch_mma<XT, AT>(ctx, H, m, X, ldx, Y, ldy, xlast);
}

template <int M, bool XV, typename XT, typename AT, typename VT>
hyeig_status launch_kernel(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                           const VT* vals, const VT* tvals, int64_t blocks, bool yvec, int xlast) {
  auto kern = k_spmm_sym<M, XV, XT, AT, VT>;
  const size_t lds = (size_t)Lay<M, XT, AT, VT>::BYTES;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(128), lds, ctx->stream, H->n,
                     H->nbr, H->tile_ptr, H->col_ptr, H->col_tiles, H->col_brow, H->tile_col, H->tile_val,
                     H->tile_mask, H->tile_cmask, vals, tvals, m, xlast, X, ldx, Y, ldy, (int)yvec);
  return hip_err(ctx, hipGetLastError(), "k_spmm_sym launch");
}

template <int M, typename XT, typename AT, typename VT>
hyeig_status run_spmm(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                      const VT* vals, const VT* tvals, bool xfull) {
  using L = Lay<M, XT, AT, VT>;
  const int64_t groups = H->nbr;
  if (groups == 0) return HYEIG_OK;
  const int64_t blocks = groups;
  if (blocks > (int64_t)INT_MAX) return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: matrix too large");
  // 32-bit buffer offsets within one x block
  if (ldx > (int64_t)(INT_MAX / 64) / (int64_t)sizeof(XT))
    return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: leading dimension of X too large");
  // 16-byte pieces of x rows when rows start 16-byte aligned and the m used
  // columns end on a piece boundary (a piece is then wholly inside or wholly
  // outside the buffer; pieces past column m feed only outputs that are not
  // stored), or when the caller guarantees rows of ldx >= M readable elements
  // (xfull); y pieces when the rows are exactly m = M wide
  const bool xvec = (ldx * (int64_t)sizeof(XT)) % 16 == 0 && ((uintptr_t)X & 15) == 0 &&
                    ((m * (int64_t)sizeof(XT)) % 16 == 0 || (xfull && ldx >= M));
  const bool yvec = m == M && (ldy * (int64_t)sizeof(AT)) % 16 == 0 && ((uintptr_t)Y & 15) == 0;
  const int xlast = (xfull && ldx >= M) ? M : m;
  if constexpr (L::VEC) {
    if (xvec) return launch_kernel<M, true>(ctx, H, m, X, ldx, Y, ldy, vals, tvals, blocks, yvec, xlast);
  }
  return launch_kernel<M, false>(ctx, H, m, X, ldx, Y, ldy, vals, tvals, blocks, yvec, xlast);
}

template <typename XT, typename AT, typename VT>
hyeig_status spmm_width(hyeig_ctx* ctx, const hyeig_mat* H, int m, const XT* X, int64_t ldx, AT* Y, int64_t ldy,
                        const VT* vals, const VT* tvals, bool xfull) {
  if (m <= 1) return run_spmm<1, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals, tvals, xfull);
  if (m <= 2) return run_spmm<2, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals, tvals, xfull);
  if (m <= 4) return run_spmm<4, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals, tvals, xfull);
  if (m <= 8) return run_spmm<8, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals, tvals, xfull);
  if (m <= 12) return run_spmm<12, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals, tvals, xfull);
  if (m <= 16) return run_spmm<16, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals, tvals, xfull);
  return run_spmm<32, XT, AT, VT>(ctx, H, m, X, ldx, Y, ldy, vals, tvals, xfull);
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

hyeig_status launch_tile_tvals(hyeig_ctx* ctx, hyeig_mat* M) {
  const int64_t blocks = (M->ntiles + 3) / 4;
  if (blocks == 0) return HYEIG_OK;
  hipLaunchKernelGGL(k_tile_tvals, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, M->ntiles, M->tile_val,
                     M->tile_mask, M->tile_cmask, M->vals, M->tvals);
  return hip_err(ctx, hipGetLastError(), "k_tile_tvals launch");
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

bool spmm_on_matrix_cores(const hyeig_mat* H, int m, hyeig_dtype xdt, hyeig_dtype acc, hyeig_dtype vdt) {
  if (vdt == HYEIG_BF16 || m > 16 || H->nbr <= 0) return false;
  if (xdt == HYEIG_F32 && acc == HYEIG_F32) return m >= MMA_MIN_WIDTH;
  if (acc == HYEIG_F64) return m >= MMA64_MIN_WIDTH;
  return false;
}

hyeig_status launch_spmm(hyeig_ctx* ctx, const hyeig_mat* H, int m, const void* X, int64_t ldx, hyeig_dtype xdt,
                         void* Y, int64_t ldy, hyeig_dtype acc, hyeig_dtype vdt, bool xfull) {
  if (vdt == HYEIG_BF16) {
    if (xdt == HYEIG_F32 && acc == HYEIG_F32)
      return spmm_width<float, float, uint16_t>(ctx, H, m, (const float*)X, ldx, (float*)Y, ldy, H->vals_bf16, H->tvals_bf16, xfull);
    return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: BF16 values need FP32 X and FP32 accumulation");
  }
  const bool mma = m <= 16 && H->nbr > 0;
  if (xdt == HYEIG_F32 && acc == HYEIG_F32) {
    if (mma && m >= MMA_MIN_WIDTH)
      return launch_mma_any<float, float>(ctx, H, m, (const float*)X, ldx, (float*)Y, ldy, m);
    return spmm_width<float, float, float>(ctx, H, m, (const float*)X, ldx, (float*)Y, ldy, H->vals, H->tvals, xfull);
  }
  if (xdt == HYEIG_F64 && acc == HYEIG_F64) {
    if (mma && m >= MMA64_MIN_WIDTH)
      return launch_mma_any<double, double>(ctx, H, m, (const double*)X, ldx, (double*)Y, ldy, m);
    return spmm_width<double, double, float>(ctx, H, m, (const double*)X, ldx, (double*)Y, ldy, H->vals, H->tvals, xfull);
  }
  if (xdt == HYEIG_F32 && acc == HYEIG_F64) {
    if (mma && m >= MMA64_MIN_WIDTH)
      return launch_mma_any<float, double>(ctx, H, m, (const float*)X, ldx, (double*)Y, ldy, m);
    return spmm_width<float, double, float>(ctx, H, m, (const float*)X, ldx, (double*)Y, ldy, H->vals, H->tvals, xfull);
  }
  return set_err(ctx, HYEIG_EUNSUPPORTED, "spmm_sym: unsupported dtype combination");
}
