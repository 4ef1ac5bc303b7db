/*
 * synthgen: seeded, counter-based synthetic inputs for the hybrid eigensolver.
 *
 * This module holds no arithmetic of the eigensolver.  It only produces the
 * synthetic test matrices (half-stored symmetric H, upper triangle incl. the
 * diagonal, CSR with int64 row pointers / int32 columns / FP32 values) and
 * seeded normal blocks (start blocks X0).  Both the oracle and the GPU path
 * read their inputs from here, so neither derives inputs from the other.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), written from its published definition:
 * ten rounds of two 32x32->64-bit multiplies (constants 0xD2511F53 and
 * 0xCD9E8D57) with a Weyl key schedule (0x9E3779B9, 0xBB67AE85).  Normals use
 * the Box-Muller transform on two uniforms u = (word + 0.5) * 2^-32.
 *
 * Matrix recipe (32x32 tiles, nbr = ceil(n/32) block rows):
 *   - block row i holds its diagonal tile plus min(t, cnt) upper tiles whose
 *     block columns are drawn without replacement (Floyd's algorithm) from the
 *     cnt = min(i+w, nbr-1) - i candidates (i, min(i+w, nbr-1)];
 *     key (seed, stream 0), counter (i, draw, 0, 0);
 *   - entry (r, c) of tile (i, j) is stored iff word < floor(p * 2^32), with
 *     word q of counter (i, j, e/4, 0), key (seed, 1), e = 32 r + c, q = e % 4;
 *     in the diagonal tile only c > r is drawn;
 *   - its value is 0.5 * N(0,1), the normal taken from counter (i, j, e/2, 0),
 *     key (seed, 2) (cos branch for even e, sin branch for odd e);
 *   - the diagonal d_k = 20 k / n + 0.1 * N(0,1) is always stored, normal from
 *     counter (k/2, 0, 0, 0), key (seed, 3);
 *   - values are formed in double and rounded to FP32 (round to nearest even);
 *     the FP32 numbers are the matrix.
 * Seeded normal blocks: element (r, c) of an n x m block uses counter
 * (r, c/2, 0, 0), key (seed, stream).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SG_M0 0xD2511F53u
#define SG_M1 0xCD9E8D57u
#define SG_W0 0x9E3779B9u
#define SG_W1 0xBB67AE85u

void sg_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += SG_W0; k1 += SG_W1; }
    uint64_t p0 = (uint64_t)SG_M0 * c0;
    uint64_t p1 = (uint64_t)SG_M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static inline void ph(uint32_t a, uint32_t b, uint32_t c, uint32_t seed, uint32_t stream, uint32_t o[4]) {
  uint32_t ctr[4] = {a, b, c, 0u};
  uint32_t key[2] = {seed, stream};
  sg_philox4x32_10(ctr, key, o);
}

static inline double sg_unit(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* Box-Muller normal from words (w0, w1); branch 0 = cos, 1 = sin. */
double sg_box_muller(uint32_t w0, uint32_t w1, int branch) {
  double u1 = sg_unit(w0), u2 = sg_unit(w1);
  double rad = sqrt(-2.0 * log(u1));
  double ang = 6.283185307179586 * u2;
  return branch ? rad * sin(ang) : rad * cos(ang);
}

/* Block columns of the upper tiles of block row i, ascending; returns count. */
int sg_tile_cols(int64_t nbr, int t, int64_t w, uint32_t seed, int64_t i, int32_t* out) {
  int64_t hi = i + w;
  if (hi > nbr - 1) hi = nbr - 1;
  int64_t cnt = hi - i;
  if (cnt <= 0) return 0;
  if (cnt <= t) {
    for (int64_t q = 0; q < cnt; ++q) out[q] = (int32_t)(i + 1 + q);
    return (int)cnt;
  }
  /* Floyd's sampling of t distinct offsets from [0, cnt). */
  int nsel = 0;
  for (int64_t jj = cnt - t; jj < cnt; ++jj) {
    uint32_t o[4];
    ph((uint32_t)i, (uint32_t)(jj - (cnt - t)), 0u, seed, 0u, o);
    int64_t r = (int64_t)(((uint64_t)o[0] * (uint64_t)(jj + 1)) >> 32);
    int found = 0;
    for (int q = 0; q < nsel; ++q) if (out[q] == (int32_t)r) { found = 1; break; }
    out[nsel++] = (int32_t)(found ? jj : r);
  }
  /* insertion sort (t is small) then shift to block-column numbers */
  for (int a = 1; a < nsel; ++a) {
    int32_t v = out[a]; int b = a - 1;
    while (b >= 0 && out[b] > v) { out[b + 1] = out[b]; --b; }
    out[b + 1] = v;
  }
  for (int q = 0; q < nsel; ++q) out[q] = (int32_t)(i + 1 + out[q]);
  return nsel;
}

static inline uint64_t sg_thr(double p) {
  if (p <= 0.0) return 0;
  if (p >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)floor(p * 4294967296.0);
}

/* 32 row masks of tile (i, j): bit c of mask[r] set iff entry (r, c) drawn. */
static void sg_tile_masks(uint32_t seed, int64_t i, int64_t j, uint64_t thr, uint32_t mask[32]) {
  memset(mask, 0, 32 * sizeof(uint32_t));
  for (uint32_t g = 0; g < 256; ++g) {
    uint32_t o[4];
    ph((uint32_t)i, (uint32_t)j, g, seed, 1u, o);
    for (int q = 0; q < 4; ++q) {
      if ((uint64_t)o[q] < thr) {
        uint32_t e = 4 * g + q;
        mask[e >> 5] |= 1u << (e & 31);
      }
    }
  }
  if (i == j) /* diagonal tile: strictly upper part only */
    for (int r = 0; r < 32; ++r) mask[r] &= (r == 31) ? 0u : (0xFFFFFFFFu << (r + 1));
}

static float sg_tile_value(uint32_t seed, int64_t i, int64_t j, uint32_t e) {
  uint32_t o[4];
  ph((uint32_t)i, (uint32_t)j, e >> 1, seed, 2u, o);
  return (float)(0.5 * sg_box_muller(o[0], o[1], (int)(e & 1)));
}

float sg_diag_value(int64_t n, uint32_t seed, int64_t k) {
  uint32_t o[4];
  ph((uint32_t)(k >> 1), 0u, 0u, seed, 3u, o);
  return (float)(20.0 * (double)k / (double)n + 0.1 * sg_box_muller(o[0], o[1], (int)(k & 1)));
}

/* Number of stored entries of each row in block rows [i0, i1); returns the sum.
 * counts has one slot per row 32*i0 .. min(32*i1, n)-1. */
int64_t sg_gen_rowcounts(int64_t n, int t, int64_t w, double p, uint32_t seed,
                         int64_t i0, int64_t i1, int64_t* counts) {
  int64_t nbr = (n + 31) / 32;
  uint64_t thr = sg_thr(p);
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
  for (int64_t i = i0; i < i1; ++i) {
    int32_t cols[1024];
    int tt = t > 1024 ? 1024 : t;
    int nt = sg_tile_cols(nbr, tt, w, seed, i, cols);
    uint32_t mask[32];
    int64_t cnt[32];
    for (int r = 0; r < 32; ++r) cnt[r] = 1; /* diagonal */
    sg_tile_masks(seed, i, i, thr, mask);
    for (int r = 0; r < 32; ++r) {
      uint32_t mk = mask[r];
      int64_t lim = n - 32 * i; /* columns c with 32i + c < n */
      if (lim < 32) mk &= (lim <= 0) ? 0u : ((1u << lim) - 1u);
      cnt[r] += __builtin_popcount(mk);
    }
    for (int q = 0; q < nt; ++q) {
      int64_t j = cols[q];
      sg_tile_masks(seed, i, j, thr, mask);
      int64_t lim = n - 32 * j;
      uint32_t cm = (lim >= 32) ? 0xFFFFFFFFu : ((1u << lim) - 1u);
      for (int r = 0; r < 32; ++r) cnt[r] += __builtin_popcount(mask[r] & cm);
    }
    for (int r = 0; r < 32; ++r) {
      int64_t k = 32 * i + r;
      if (k >= n) break;
      counts[k - 32 * i0] = cnt[r];
      total += cnt[r];
    }
  }
  return total;
}

/* Fill colidx/vals for block rows [i0, i1).  rowptr is indexed from row 32*i0
 * (rowptr[0] is the offset of that row inside colidx/vals). */
void sg_gen_fill(int64_t n, int t, int64_t w, double p, uint32_t seed, int64_t i0, int64_t i1,
                 const int64_t* rowptr, int32_t* colidx, float* vals) {
  int64_t nbr = (n + 31) / 32;
  uint64_t thr = sg_thr(p);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = i0; i < i1; ++i) {
    int32_t cols[1025];
    int tt = t > 1024 ? 1024 : t;
    int nt = sg_tile_cols(nbr, tt, w, seed, i, cols + 1);
    cols[0] = (int32_t)i;
    int64_t pos[32];
    for (int r = 0; r < 32; ++r) {
      int64_t k = 32 * i + r;
      if (k >= n) break;
      pos[r] = rowptr[k - 32 * i0];
      colidx[pos[r]] = (int32_t)k;
      vals[pos[r]] = sg_diag_value(n, seed, k);
      pos[r]++;
    }
    uint32_t mask[32];
    for (int q = 0; q <= nt; ++q) {
      int64_t j = cols[q];
      sg_tile_masks(seed, i, j, thr, mask);
      for (int r = 0; r < 32; ++r) {
        int64_t k = 32 * i + r;
        if (k >= n) break;
        uint32_t mk = mask[r];
        while (mk) {
          int c = __builtin_ctz(mk);
          mk &= mk - 1;
          int64_t col = 32 * j + c;
          if (col >= n) break;
          colidx[pos[r]] = (int32_t)col;
          vals[pos[r]] = sg_tile_value(seed, i, j, (uint32_t)(32 * r + c));
          pos[r]++;
        }
      }
    }
  }
}

/* Whole matrix: rowptr[n+1] must be allocated; returns nnz after filling
 * rowptr only when colidx == NULL (sizing call), else fills everything. */
int64_t sg_gen_csr(int64_t n, int t, int64_t w, double p, uint32_t seed,
                   int64_t* rowptr, int32_t* colidx, float* vals) {
  int64_t nbr = (n + 31) / 32;
  int64_t nnz = sg_gen_rowcounts(n, t, w, p, seed, 0, nbr, rowptr + 1);
  rowptr[0] = 0;
  for (int64_t k = 0; k < n; ++k) rowptr[k + 1] += rowptr[k];
  if (colidx && vals) sg_gen_fill(n, t, w, p, seed, 0, nbr, rowptr, colidx, vals);
  return nnz;
}

/* Seeded N(0,1) block, row-major n x m with leading dimension ld (doubles). */
void sg_normal_block_f64(int64_t n, int m, int64_t ld, uint32_t seed, uint32_t stream, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    for (int c = 0; c < m; c += 2) {
      uint32_t o[4];
      ph((uint32_t)r, (uint32_t)(c >> 1), 0u, seed, stream, o);
      out[r * ld + c] = sg_box_muller(o[0], o[1], 0);
      if (c + 1 < m) out[r * ld + c + 1] = sg_box_muller(o[0], o[1], 1);
    }
  }
}
