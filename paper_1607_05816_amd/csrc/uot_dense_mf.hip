// Dense point-cloud product of libuot with the squared Euclidean cost on the
// gfx950 matrix cores, with its launcher.
#include <cstdlib>

#include "uot_device.h"
#include "uot_epilogue.h"
#include "uot_launch.h"

// ---------------------------------------------------------------------------
// Row i of a half-step needs log2 sum_j 2^{w_j - c |x_i - y_j|^2} (c =
// log2(e) / eps, w_j the column's log2 weight).  Around a centre xbar shared
// by the rows of a block, with e_i = x_i - xbar,
//   w_j - c |x_i - y_j|^2 = R_i + G_j + e_i . B_j,
//   R_i = -c |e_i|^2,  G_j = w_j - c |y_j - xbar|^2,  B_j = 2 c (y_j - xbar),
// exactly (the host passes Morton-ordered clouds, so the rows of a block lie
// close together and |e_i . B_j| stays small for the columns that matter).
// The exponents of 16 columns x 16 rows are then the product of a
// 16 x K matrix (column operands) with a K x 16 matrix (row operands), one
// MFMA, which leaves one exp2 and one add per pair to the vector units.  Two
// operand forms:
//   FP32 (SPLIT = false): K = 4, column (B_j, G_j), row (e_i, 1), one
//     v_mfma_f32_16x16x4f32.  FP32 matrix instructions run on the vector
//     ALUs: they do not overlap the exp2.
//   BF16 x 3 (SPLIT = true): every FP32 operand a is split into three bf16
//     parts a = a1 + a2 + a3 (each the bf16 rounding of what the previous
//     parts leave; 24 significant bits together), and e.B is summed from the
//     six part products e_r B_s with r + s <= 4 per coordinate, G from its
//     three parts against 1: 21 of the 32 slots of one
//     v_mfma_f32_16x16x32_bf16 (products exact, FP32 accumulation; dropped
//     part products are below 2^-24 of |e_d B_d|).  These run on the matrix
//     cores, next to the exp2 of other groups.
// The column operands of a chunk of columns (512 in the dense kernel, 256 in
// the batch one) are built once in LDS.
// Layout of the 16 x 16 MFMAs (64 lanes, q = lane / 16, l = lane % 16): a
// lane supplies A[l][k in slots of q] and B[k in slots of q][l] (the same K
// slots for both), and gets D[4 q + r][l], r = 0..3.  Here A holds the
// columns and B the rows (row 16 g + l of the wave), so lane (q, l) gets the
// exponents of row 16 g + l against columns 4 q .. 4 q + 3 of the tile:
// every lane keeps one running sum per row group, and a row is spread over
// the 4 lanes l + 16 q.
// Shift: the sum pass feeds minus a running maximum m of each row in as the
// accumulator input.  m starts from the row's maximum over the same columns
// (the block's column split; all columns of a batch problem) in the previous
// product of this side (pw; the potentials move little between iterations),
// or is not finite (the first product of a solve).  A wave whose rows all
// start from a finite m runs the sum pass alone over every chunk and checks
// the row totals at the end of the split.  Otherwise a chunk where some row
// has no finite m takes a maximum pass first (lane maxima, then over the 4
// lanes of the row), so every exp2 argument is <= 0, and later chunks run the
// sum pass against m, redone with both passes when a row total is not below
// 2^100 (a term above m stays finite up to 2^127, and an overflow fails the
// test too); accepted chunks move whole powers of two of the total into m.
// A row whose final total is below 2^-60 (under a finite m) started from an
// m too high, one not below 2^100 (unchecked chunks) from one too low: the
// block then sums its split again from no maximum, checking every chunk.  So
// every accepted total has a term within 2^60 of m, and the terms that
// underflow (more than 2^126 below m) do not change it.
// Columns without mass (and padding) carry G = -inf, so their terms are 0.
// G row groups of 16 per wave (64 G rows per block);
// grid = (ceil(Nr / (64 G)), splits); partials (m, s) per split as the
// direct kernel: log2 sum = m + log2 s.
// ---------------------------------------------------------------------------
namespace uot {

typedef float mf_f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 mf_bf16x8 __attribute__((ext_vector_type(8)));
// LDS columns for chunks of C columns: C staged plus two padding tiles of 16
constexpr int mf_cols(int C) { return C + 32; }

// sum over the four lanes l % 16 + {0, 16, 32, 48}
__device__ __forceinline__ float sum_over_rows(float x) {
  const LanePair p = lane_xor16(x);
  const float y = p.a + p.b;
  const LanePair r = lane_xor32(y);
  return r.a + r.b;
}

// Operands built as packed words.  split3f(a) gives the three bf16 parts of
// a (a1 = bf16(a), a2 = bf16(a - a1), a3 = bf16(a - a1 - a2); together 24
// significant bits) as floats, a1 and a2 exact and a3 left unrounded: pk2
// rounds it to bf16, and every other value it packs is a bf16 value already.
// pk2(lo, hi) is one v_cvt_pk_bf16_f32: the word of two K slots.
typedef float mf_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 mf_bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t mf_u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pk2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(mf_f32x2{lo, hi}, mf_bf16x2));
}
__device__ __forceinline__ float bf16r(float x) { return (float)(__bf16)x; }
__device__ __forceinline__ void split3f(float a, float (&p)[3]) {
  p[0] = bf16r(a);
  const float r1 = a - p[0];
  p[1] = bf16r(r1);
  p[2] = r1 - p[1];
}
// -inf -> (-inf, 0, 0)
__device__ __forceinline__ void split3f_inf(float a, float (&p)[3]) {
  const bool fin = a > -__builtin_inff();
  split3f(fin ? a : 0.f, p);
  p[0] = fin ? p[0] : a;
}

// The K = 32 slots of both operands: slot k < 18 is part product u = k % 6
// of coordinate k / 6, with (row part, column part) = (1,1) (1,2) (2,1)
// (1,3) (2,2) (3,1); slots 18, 19, 20 carry G's three parts against 1; the
// rest are 0.  Words (slot pairs) of a column with parts b[d][.] of 2c(y -
// xbar)_d and g[.] of G, and of a row with parts e[d][.] of (x - xbar)_d;
// lane quarter q holds words 4q .. 4q + 3.
__device__ __forceinline__ void col_words(const float (&b)[3][3], const float (&g)[3], mf_u32x4 (&w)[4]) {
  uint32_t c[9];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c[3 * d] = pk2(b[d][0], b[d][1]);
    c[3 * d + 1] = pk2(b[d][0], b[d][2]);
    c[3 * d + 2] = pk2(b[d][1], b[d][0]);
  }
  w[0] = mf_u32x4{c[0], c[1], c[2], c[3]};
  w[1] = mf_u32x4{c[4], c[5], c[6], c[7]};
  w[2] = mf_u32x4{c[8], pk2(g[0], g[1]), pk2(g[2], 0.f), 0u};
  w[3] = mf_u32x4{0u, 0u, 0u, 0u};
}
__device__ __forceinline__ void row_words(const float (&e)[3][3], mf_u32x4 (&w)[4]) {
  uint32_t c[9];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c[3 * d] = pk2(e[d][0], e[d][0]);
    c[3 * d + 1] = pk2(e[d][1], e[d][0]);
    c[3 * d + 2] = pk2(e[d][1], e[d][2]);
  }
  w[0] = mf_u32x4{c[0], c[1], c[2], c[3]};
  w[1] = mf_u32x4{c[4], c[5], c[6], c[7]};
  w[2] = mf_u32x4{c[8], pk2(1.f, 1.f), pk2(1.f, 0.f), 0u};
  w[3] = mf_u32x4{0u, 0u, 0u, 0u};
}

// operand forms: the lane's column operand of tile t (16 columns) from its
// LDS base, and the product
template <bool SPLIT>
struct MfOps;
template <>
struct MfOps<false> {
  using Op = float;                   // staged as [k][column]: base = &st[q][l]
  static __device__ __forceinline__ Op col(const Op* base, int t) { return base[t * 16]; }
  static __device__ __forceinline__ mf_f32x4 mma(Op a, Op b, mf_f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfOps<true> {
  using Op = mf_bf16x8;               // staged as [column][q]: base = &st[l][q]
  static __device__ __forceinline__ Op col(const Op* base, int t) { return base[t * 64]; }
  static __device__ __forceinline__ mf_f32x4 mma(Op a, Op b, mf_f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// The two product passes over the tiles of a staged chunk that `mask` keeps
// (bit t: tile t of 16 columns; wave-uniform).  Both are software-pipelined
// by one row group: the products of group g are issued before the vector
// work on group g - 1 (the last group's follower is group 0 of the next kept
// tile; after the last tile it repeats that tile and is discarded), so the
// exp2 of one group never waits on its own product.
// maximum pass: mx[g] = this lane's maximum exponent of row 16 g + l
template <bool SPLIT, int G, int NT>
__device__ __forceinline__ void mf_max_pass(const typename MfOps<SPLIT>::Op* base,
                                            const typename MfOps<SPLIT>::Op (&E)[G], uint32_t kept, float (&mx)[G]) {
  using O = MfOps<SPLIT>;
  const mf_f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int g = 0; g < G; ++g) mx[g] = -__builtin_inff();
  // a counted loop over the kept tiles; bit NT (the first padding tile)
  // stays set, so the follower of the last kept tile is a padding tile
  const int n = __builtin_popcount(kept);
  if (n == 0) return;
  uint64_t mask = (uint64_t)kept | (1ull << NT);
  int jt = __builtin_ctzll(mask);
  mask &= mask - 1;
  mf_f32x4 c0 = O::mma(O::col(base, jt), E[0], zero);
  for (int k = 0; k < n; ++k) {
    const int jn = __builtin_ctzll(mask);
    mask &= mask - 1;
    const auto b = O::col(base, jt), bn = O::col(base, jn);
#pragma unroll
    for (int g = 1; g <= G; ++g) {
      const mf_f32x4 e0 = O::mma(g < G ? b : bn, E[g % G], zero);
      __builtin_amdgcn_sched_barrier(0);   // the product goes out first
      const float t = fmaxf(fmaxf(mx[g - 1], c0[0]), c0[1]);
      mx[g - 1] = fmaxf(fmaxf(t, c0[2]), c0[3]);
      c0 = e0;
      __builtin_amdgcn_sched_barrier(0);
    }
    jt = jn;
  }
}
// sum pass: s[g] += sum of 2^{exponent - max} (nm = minus the row maxima)
template <bool SPLIT, int G, int NT>
__device__ __forceinline__ void mf_sum_pass(const typename MfOps<SPLIT>::Op* base,
                                            const typename MfOps<SPLIT>::Op (&E)[G], const mf_f32x4 (&nm)[G],
                                            uint32_t kept, float (&s)[G]) {
  using O = MfOps<SPLIT>;
  const int n = __builtin_popcount(kept);
  if (n == 0) return;
  uint64_t mask = (uint64_t)kept | (1ull << NT);
  int jt = __builtin_ctzll(mask);
  mask &= mask - 1;
  mf_f32x4 dc = O::mma(O::col(base, jt), E[0], nm[0]);
  for (int k = 0; k < n; ++k) {
    const int jn = __builtin_ctzll(mask);
    mask &= mask - 1;
    const auto b = O::col(base, jt), bn = O::col(base, jn);
#pragma unroll
    for (int g = 1; g <= G; ++g) {
      const mf_f32x4 dn = O::mma(g < G ? b : bn, E[g % G], nm[g % G]);
      __builtin_amdgcn_sched_barrier(0);
      s[g - 1] += (__builtin_amdgcn_exp2f(dc[0]) + __builtin_amdgcn_exp2f(dc[1])) +
                  (__builtin_amdgcn_exp2f(dc[2]) + __builtin_amdgcn_exp2f(dc[3]));
      dc = dn;
      __builtin_amdgcn_sched_barrier(0);
    }
    jt = jn;
  }
}

// maximum over the 16 lanes of a DPP row (lanes 16 k .. 16 k + 15)
__device__ __forceinline__ float row16_max(float v) {
  v = fmaxf(v, dpp_mov<kDppXor1>(v));
  v = fmaxf(v, dpp_mov<kDppXor2>(v));
  v = fmaxf(v, dpp_mov<kDppHalfMirror>(v));
  return fmaxf(v, dpp_mov<kDppMirror>(v));
}
__device__ __forceinline__ float row16_min(float v) {
  v = fminf(v, dpp_mov<kDppXor1>(v));
  v = fminf(v, dpp_mov<kDppXor2>(v));
  v = fminf(v, dpp_mov<kDppHalfMirror>(v));
  return fminf(v, dpp_mov<kDppMirror>(v));
}
// minimum / maximum over the wave (every lane gets it): DPP within each row
// of 16 lanes, then the lane swaps across rows (no LDS crossbar)
__device__ __forceinline__ float wave_min(float v) {
  v = row16_min(v);
  const LanePair p = lane_xor16(v);
  const LanePair r = lane_xor32(fminf(p.a, p.b));
  return fminf(r.a, r.b);
}
__device__ __forceinline__ float wave_max(float v) { return max_over_rows(row16_max(v)); }

// the pair evaluations of a block (its waves' tile counts, wave-uniform) added
// to *pairs with one atomic per block (every thread of the block calls it)
template <int G>
__device__ __forceinline__ void count_pairs(unsigned long long* pairs, uint32_t evaluated) {
  __shared__ uint32_t wsum[kBlock / 64];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = evaluated;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) t += wsum[k];
    if (t) atomicAdd(pairs, t * (256ull * G));
  }
}

// Negligible tiles (the adaptive truncation of the kernel discussed in the
// section on the further tricks of the sparse scaling literature, applied on
// the fly).  With e_i = x_i - xbar, the exponent a product pass evaluates is
//   D_ij = w_j - c |x_i - y_j|^2 + c |e_i|^2,
// and a row's sum is taken against its running maximum m_i.  For a wave's
// rows (box Bx) and a 16-column tile (box By, largest weight wmax),
//   D_ij - m_i <= wmax - c gap(Bx, By)^2 + max_i (c |e_i|^2 - m_i),
// so a tile whose bound is below -kSkipLog2 contributes less than 2^-50 of
// 2^{m_i} per column to every row of the wave and is left out.  m_i only
// grows during a split, so a bound taken at its start stays valid.  A row
// whose final total (relative to 2^{m_i}) is below 2^-8 after tiles were
// left out started from a maximum far above its terms (the previous
// product's, after a large move of the potentials): its split is summed
// again with nothing left out.  Otherwise the left-out mass is below
// ncol 2^-50 / 2^-8 <= 2^-27 of the row's total for ncol <= 2^15, under
// the FP32 rounding of the total.
constexpr float kSkipLog2 = 50.f;
constexpr float kSkipCheck = 0x1p-8f;

// The product of one block's rows (xr: first row, coordinate stride xs, nrow
// of its 64 G rows valid) with ncol columns (yc: first column, stride ys; w
// their log2 weights): for row 16 g + l of this wave, m[g] (the shift; -inf
// if no term is finite), tot[g] (the total over the row's 4 lanes, relative
// to 2^m) and rc[g] = R_i.  Rows past nrow repeat the last valid row (their
// results are not used).  pw holds the rows' starting maxima on entry and is
// not written.  st, sbox, tb: the block's LDS (st and tb hold two buffers
// for chunks of 256 columns).  skip_tiles: leave negligible
// tiles out; evaluated (wave-uniform) counts the 16-column tiles the wave's
// product passes take.
template <int DIM, int G, bool SPLIT, int CHUNK>
__device__ __forceinline__ void mf_tile(const float* __restrict__ xr, int64_t xs, int nrow,
                                        const float* __restrict__ yc, int64_t ys, const float* __restrict__ w,
                                        int64_t ncol, float cc, const float* __restrict__ pw,
                                        typename MfOps<SPLIT>::Op* st, float (*sbox)[6], float (*tb)[8],
                                        bool skip_tiles, float (&m)[G], float (&tot)[G], float (&rc)[G],
                                        uint32_t& evaluated) {
  static_assert(G % 4 == 0, "a wave's rows are loaded 64 at a time");
  using Op = typename MfOps<SPLIT>::Op;
  static_assert(CHUNK % kBlock == 0 && CHUNK / 16 <= 32, "chunks of 256 or 512 columns");
  constexpr int kCols = mf_cols(CHUNK);
  constexpr int kTiles = CHUNK / 16;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, q = lane >> 4;
  const int wbase = wv * (16 * G);
  // a wave with no valid row (the last rows of a ragged item) only helps to
  // stage the column operands: its product passes are skipped (wave-uniform)
  const bool wave_rows = wbase < nrow;
  // the box of this wave's valid rows, then the block centre: middle of the
  // box of all valid rows
  float wlo[3] = {0.f, 0.f, 0.f}, whi[3] = {0.f, 0.f, 0.f};
  float xb[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    float lo = __builtin_inff(), hi = -__builtin_inff();
#pragma unroll
    for (int t = 0; t < G / 4; ++t) {
      const int row = wbase + t * 64 + lane;
      if (row < nrow) {
        const float v = xr[d * xs + row];
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
      }
    }
    // (wave-uniform values live in scalar registers through the chunk loop)
    wlo[d] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, wave_min(lo))));
    whi[d] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, wave_max(hi))));
    if (lane == 0) {
      sbox[wv][2 * d] = wlo[d];
      sbox[wv][2 * d + 1] = whi[d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const float lo = fminf(fminf(sbox[0][2 * d], sbox[1][2 * d]), fminf(sbox[2][2 * d], sbox[3][2 * d]));
    const float hi =
        fmaxf(fmaxf(sbox[0][2 * d + 1], sbox[1][2 * d + 1]), fmaxf(sbox[2][2 * d + 1], sbox[3][2 * d + 1]));
    xb[d] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(
                                          __builtin_bit_cast(int, lo <= hi ? 0.5f * (lo + hi) : 0.f)));
  }
  // row operands of rows 16 g + l (rows past the end repeat the last one);
  // the running maxima start from the previous product's (pw) and the bound
  // term max_i (c |e_i|^2 - m_i) of the wave from them
  Op E[G];
  float s[G], wm[G];
  float mw = -__builtin_inff();
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int row = min(wbase + g * 16 + li, nrow - 1);
    float e[3], e2 = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      e[d] = d < DIM ? xr[d * xs + row] - xb[d] : 0.f;
      e2 = __builtin_fmaf(e[d], e[d], e2);
    }
    if constexpr (SPLIT) {
      float p[3][3];
#pragma unroll
      for (int d = 0; d < 3; ++d) split3f(e[d], p[d]);
      mf_u32x4 rw[4];
      row_words(p, rw);
      E[g] = __builtin_bit_cast(mf_bf16x8, q == 0 ? rw[0] : (q == 1 ? rw[1] : (q == 2 ? rw[2] : rw[3])));
    } else {
      E[g] = q == 3 ? 1.f : (q == 0 ? e[0] : (q == 1 ? e[1] : e[2]));
    }
    const float v = pw[row];
    wm[g] = __builtin_isfinite(v) ? v : -__builtin_inff();
    mw = fmaxf(mw, cc * e2 - wm[g]);
  }
  // +inf when a row has no finite starting maximum
  mw = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, wave_max(mw))));
  const Op* base = SPLIT ? &st[li * 4 + q] : &st[q * kCols + li];
  // a wave whose rows all start from a finite maximum sums every chunk
  // against it and checks its totals once, at the end of the split; a failed
  // check sums the split again from no maximum, checking every chunk, with
  // every tile
  bool cold = false;
#pragma unroll
  for (int g = 0; g < G; ++g) cold = cold || wm[g] == -__builtin_inff();
  const bool warm_wave = !__any(cold);
  for (int attempt = 0;; ++attempt) {
    const bool unchecked = attempt == 0 && warm_wave;
    // the tile records are staged by the whole block (block-uniform); each
    // wave uses them when its rows all have a starting maximum
    const bool records = skip_tiles && attempt == 0;
    const bool skip_on = records && mw < __builtin_inff();
    bool skipped = false;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      m[g] = attempt == 0 ? wm[g] : -__builtin_inff();
      s[g] = 0.f;
    }
    // this thread's columns h kBlock + t of a chunk; with chunks of 256
    // columns (the batch form) loaded one chunk ahead, in flight during the
    // previous chunk's products (the 512-column dense form has no registers
    // to spare for it)
    constexpr bool kAhead = CHUNK == 256;
    constexpr int H = CHUNK / kBlock;
    // the batch form also stages into two LDS buffers in turn (one barrier
    // per chunk: a buffer is written again only after the barrier that
    // follows the next chunk's staging, which every wave reaches after its
    // products on that buffer); the dense form has one
    auto buf_of = [](int64_t c0) -> int { return kAhead ? (int)((c0 / CHUNK) & 1) : 0; };
    float y[H][3], wj[H];
    auto load_cols = [&](int64_t c0) {
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int64_t col = c0 + h * kBlock + threadIdx.x;
        y[h][0] = y[h][1] = y[h][2] = 0.f;
        wj[h] = -__builtin_inff();
        if (col < ncol) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) y[h][d] = yc[d * ys + col];
          wj[h] = w[col];
        }
      }
    };
    if constexpr (kAhead) load_cols(0);
    // chunk c0: staged by the whole block (two barriers), the loads of the
    // next chunk started, and the tiles this wave evaluates returned (bit t:
    // tile t; wave-uniform; 0 for a wave with no valid row)
    auto stage = [&](int64_t c0) -> uint32_t {
      Op* const sb = st + buf_of(c0) * (4 * kCols);
      float(*const tbb)[8] = tb + buf_of(c0) * kTiles;
      if constexpr (!kAhead) {
        load_cols(c0);
        __syncthreads();                   // the previous chunk's reads are done
      }
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int lc = h * kBlock + threadIdx.x;
        float bd[3], d2 = 0.f;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float a = d < DIM ? y[h][d] - xb[d] : 0.f;
          bd[d] = 2.f * cc * a;
          d2 = __builtin_fmaf(a, a, d2);
        }
        const float gj = wj[h] == -__builtin_inff() ? wj[h] : __builtin_fmaf(-cc, d2, wj[h]);
        if constexpr (SPLIT) {
          float b[3][3], gp[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) split3f(bd[d], b[d]);
          split3f_inf(gj, gp);
          mf_u32x4 cw[4];
          col_words(b, gp, cw);
#pragma unroll
          for (int k = 0; k < 4; ++k) sb[lc * 4 + k] = __builtin_bit_cast(mf_bf16x8, cw[k]);
        } else {
#pragma unroll
          for (int d = 0; d < 3; ++d) sb[d * kCols + lc] = bd[d];
          sb[3 * kCols + lc] = gj;
        }
        if (records) {
          // the tile's box (columns of weight -inf left out) and largest weight
          const bool live = wj[h] > -__builtin_inff();
          float rec[7];
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            rec[d] = row16_min(live ? y[h][d] : __builtin_inff());
            rec[3 + d] = row16_max(live ? y[h][d] : -__builtin_inff());
          }
          rec[6] = row16_max(wj[h]);
          if (li == 0) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
              tbb[lc >> 4][d] = rec[d];
              tbb[lc >> 4][3 + d] = rec[3 + d];
            }
            tbb[lc >> 4][6] = rec[6];
          }
        }
      }
      __syncthreads();
      if constexpr (kAhead) {
        if (c0 + CHUNK < ncol) load_cols(c0 + CHUNK);
      }
      const int64_t rem = ncol - c0;
      const int cnt = rem < CHUNK ? (int)rem : CHUNK;
      const int ntl = (cnt + 15) >> 4;
      if (!wave_rows) return 0u;            // (after the staging and its barriers)
      // the tiles this wave evaluates: lane t tests tile t
      uint32_t mask = ntl >= 32 ? 0xFFFFFFFFu : ((1u << ntl) - 1u);
      if (skip_on) {
        bool keep = false;
        if (lane < ntl) {
          float gap2 = 0.f;
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            const float g = fmaxf(fmaxf(tbb[lane][d] - whi[d], wlo[d] - tbb[lane][3 + d]), 0.f);
            gap2 = __builtin_fmaf(g, g, gap2);
          }
          keep = tbb[lane][6] - cc * gap2 + mw >= -kSkipLog2;
        }
        const uint32_t kept = (uint32_t)__ballot(keep);
        skipped = skipped || kept != mask;
        mask = kept;
      }
      mask = __builtin_amdgcn_readfirstlane(mask);
      evaluated += (uint32_t)__builtin_popcount(mask);
      return mask;
    };
    if (kAhead && unchecked) {
      // every row of the wave starts from a finite m, fixed through the
      // split: the accumulator inputs -m are built once
      mf_f32x4 nm[G];
#pragma unroll
      for (int g = 0; g < G; ++g) nm[g] = mf_f32x4{-m[g], -m[g], -m[g], -m[g]};
      for (int64_t c0 = 0; c0 < ncol; c0 += CHUNK) {
        const uint32_t mask = __builtin_amdgcn_readfirstlane(stage(c0));
        mf_sum_pass<SPLIT, G, kTiles>(base + buf_of(c0) * (4 * kCols), E, nm, mask, s);
      }
    } else {
      for (int64_t c0 = 0; c0 < ncol; c0 += CHUNK) {
        const uint32_t mask = __builtin_amdgcn_readfirstlane(stage(c0));
        if (!wave_rows) continue;
        if (!kAhead && unchecked) {
          mf_f32x4 nm[G];
#pragma unroll
          for (int g = 0; g < G; ++g) nm[g] = mf_f32x4{-m[g], -m[g], -m[g], -m[g]};
          mf_sum_pass<SPLIT, G, kTiles>(base + buf_of(c0) * (4 * kCols), E, nm, mask, s);
          continue;
        }
        // a chunk with a row that has no finite running maximum yet (the
        // first chunk) takes the maximum pass first; others run the sum pass
        // against the running maxima and take the two passes only when a
        // row's sum leaves [0, 2^100) (a new maximum far above the old one)
        bool two = false;
#pragma unroll
        for (int g = 0; g < G; ++g) two = two || m[g] == -__builtin_inff();
        two = __any(two);
        if (!two) {
          float s0[G];
          mf_f32x4 nm[G];
#pragma unroll
          for (int g = 0; g < G; ++g) {
            s0[g] = s[g];
            nm[g] = mf_f32x4{-m[g], -m[g], -m[g], -m[g]};
          }
          mf_sum_pass<SPLIT, G, kTiles>(base + buf_of(c0) * (4 * kCols), E, nm, mask, s);
          bool bad = false;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            tot[g] = sum_over_rows(s[g]);
            bad = bad || !(tot[g] < 0x1p100f);
          }
          if (__any(bad)) {
#pragma unroll
            for (int g = 0; g < G; ++g) s[g] = s0[g];
            two = true;
          } else {
            // keep the sums near 1: move whole powers of two into the maxima (the
            // same in the 4 lanes of a row, whose totals are equal)
#pragma unroll
            for (int g = 0; g < G; ++g)
              if (tot[g] > 0x1p32f) {
                const int k = __builtin_amdgcn_frexp_expf(tot[g]);
                m[g] += float(k);
                s[g] = __builtin_amdgcn_ldexpf(s[g], -k);
              }
          }
        }
        if (two) {
          float mx[G];
          mf_max_pass<SPLIT, G, kTiles>(base + buf_of(c0) * (4 * kCols), E, mask, mx);
          // new running maxima; rescale the sums; accumulator input -max
          mf_f32x4 nm[G];
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const float mn = fmaxf(m[g], max_over_rows(mx[g]));
            const float sh = mn == -__builtin_inff() ? 0.f : mn;
            s[g] *= __builtin_amdgcn_exp2f(m[g] - sh);
            m[g] = mn;
            nm[g] = mf_f32x4{-sh, -sh, -sh, -sh};
          }
          mf_sum_pass<SPLIT, G, kTiles>(base + buf_of(c0) * (4 * kCols), E, nm, mask, s);
        }
      }
    }
    // totals of each row over its 4 lanes; a total below 2^-60 under a finite
    // maximum came from a starting maximum too high (below 2^-8 once tiles
    // were left out), one not below 2^100 (unchecked chunks) from one too
    // low: sum the split again from none (the whole block, as the chunk loop
    // holds barriers)
    const float low = skipped ? kSkipCheck : 0x1p-60f;
    bool redo = false;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      tot[g] = sum_over_rows(s[g]);
      redo = redo || (m[g] != -__builtin_inff() && !(tot[g] >= low)) || !(tot[g] < 0x1p100f);
    }
    redo = redo && wave_rows;
    if (attempt > 0 || !__syncthreads_or(redo)) break;
  }
  // row constants R_i = -c |e_i|^2
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int row = min(wbase + g * 16 + li, nrow - 1);
    float e2 = 0.f;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const float e = xr[d * xs + row] - xb[d];
      e2 = __builtin_fmaf(e, e, e2);
    }
    rc[g] = -cc * e2;
  }
}

template <int DIM, int G, bool SPLIT>
__global__ __launch_bounds__(kBlock, G == 4 ? 4 : 2) void k_dense_mf(const float* __restrict__ xr, int64_t Nr,
                                                      const float* __restrict__ yc, const float* __restrict__ w,
                                                      int64_t Mc, int64_t cols_per_split,
                                                      float* __restrict__ pm, float* __restrict__ ps,
                                                      float* __restrict__ pw, int side, const Ctrl* __restrict__ c,
                                                      int skip_tiles, unsigned long long* __restrict__ pairs) {
  using Op = typename MfOps<SPLIT>::Op;
  if (skip_side(c, side)) return;
  // column operands of a chunk of 512 columns and two padding tiles (read
  // by the discarded final products of the passes): FP32 [k][column], BF16
  // x 3 [column][q]; the chunk's tile records
  __shared__ Op st[4 * mf_cols(512)];
  __shared__ float sbox[4][6];
  __shared__ float tb[32][8];
  const float cc = float(kLog2e / eps_of(c, side));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, q = lane >> 4;
  const int64_t bbase = (int64_t)blockIdx.x * (64 * G);
  const int64_t cb = (int64_t)blockIdx.y * cols_per_split;
  const int64_t ce = (cb + cols_per_split < Mc) ? cb + cols_per_split : Mc;
  const int nrow = (int)(Nr - bbase < 64 * G ? Nr - bbase : 64 * G);
  float* pws = pw + blockIdx.y * Nr + bbase;
  float m[G], tot[G], rc[G];
  uint32_t evaluated = 0;
  mf_tile<DIM, G, SPLIT, 512>(xr + bbase, Nr, nrow, yc + cb, Mc, w + cb, ce - cb, cc, pws, st, sbox, tb,
                              skip_tiles != 0, m, tot, rc, evaluated);
  if (pairs) count_pairs<G>(pairs, evaluated);
  // lanes q = 0 write row 16 g + l: (m + R_i, total), and m for the next
  // product of this side
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int row = wv * (16 * G) + g * 16 + li;
    if (q == 0 && row < nrow) {
      pm[blockIdx.y * Nr + bbase + row] = m[g] == -__builtin_inff() ? m[g] : m[g] + rc[g];
      ps[blockIdx.y * Nr + bbase + row] = tot[g];
      pws[row] = m[g];
    }
  }
}

// Ragged batch on the matrix cores: persistent blocks pull (problem, 64 G
// rows) items from the list as k_batch_lse does, take the product of the
// item's rows with all columns of the problem (the clouds in Morton order per
// problem) and apply the proxdiv epilogue; pw: starting maxima per row, left
// for the next iteration.
// (4 row groups per wave fit 128 VGPRs: 4 waves per SIMD; 8 groups take 2)
template <int DIM, int G, bool SPLIT>
__global__ __launch_bounds__(kBlock, G == 4 ? 4 : 2) void k_batch_mf(const BItem* __restrict__ items,
                                                      const int* __restrict__ count, int* __restrict__ cursor,
                                                      const int64_t* __restrict__ offR,
                                                      const int64_t* __restrict__ offC, const float* __restrict__ xr,
                                                      int64_t totR, const float* __restrict__ yc, int64_t totC,
                                                      const float* __restrict__ w, float* __restrict__ pw,
                                                      const BCtrl* __restrict__ bc, const Ctrl* __restrict__ c,
                                                      int side, EpiArgs<float> ep, int skip_tiles,
                                                      unsigned long long* __restrict__ pairs) {
  using Op = typename MfOps<SPLIT>::Op;
  __shared__ Op st[2 * 4 * mf_cols(256)];   // two buffers of 256 columns: batch problems are small
  __shared__ float sbox[4][6];
  __shared__ float tb[2 * 16][8];
  __shared__ int item_sh;
  uint32_t evaluated = 0;
  const float cc = float(kLog2e / eps_of(c, side));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, q = lane >> 4;
  const int n_items = *count;
  const int32_t* __restrict__ skip = half_of(side) == 0 ? bc->stop : bc->yskip;
  while (true) {
    __syncthreads();   // the previous item's reads of the block's LDS are done
    if (threadIdx.x == 0) item_sh = atomicAdd(cursor, 1);
    __syncthreads();
    const int it = item_sh;
    if (it >= n_items) break;
    const BItem I = items[it];
    if (skip[I.prob]) continue;
    const int64_t rb = offR[I.prob] + I.row0;
    const int64_t cb = offC[I.prob], ce = offC[I.prob + 1];
    float m[G], tot[G], rc[G];
    mf_tile<DIM, G, SPLIT, 256>(xr + rb, totR, I.nrows, yc + cb, totC, w + cb, ce - cb, cc, pw + rb, st, sbox, tb,
                                skip_tiles != 0, m, tot, rc, evaluated);
    ResAcc<float> ra;
    ra.init();
    const bool bal = bal_on<float>(ep, c);   // (block-uniform)
    MassAcc<float> mb;
    mb.init();
    // every lane of a row holds its (m, total); lane (q, l) finishes row
    // 16 (4 h + q) + l of the wave, so each epilogue round has all 64 lanes
    // busy (G / 4 rounds instead of G rounds of 16 lanes)
#pragma unroll
    for (int h = 0; h < G / 4; ++h) {
      const float mg = q == 0 ? m[4 * h] : (q == 1 ? m[4 * h + 1] : (q == 2 ? m[4 * h + 2] : m[4 * h + 3]));
      const float tg = q == 0 ? tot[4 * h] : (q == 1 ? tot[4 * h + 1] : (q == 2 ? tot[4 * h + 2] : tot[4 * h + 3]));
      const float rg = q == 0 ? rc[4 * h] : (q == 1 ? rc[4 * h + 1] : (q == 2 ? rc[4 * h + 2] : rc[4 * h + 3]));
      const int row = wv * (16 * G) + (4 * h + q) * 16 + li;
      if (row < I.nrows) {
        const float lse = mg == -__builtin_inff() ? mg : mg + rg + __builtin_log2f(tg);
        epi_elem<float>(rb + row, lse, c, side, ep, ra);
        if (bal) bal_elem<float>(rb + row, lse, c, side, ep, mb);
        pw[rb + row] = mg;
      }
    }
    epi_finish<float>(ep, ra, I.part);
    if (bal) block_lse_reduce<float>(mb.m, mb.s, ep.bal_m + I.part, ep.bal_s + I.part);
  }
  if (pairs) count_pairs<G>(pairs, evaluated);
}

bool tile_skip_enabled() {
  const char* e = std::getenv("UOT_TILE_SKIP");
  return !(e && e[0] == '0' && e[1] == 0);
}

void launch_dense_mf(int dim, int groups, bool split, const float* xr, int64_t Nr, const float* yc, const float* w,
                     int64_t Mc, int nsplit, int64_t cps, float* pm, float* ps, float* pw, int side, const Ctrl* c,
                     const MfSkip& sk, hipStream_t s) {
  // tiles are left out only within a single column split: with several,
  // each split's bound is relative to its own maximum, whose tile is always
  // kept, so little goes and the tile records cost more than they save
  const int skip = sk.on && nsplit == 1 ? 1 : 0;
#define UOT_MF(D, G, S)                                                                                        \
  hipLaunchKernelGGL((k_dense_mf<D, G, S>), dim3((unsigned)((Nr + 64 * G - 1) / (64 * G)), (unsigned)nsplit), \
                     dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, cps, pm, ps, pw, side, c, skip, sk.pairs)
#define UOT_MF_DIM(G, S)              \
  if (dim == 1) UOT_MF(1, G, S);      \
  else if (dim == 2) UOT_MF(2, G, S); \
  else UOT_MF(3, G, S);
  if (split) {
    if (groups == 8) {
      UOT_MF_DIM(8, true)
    } else {
      UOT_MF_DIM(4, true)
    }
  } else {
    if (groups == 8) {
      UOT_MF_DIM(8, false)
    } else {
      UOT_MF_DIM(4, false)
    }
  }
#undef UOT_MF_DIM
#undef UOT_MF
}

}  // namespace uot

namespace uot {

int batch_mf_resident_blocks(int dim, int groups) {
  int n = 0;
  hipError_t e = hipSuccess;
#define UOT_BMF_OCC(D, G) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_mf<D, G, true>, kBlock, 0)
  if (groups == 8) {
    if (dim == 1) UOT_BMF_OCC(1, 8);
    else if (dim == 2) UOT_BMF_OCC(2, 8);
    else UOT_BMF_OCC(3, 8);
  } else {
    if (dim == 1) UOT_BMF_OCC(1, 4);
    else if (dim == 2) UOT_BMF_OCC(2, 4);
    else UOT_BMF_OCC(3, 4);
  }
#undef UOT_BMF_OCC
  return e == hipSuccess && n > 0 ? n : 0;
}

void launch_batch_mf(int dim, int groups, int blocks, const BItem* items, const int* count, int* cursor,
                     const int64_t* offR, const int64_t* offC, const float* xr, int64_t totR, const float* yc,
                     int64_t totC, const float* w, float* pw, const BCtrl* bc, const Ctrl* c, int side,
                     const EpiArgs<float>& ep, const MfSkip& sk, hipStream_t s) {
#define UOT_BMF(D, G)                                                                                           \
  hipLaunchKernelGGL((k_batch_mf<D, G, true>), dim3(blocks), dim3(kBlock), 0, s, items, count, cursor, offR, offC, \
                     xr, totR, yc, totC, w, pw, bc, c, side, ep, sk.on, sk.pairs)
  if (groups == 8) {
    if (dim == 1) UOT_BMF(1, 8);
    else if (dim == 2) UOT_BMF(2, 8);
    else UOT_BMF(3, 8);
  } else {
    if (dim == 1) UOT_BMF(1, 4);
    else if (dim == 2) UOT_BMF(2, 4);
    else UOT_BMF(3, 4);
  }
#undef UOT_BMF
}

}  // namespace uot
