// Warm-start network for the scaling iteration: a 4-layer MLP
//   n_in -> width -> width -> width -> n_out   (ReLU on the hidden layers)
// predicting the dual potential v from the two input measures.  Only v^(0)
// matters for the iterates (Prop. "alternating": the first X half-step
// overwrites u), so a good v^(0) shortens the iteration while the iteration
// itself still decides the answer.
//
// Every GEMM input (weights and activations) is BF16, accumulation is FP32 on
// MFMA (v_mfma_f32_16x16x32_bf16); the optimiser keeps FP32 master weights
// (Adam).  Parameter layout in every parameter-sized array:
//   W1 [width x n_in], b1 [width], W2 [width x width], b2, W3 [width x width],
//   b3, W4 [n_out x width], b4 [n_out].
#include <hip/hip_runtime.h>
#include <cstdlib>

#include <cmath>
#include <vector>

#include "uot_ctx.h"
#include "uot_launch.h"

namespace uot {
namespace net {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kB = 256;

// FP32 -> BF16 bits, round to nearest even (NaN stays NaN)
__device__ __forceinline__ u16 f2bf(float f) {
  const uint32_t x = __float_as_uint(f);
  const uint32_t special = (x >> 16) | ((x & 0xffffu) ? 0x40u : 0u);   // Inf stays Inf, NaN stays NaN
  const uint32_t rounded = (x + 0x7fffu + ((x >> 16) & 1u)) >> 16;
  return (u16)((x & 0x7f800000u) == 0x7f800000u ? special : rounded);
}
__device__ __forceinline__ float bf2f(u16 b) { return __uint_as_float((uint32_t)b << 16); }

static inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// C[M x N] = op(A)[M x K] * op(B)[K x N] (+ bias[n]) (ReLU), BF16 in, FP32 acc.
//   TA = false: A[m][k] = A[m*lda + k];  TA = true: A[m][k] = A[k*lda + m]
//   TB = false: B[k][n] = B[k*ldb + n];  TB = true: B[k][n] = B[n*ldb + k]
// Block tile 64 x 64, K tile 32, 4 waves of 32 x 32 (2 x 2 MFMA 16x16x32).
// Split K (blockIdx.z): each block sums the K range [z kc, (z + 1) kc) and
// stores its partial tile in P[z] (M x N, row-major); k_splitk_reduce then
// adds the partials in a fixed order, with the bias, into C.  Used when there
// are too few output tiles to fill the chip and the caller gives room for the
// partials.
// Operands move as 16-byte vectors along their contiguous axis where the
// leading dimension and the tile edge allow, element by element otherwise.
// ---------------------------------------------------------------------------
constexpr int TM = 64, TN = 64, TK = 32, LK = TK + 8;

// 8 consecutive u16 from p (16-byte aligned), or element by element with
// zeros past `avail` elements
__device__ __forceinline__ void load8(const u16* __restrict__ p, int avail, bool vec, u16 (&v)[8]) {
  if (vec && avail >= 8) {
    const uint4 q = *reinterpret_cast<const uint4*>(p);
    __builtin_memcpy(v, &q, sizeof(q));
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = j < avail ? p[j] : (u16)0;
  }
}

// LDS tiles are stored with their 16-byte k chunks permuted per row: element
// (row, k) sits at column k ^ (sw(row) << 3), which keeps every 8-element
// chunk whole (the MFMA operand reads stay single 16-byte reads) and spreads
// over the banks the rows that one store or read instruction touches: the
// element-wise stores of transposed tiles (rows 8 apart), the 16-byte stores
// (4 rows of 4 chunks) and the operand reads (16 rows, one chunk).  sw takes
// row bits 5, 4 (and 0 for whole-K tiles, whose rows hold 32 chunks).
__device__ __forceinline__ int sw_step(int r) { return ((r >> 5) & 1) | (((r >> 4) & 1) << 1); }
__device__ __forceinline__ int sw_whole(int r) { return sw_step(r) | ((r & 1) << 2); }

// One 64 x 32 operand tile, as T[row][k] in LDS, moved in two steps so the
// global loads of the next K tile overlap the MFMAs of the current one:
// fetch_tile (global -> 8 registers per thread), store_tile (registers ->
// LDS).  Row-major source (rows contiguous in k) when !TRANS, k-major source
// (rows contiguous) when TRANS.
template <bool TRANS>
__device__ __forceinline__ void fetch_tile(u16 (&v)[8], const u16* __restrict__ X, int64_t ld, int r0, int R, int k0,
                                           int kend, bool vec) {
  const int tid = threadIdx.x;
  if (!TRANS) {
    const int r = tid >> 2, c = (tid & 3) * 8;
    const int row = r0 + r, k = k0 + c;
    const int avail = (row < R) ? (kend - k) : 0;
    load8(X + (int64_t)(row < R ? row : 0) * ld + (k < kend ? k : 0), avail, vec, v);
  } else {
    const int kk = tid >> 3, c = (tid & 7) * 8;
    const int k = k0 + kk, row = r0 + c;
    const int avail = (k < kend) ? (R - row) : 0;
    load8(X + (int64_t)(k < kend ? k : 0) * ld + (row < R ? row : 0), avail, vec, v);
  }
}

template <bool TRANS>
__device__ __forceinline__ void store_tile(u16 (*T)[LK], const u16 (&v)[8]) {
  const int tid = threadIdx.x;
  if (!TRANS) {
    const int r = tid >> 2, c = (tid & 3) * 8;
    uint4 q;
    __builtin_memcpy(&q, v, sizeof(q));
    *reinterpret_cast<uint4*>(&T[r][c ^ (sw_step(r) << 3)]) = q;
  } else {
    const int kk = tid >> 3, c = (tid & 7) * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) T[c + j][kk ^ (sw_step(c + j) << 3)] = v[j];
  }
}

// store_tile into a whole-K LDS array (rows of LW elements) at column k0
template <bool TRANS, int LD>
__device__ __forceinline__ void store_tile_at(u16 (*T)[LD], int k0, const u16 (&v)[8]) {
  const int tid = threadIdx.x;
  if (!TRANS) {
    const int r = tid >> 2, c = (tid & 3) * 8;
    uint4 q;
    __builtin_memcpy(&q, v, sizeof(q));
    *reinterpret_cast<uint4*>(&T[r][(k0 + c) ^ (sw_whole(r) << 3)]) = q;
  } else {
    const int kk = tid >> 3, c = (tid & 7) * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) T[c + j][(k0 + kk) ^ (sw_whole(c + j) << 3)] = v[j];
  }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(kB) void k_gemm(const u16* __restrict__ A, int64_t lda, const u16* __restrict__ Bm,
                                              int64_t ldb, int M, int N, int K, float* __restrict__ C, int64_t ldc,
                                              u16* __restrict__ Cb, const float* __restrict__ bias, int relu, int kc,
                                              float* __restrict__ P) {
  __shared__ __align__(16) u16 As[TM][LK];
  __shared__ __align__(16) u16 Bs[TN][LK];
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = blockIdx.z * kc;
  const int ke = kb + kc < K ? kb + kc : K;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  // 16-byte loads need 8-element aligned rows (base pointers are 256-byte aligned)
  const bool va = (lda % 8) == 0 && (reinterpret_cast<uintptr_t>(A) % 16) == 0;
  const bool vb = (ldb % 8) == 0 && (reinterpret_cast<uintptr_t>(Bm) % 16) == 0;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  u16 ra[8], rb[8];
  fetch_tile<TA>(ra, A, lda, m0, M, kb, ke, va);
  fetch_tile<!TB>(rb, Bm, ldb, n0, N, kb, ke, vb);
  for (int k0 = kb; k0 < ke; k0 += TK) {
    store_tile<TA>(As, ra);
    store_tile<!TB>(Bs, rb);
    __syncthreads();
    if (k0 + TK < ke) {
      fetch_tile<TA>(ra, A, lda, m0, M, k0 + TK, ke, va);
      fetch_tile<!TB>(rb, Bm, ldb, n0, N, k0 + TK, ke, vb);
    }
    // operand layout of v_mfma_f32_16x16x32_bf16: lane l holds row (l % 16)
    // of A and column (l % 16) of B, k = 8 (l / 16) .. 8 (l / 16) + 7
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ra_ = wm + i * 16 + (lane & 15);
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[ra_][((lane >> 4) * 8) ^ (sw_step(ra_) << 3)]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int rb_ = wn + j * 16 + (lane & 15);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[rb_][((lane >> 4) * 8) ^ (sw_step(rb_) << 3)]);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // result layout: lane l holds rows 4 (l / 16) + r (r = 0..3), column l % 16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m < M && n < N) {
          float x = acc[i][j][r];
          if (P) {
            P[((int64_t)blockIdx.z * M + m) * N + n] = x;
          } else {
            if (bias) x += bias[n];
            if (relu) x = x > 0.f ? x : 0.f;
            if (C) C[(int64_t)m * ldc + n] = x;
            if (Cb) Cb[(int64_t)m * ldc + n] = f2bf(x);
          }
        }
      }
}

// The same product for a K range of at most kWholeK per block (every product
// of the network at batch 256 after its K split): the block loads its whole
// K range of both operands into LDS first (every global load in flight at
// once, one memory round trip), then runs the MFMAs of all K tiles; the
// stepped kernel above waits for one round trip per K tile.
constexpr int kWholeK = 256, LW = kWholeK + 8;

// Block coordinates (output tile column, row, K range).  Workgroups go to
// the 8 XCDs round-robin by linear id; with a K split of a multiple of 8
// ranges, the tiles of one K range are all placed on one XCD, so each K
// slice of both operands is fetched into one L2 and read there by every tile
// that needs it (the plain order spreads them over 2-4 XCDs, each fetching
// its own copy).
__device__ __forceinline__ void block_coords(int& bx, int& by, int& bz) {
  const int nx = gridDim.x, ny = gridDim.y, nz = gridDim.z;
  if (nz % 8 != 0) {
    bx = blockIdx.x;
    by = blockIdx.y;
    bz = blockIdx.z;
    return;
  }
  const int nxy = nx * ny;
  const int id = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const int slot = id >> 3, t = slot % nxy;
  bz = (id & 7) + 8 * (slot / nxy);
  bx = t % nx;
  by = t / nx;
}

// FULL: every tile of the launch lies inside both operands and the result
// (M, N multiples of 64, K a multiple of kc, kc of 32) and both operands move
// as 16-byte vectors: no bounds tests and no element-wise fallback, which
// keeps the kernel a fraction of the general one's code.
template <bool TRANS>
__device__ __forceinline__ void fetch_full(u16 (&v)[8], const u16* __restrict__ X, int64_t ld, int r0, int k0) {
  const int tid = threadIdx.x;
  const u16* p = !TRANS ? X + (int64_t)(r0 + (tid >> 2)) * ld + k0 + (tid & 3) * 8
                        : X + (int64_t)(k0 + (tid >> 3)) * ld + r0 + (tid & 7) * 8;
  const uint4 q = *reinterpret_cast<const uint4*>(p);
  __builtin_memcpy(v, &q, sizeof(q));
}

template <bool TA, bool TB, bool FULL>
__global__ __launch_bounds__(kB) void k_gemm_whole(const u16* __restrict__ A, int64_t lda,
                                                    const u16* __restrict__ Bm, int64_t ldb, int M, int N, int K,
                                                    float* __restrict__ C, int64_t ldc, u16* __restrict__ Cb,
                                                    const float* __restrict__ bias, int relu, int kc,
                                                    float* __restrict__ P) {
  extern __shared__ __align__(16) u16 lds[];
  u16(*As)[LW] = reinterpret_cast<u16(*)[LW]>(lds);
  u16(*Bs)[LW] = reinterpret_cast<u16(*)[LW]>(lds + TM * LW);
  int bx, by, bz;
  block_coords(bx, by, bz);
  const int m0 = by * TM, n0 = bx * TN;
  const int kb = bz * kc;
  const int ke = kb + kc < K ? kb + kc : K;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const bool va = (lda % 8) == 0 && (reinterpret_cast<uintptr_t>(A) % 16) == 0;
  const bool vb = (ldb % 8) == 0 && (reinterpret_cast<uintptr_t>(Bm) % 16) == 0;
  const int nkt = (ke - kb + TK - 1) / TK;   // K tiles of this block, <= kWholeK / TK
  u16 ra[kWholeK / TK][8], rb[kWholeK / TK][8];
#pragma unroll
  for (int t = 0; t < kWholeK / TK; ++t) {
    if (t < nkt) {
      if constexpr (FULL) {
        fetch_full<TA>(ra[t], A, lda, m0, kb + t * TK);
        fetch_full<!TB>(rb[t], Bm, ldb, n0, kb + t * TK);
      } else {
        fetch_tile<TA>(ra[t], A, lda, m0, M, kb + t * TK, ke, va);
        fetch_tile<!TB>(rb[t], Bm, ldb, n0, N, kb + t * TK, ke, vb);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kWholeK / TK; ++t) {
    if (t < nkt) {
      store_tile_at<TA>(As, t * TK, ra[t]);
      store_tile_at<!TB>(Bs, t * TK, rb[t]);
    }
  }
  __syncthreads();
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int t = 0; t < nkt; ++t) {
    const int kk = t * TK + (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ra_ = wm + i * 16 + (lane & 15);
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[ra_][kk ^ (sw_whole(ra_) << 3)]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int rb_ = wn + j * 16 + (lane & 15);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[rb_][kk ^ (sw_whole(rb_) << 3)]);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
      }
    }
  }
  // result layout: lane l holds rows 4 (l / 16) + r (r = 0..3), column l % 16
  float* const Pz = P ? P + (int64_t)bz * M * N : nullptr;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = n0 + wn + j * 16 + (lane & 15);
    const float bn = (!P && bias && (FULL || n < N)) ? bias[n] : 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int mb = m0 + wm + i * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mb + r;
        if (FULL || (m < M && n < N)) {
          float x = acc[i][j][r];
          if (Pz) {
            Pz[(int64_t)m * N + n] = x;
          } else {
            x += bn;
            if (relu) x = x > 0.f ? x : 0.f;
            if (C) C[(int64_t)m * ldc + n] = x;
            if (Cb) Cb[(int64_t)m * ldc + n] = f2bf(x);
          }
        }
      }
    }
  }
}

// C[m][n] = bias[n] + sum_z P[z][m][n] (z in order: the result does not
// depend on the schedule)
__global__ void k_splitk_reduce(const float* __restrict__ P, int S, int M, int N, const float* __restrict__ bias,
                                float* __restrict__ C, int64_t ldc) {
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (t >= (int64_t)M * N) return;
  const int64_t mn = (int64_t)M * N;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  int z = 0;
  for (; z + 4 <= S; z += 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += P[(z + k) * mn + t];
  }
  for (; z < S; ++z) acc[0] += P[z * mn + t];
  const int n = (int)(t % N);
  C[(t / N) * ldc + n] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + (bias ? bias[n] : 0.f);
}

constexpr int kMaxSplitK = 32;

// K-splits for a product: enough blocks for the chip (>= 512) when the
// output has few tiles and K is long; 1 when the result needs ReLU or BF16
// (those are not additive)
static int gemm_splits(int M, int N, int K, bool additive) {
  if (!additive) return 1;
  const int64_t tiles = (int64_t)cdiv(M, TM) * cdiv(N, TN);
  int s = 1;
  while (tiles * s < 512 && K / (2 * s) >= 256 && 2 * s <= kMaxSplitK) s *= 2;
  return s;
}

// floats of partials a product needs (0: no split)
static int64_t gemm_partials(int M, int N, int K, bool additive) {
  const int sp = gemm_splits(M, N, K, additive);
  return sp > 1 ? (int64_t)sp * M * N : 0;
}

template <bool TA, bool TB>
static void gemm(const u16* A, int64_t lda, const u16* B, int64_t ldb, int M, int N, int K, float* C, int64_t ldc,
                 u16* Cb, const float* bias, int relu, hipStream_t s, float* part = nullptr,
                 int64_t part_floats = 0) {
  const bool additive = C != nullptr && Cb == nullptr && !relu;
  int sp = gemm_splits(M, N, K, additive);
  if (!part || (int64_t)sp * M * N > part_floats) sp = 1;
  const int kc = sp > 1 ? (int)(cdiv(cdiv(K, sp), TK) * TK) : K;
  const int sz = sp > 1 ? (int)cdiv(K, kc) : 1;
  const dim3 grid(cdiv(N, TN), cdiv(M, TM), sz);
  constexpr int whole_lds = 2 * TM * LW * sizeof(u16);   // 66 KB: above the default 64 KB limit
  static const bool whole_ok = [] {
    bool ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_whole<TA, TB, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, whole_lds) == hipSuccess;
    ok = ok && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_whole<TA, TB, true>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, whole_lds) == hipSuccess;
    if (!ok) (void)hipGetLastError();   // the stepped kernel runs instead; clear the error
    return ok;
  }();
  // 16-byte rows (leading dimensions of 8 elements, 16-byte aligned bases)
  // and whole tiles everywhere: the bounds-free kernel
  const bool full = lda % 8 == 0 && ldb % 8 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
                    reinterpret_cast<uintptr_t>(B) % 16 == 0 && M % TM == 0 && N % TN == 0 && kc % TK == 0 &&
                    K % kc == 0;
  if (kc <= kWholeK && whole_ok && full)
    hipLaunchKernelGGL((k_gemm_whole<TA, TB, true>), grid, dim3(kB), whole_lds, s, A, lda, B, ldb, M, N, K, C, ldc,
                       Cb, bias, relu, kc, sz > 1 ? part : nullptr);
  else if (kc <= kWholeK && whole_ok)
    hipLaunchKernelGGL((k_gemm_whole<TA, TB, false>), grid, dim3(kB), whole_lds, s, A, lda, B, ldb, M, N, K, C, ldc,
                       Cb, bias, relu, kc, sz > 1 ? part : nullptr);
  else
    hipLaunchKernelGGL((k_gemm<TA, TB>), grid, dim3(kB), 0, s, A, lda, B, ldb, M, N, K, C, ldc, Cb, bias, relu, kc,
                       sz > 1 ? part : nullptr);
  if (sz > 1)
    hipLaunchKernelGGL(k_splitk_reduce, dim3(cdiv((int64_t)M * N, kB)), dim3(kB), 0, s, part, sz, M, N, bias, C,
                       ldc);
}

// y = bf16(scale * x + shift)
__global__ void k_cast(const float* __restrict__ x, u16* __restrict__ y, int64_t n, float scale, float shift) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) y[i] = f2bf(scale * x[i] + shift);
}

// g = bf16(coef * (y - t)); part[block] = sum (y - t)^2
__global__ void k_loss_grad(const float* __restrict__ y, const float* __restrict__ t, u16* __restrict__ g, int64_t n,
                            float coef, double* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  double e2 = 0.0;
  if (i < n) {
    const float d = y[i] - t[i];
    if (g) g[i] = f2bf(coef * d);
    e2 = double(d) * double(d);
  }
  __shared__ double sm[kB];
  sm[threadIdx.x] = e2;
  __syncthreads();
  for (int off = kB / 2; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) sm[threadIdx.x] += sm[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// g = bf16(dh) where the pre-activation z > 0, else 0
__global__ void k_relu_grad(const float* __restrict__ dh, const float* __restrict__ z, u16* __restrict__ g, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) g[i] = z[i] > 0.f ? f2bf(dh[i]) : (u16)0;
}

// out[n] = sum_b g[b][n]  (bias gradients): 64 columns per block (one row
// segment of 128 bytes per load), the 4 waves take every 4th row with 4
// independent partial sums each, merged in LDS (fixed order)
__global__ __launch_bounds__(kB) void k_colsum(const u16* __restrict__ g, int rows, int cols, float* __restrict__ out) {
  __shared__ float part[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (n < cols) {
    int b = wv;
    for (; b + 12 < rows; b += 16) {
      s0 += bf2f(g[(int64_t)b * cols + n]);
      s1 += bf2f(g[(int64_t)(b + 4) * cols + n]);
      s2 += bf2f(g[(int64_t)(b + 8) * cols + n]);
      s3 += bf2f(g[(int64_t)(b + 12) * cols + n]);
    }
    for (; b < rows; b += 4) s0 += bf2f(g[(int64_t)b * cols + n]);
  }
  part[wv][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (wv == 0 && n < cols) out[n] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// Adam with bias correction; refreshes the BF16 copy of the weights
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       u16* __restrict__ wb, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wb[i] = f2bf(wi);
}

__global__ void k_to_bf16(const float* __restrict__ w, u16* __restrict__ wb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) wb[i] = f2bf(w[i]);
}

// features of a grid pair: 2x2..sxs average pooling of p and q from R x R to
// r x r (R = s r), then x[b] = [log p_r, log q_r]
__global__ void k_features(const float* __restrict__ p, const float* __restrict__ q, int64_t nb, int R, int r,
                           float* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  const int64_t per = (int64_t)r * r;
  if (t >= nb * per * 2) return;
  const int64_t b = t / (2 * per);
  const int which = (int)((t / per) % 2);
  const int64_t cell = t % per;
  const int i = (int)(cell / r), j = (int)(cell % r);
  const int s = R / r;
  const float* src = (which == 0 ? p : q) + b * (int64_t)R * R;
  float acc = 0.f;
  for (int a = 0; a < s; ++a)
    for (int c = 0; c < s; ++c) acc += src[(int64_t)(i * s + a) * R + (j * s + c)];
  acc /= float(s * s);
  x[b * 2 * per + which * per + cell] = acc > 0.f ? logf(acc) : -80.f;
}

// bilinear upsampling of r x r cell-centred fields to R x R (clamped at the border)
__global__ void k_upsample(const float* __restrict__ y, int64_t nb, int r, int R, float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  const int64_t per = (int64_t)R * R;
  if (t >= nb * per) return;
  const int64_t b = t / per;
  const int i = (int)((t % per) / R), j = (int)(t % R);
  const float sc = float(r) / float(R);
  float fi = (i + 0.5f) * sc - 0.5f, fj = (j + 0.5f) * sc - 0.5f;
  fi = fminf(fmaxf(fi, 0.f), float(r - 1));
  fj = fminf(fmaxf(fj, 0.f), float(r - 1));
  const int i0 = (int)floorf(fi), j0 = (int)floorf(fj);
  const int i1 = i0 + 1 < r ? i0 + 1 : r - 1, j1 = j0 + 1 < r ? j0 + 1 : r - 1;
  const float a = fi - i0, c = fj - j0;
  const float* src = y + b * (int64_t)r * r;
  out[t] = (1 - a) * ((1 - c) * src[i0 * r + j0] + c * src[i0 * r + j1]) +
           a * ((1 - c) * src[i1 * r + j0] + c * src[i1 * r + j1]);
}

// first barycentre estimate for the warm start: the pointwise combination of
// Table estimatebary applied to the input densities themselves,
// (i) equality: log h = sum_k alpha_k log p_k / sum alpha;
// (ii) lam KL: log h = ((eps+lam)/eps) [LSE_k(log alpha_k + eps/(eps+lam) log p_k) - log sum alpha]
__global__ void k_bary_estimate(const float* __restrict__ p, int n, int64_t size, BaryW la, double log_sum_alpha,
                                float eps, float lam, int kind, float* __restrict__ h) {
  const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (j >= size) return;
  float logh;
  if (kind == 0) {
    double acc = 0.0, asum = 0.0;
    for (int k = 0; k < n; ++k) {
      const double al = ::exp(la.v[k]);
      acc += al * ::log((double)p[k * size + j]);
      asum += al;
    }
    logh = float(acc / asum);
  } else {
    const float g = eps / (eps + lam);
    float m = -__builtin_inff();
    for (int k = 0; k < n; ++k) m = fmaxf(m, float(la.v[k]) + g * logf(p[k * size + j]));
    float s = 0.f;
    for (int k = 0; k < n; ++k) s += expf(float(la.v[k]) + g * logf(p[k * size + j]) - m);
    logh = (m + logf(s) - float(log_sum_alpha)) / g;
  }
  h[j] = expf(logh);
}

// local (no transport) estimate of the barycentre potentials on a 2-D grid:
// with K replaced by its row mass kappa_i = sum_j dy_j exp(-|x_i - y_j|^2/eps)
// at each cell, the KL(lam) coupling between p_k and h reduces to the
// one-point problem at that cell, whose plan density is
//   log r = (lam log p_k + lam log h + eps log kappa) / (2 lam + eps)
// and whose second potential is v = -lam log(r / h).  kappa is the product of
// the two 1-D kernel masses of the cell.
__global__ void k_bary_local_v0(const float* __restrict__ p, const float* __restrict__ h0, int n, int n1, int n2,
                                float h1, float h2, float lam, float eps, float* __restrict__ v0) {
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  const int64_t size = (int64_t)n1 * n2;
  if (t >= (int64_t)n * size) return;
  const int64_t cell = t % size;
  const int i1 = (int)(cell / n2), i2 = (int)(cell % n2);
  float k1 = 0.f, k2 = 0.f;
  for (int j = 0; j < n1; ++j) {
    const float d = h1 * float(i1 - j);
    k1 += h1 * expf(-d * d / eps);
  }
  for (int j = 0; j < n2; ++j) {
    const float d = h2 * float(i2 - j);
    k2 += h2 * expf(-d * d / eps);
  }
  const float lh = logf(h0[cell]);
  const float logr = (lam * logf(p[t]) + lam * lh + eps * (logf(k1) + logf(k2))) / (2.f * lam + eps);
  v0[t] = -lam * (logr - lh);
}

// ---------------------------------------------------------------------------
// warm start of ragged point-cloud batches: per-point features of the
// second cloud (the side v lives on) and the composition of v^(0)
// ---------------------------------------------------------------------------
__global__ void k_log_sum(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ out,
                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) out[i] = logf(a[i]) + logf(b[i]);
}

struct FeatNorm {
  float shift[kCloudFeatures], scale[kCloudFeatures];
};

// x[j][k] = (c_k(j) - shift_k) scale_k with c_0 = eps log q_j, c_1..c_np the
// Gibbs products prod[k-1][j] (natural log) times eps, and the last column
// eps log(N_b / M_b) of the problem b that point j belongs to
__global__ void k_cloud_assemble(const float* __restrict__ prod, int n_prod, const float* __restrict__ logq,
                                 const int64_t* __restrict__ offN, const int64_t* __restrict__ offM, int64_t B,
                                 int64_t totM, float eps, FeatNorm nm, float* __restrict__ x) {
  const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (j >= totM) return;
  int64_t lo = 0, hi = B;   // offM[lo] <= j < offM[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (offM[mid] <= j) lo = mid;
    else hi = mid;
  }
  float c[kCloudFeatures];
  c[0] = eps * logq[j];
  for (int k = 0; k < kCloudFeatures - 2; ++k) c[k + 1] = k < n_prod ? eps * prod[(int64_t)k * totM + j] : 0.f;
  c[kCloudFeatures - 1] = eps * logf(float(offN[lo + 1] - offN[lo]) / float(offM[lo + 1] - offM[lo]));
  float* xo = x + j * kCloudFeatures;
#pragma unroll
  for (int k = 0; k < kCloudFeatures; ++k) xo[k] = (c[k] - nm.shift[k]) * nm.scale[k];
}

// out_i = log sum_j exp(w_j) over the columns j of the problem that row i
// belongs to, on every row of it: the product of a kernel equal to 1 (a
// total mass), which needs no pair.  One block per problem: the maximum,
// then the sum of exp(w_j - max) accumulated in FP64.
__global__ void k_problem_lse(const float* __restrict__ w, const int64_t* __restrict__ offC,
                              const int64_t* __restrict__ offR, float* __restrict__ out) {
  __shared__ float sm[kB / 64];
  __shared__ double ss[kB / 64];
  const int64_t b = blockIdx.x;
  const int64_t c0 = offC[b], c1 = offC[b + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float m = -__builtin_inff();
  for (int64_t j = c0 + threadIdx.x; j < c1; j += kB) m = fmaxf(m, w[j]);
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane == 0) sm[wv] = m;
  __syncthreads();
  m = sm[0];
  for (int k = 1; k < kB / 64; ++k) m = fmaxf(m, sm[k]);
  double acc = 0.0;
  if (m > -__builtin_inff())
    for (int64_t j = c0 + threadIdx.x; j < c1; j += kB) acc += (double)expf(w[j] - m);
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) ss[wv] = acc;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < kB / 64; ++k) t += ss[k];
  const float r = m > -__builtin_inff() ? m + (float)log(t) : m;
  for (int64_t i = offR[b] + threadIdx.x; i < offR[b + 1]; i += kB) out[i] = r;
}

// v0_j = z eps log q_j + out_scale y_j + out_shift (the network predicts the
// smooth part of v, the pointwise part z eps log q_j is exact)
__global__ void k_cloud_v0(const float* __restrict__ y, const float* __restrict__ q, int64_t n, float zeps,
                           float out_scale, float out_shift, float* __restrict__ v0) {
  const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (j < n) v0[j] = zeps * logf(q[j]) + out_scale * y[j] + out_shift;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Layout {
  int64_t w[4], b[4], total;
  int in[4], out[4];
};

Layout layout(const uot_net* n) {
  Layout L;
  const int ins[4] = {n->n_in, n->width, n->width, n->width};
  const int outs[4] = {n->width, n->width, n->width, n->n_out};
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    L.in[l] = ins[l];
    L.out[l] = outs[l];
    L.w[l] = o;
    o += (int64_t)ins[l] * outs[l];
    L.b[l] = o;
    o += outs[l];
  }
  L.total = o;
  return L;
}

struct Act {
  u16* xb;          // batch x n_in
  float* z[3];      // pre-activations, batch x width
  u16* h[3];        // BF16 hidden activations
  float* y;         // batch x n_out
  u16* g4;          // batch x n_out
  float* dh;        // batch x width
  u16* g;           // batch x width
  double* part;     // loss partials
  float* grad;      // gradient (parameter-sized)
  float* splitk;    // split-K partials of the long-K products
  int64_t splitk_floats;
  size_t total;
};

Act carve(const uot_net* n, int64_t batch, char* ws) {
  Act a;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = (o + bytes + 255) / 256 * 256;
    return ws ? ws + r : nullptr;
  };
  const Layout L = layout(n);
  a.xb = reinterpret_cast<u16*>(take(2 * batch * n->n_in));
  for (int l = 0; l < 3; ++l) {
    a.z[l] = reinterpret_cast<float*>(take(4 * batch * n->width));
    a.h[l] = reinterpret_cast<u16*>(take(2 * batch * n->width));
  }
  a.y = reinterpret_cast<float*>(take(4 * batch * n->n_out));
  a.g4 = reinterpret_cast<u16*>(take(2 * batch * n->n_out));
  a.dh = reinterpret_cast<float*>(take(4 * batch * n->width));
  a.g = reinterpret_cast<u16*>(take(2 * batch * n->width));
  a.part = reinterpret_cast<double*>(take(8 * (size_t)cdiv(batch * n->n_out, kB)));
  a.grad = reinterpret_cast<float*>(take(4 * L.total));
  // the additive products that can split: layer 1 forward, input gradients
  int64_t sk = gemm_partials((int)batch, L.out[0], L.in[0], true);
  for (int l = 1; l < 4; ++l) sk = std::max(sk, gemm_partials((int)batch, L.in[l], L.out[l], true));
  a.splitk_floats = sk;
  a.splitk = reinterpret_cast<float*>(take(4 * (size_t)sk));
  a.total = o;
  return a;
}

int check_net(const uot_net* n) {
  if (!n) return fail(UOT_E_INVALID, "net is NULL");
  if (n->n_in < 1 || n->width < 1 || n->n_out < 1) return fail(UOT_E_INVALID, "net sizes must be >= 1");
  if (n->width % 8 || n->n_in % 8) return fail(UOT_E_UNSUPPORTED, "n_in and width must be multiples of 8");
  return UOT_OK;
}

// train: keep the FP32 pre-activations z for the backward pass; inference
// writes only the BF16 activations, bias and ReLU applied in the product's
// epilogue (the same values: bf16(max(z, 0)))
void forward(const uot_net* n, const Layout& L, const Act& a, const float* x, int64_t batch, hipStream_t s,
             bool train = true) {
  hipLaunchKernelGGL(k_cast, dim3(cdiv(batch * n->n_in, kB)), dim3(kB), 0, s, x, a.xb, batch * n->n_in, n->in_scale,
                     n->in_shift);
  const u16* inp = a.xb;
  for (int l = 0; l < 3; ++l) {
    if (!train) {
      gemm<false, true>(inp, L.in[l], n->wbf16 + L.w[l], L.in[l], (int)batch, L.out[l], L.in[l], nullptr, L.out[l],
                        a.h[l], n->master + L.b[l], 1, s);
      inp = a.h[l];
      continue;
    }
    gemm<false, true>(inp, L.in[l], n->wbf16 + L.w[l], L.in[l], (int)batch, L.out[l], L.in[l], a.z[l], L.out[l],
                      nullptr, n->master + L.b[l], 0, s, a.splitk, a.splitk_floats);
    // ReLU copy in BF16 (z keeps the pre-activation for the backward mask)
    hipLaunchKernelGGL(k_relu_grad, dim3(cdiv(batch * L.out[l], kB)), dim3(kB), 0, s, a.z[l], a.z[l], a.h[l],
                       batch * L.out[l]);
    inp = a.h[l];
  }
  gemm<false, true>(inp, L.in[3], n->wbf16 + L.w[3], L.in[3], (int)batch, L.out[3], L.in[3], a.y, L.out[3], nullptr,
                    n->master + L.b[3], 0, s);
}

// gradient of loss = mean (y - t)^2 over batch x n_out into a.grad
void backward(const uot_net* n, const Layout& L, const Act& a, const float* t, int64_t batch, hipStream_t s) {
  const int64_t ny = batch * n->n_out;
  hipLaunchKernelGGL(k_loss_grad, dim3(cdiv(ny, kB)), dim3(kB), 0, s, a.y, t, a.g4, ny, 2.f / float(ny), a.part);
  const u16* g = a.g4;
  for (int l = 3; l >= 0; --l) {
    const u16* inp = l == 0 ? a.xb : a.h[l - 1];
    // dW_l [out x in] = g^T [out x batch] * inp [batch x in]
    gemm<true, false>(g, L.out[l], inp, L.in[l], L.out[l], L.in[l], (int)batch, a.grad + L.w[l], L.in[l], nullptr,
                      nullptr, 0, s);
    hipLaunchKernelGGL(k_colsum, dim3(cdiv(L.out[l], 64)), dim3(kB), 0, s, g, (int)batch, L.out[l], a.grad + L.b[l]);
    if (l == 0) break;
    // dh_{l-1} [batch x in] = g [batch x out] * W_l [out x in], then the ReLU mask
    gemm<false, false>(g, L.out[l], n->wbf16 + L.w[l], L.in[l], (int)batch, L.in[l], L.out[l], a.dh, L.in[l], nullptr,
                       nullptr, 0, s, a.splitk, a.splitk_floats);
    hipLaunchKernelGGL(k_relu_grad, dim3(cdiv(batch * L.in[l], kB)), dim3(kB), 0, s, a.dh, a.z[l - 1], a.g,
                       batch * L.in[l]);
    g = a.g;
  }
}

double loss_from_parts(const Act& a, int64_t ny, hipStream_t s, int* rc) {
  const int nb = (int)cdiv(ny, kB);
  std::vector<double> h(nb);
  *rc = UOT_OK;
  if (hipStreamSynchronize(s) != hipSuccess || hipMemcpy(h.data(), a.part, 8 * nb, hipMemcpyDeviceToHost) != hipSuccess) {
    *rc = fail(UOT_E_HIP, "loss readback failed");
    return 0.0;
  }
  double tot = 0.0;
  for (double v : h) tot += v;
  return tot / double(ny);
}

}  // namespace net

void launch_log_sum(const float* a, const float* b, float* out, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(net::k_log_sum, dim3(net::cdiv(n, net::kB)), dim3(net::kB), 0, s, a, b, out, n);
}

void launch_cloud_assemble(const float* prod, int n_prod, const float* logq, const int64_t* offN, const int64_t* offM,
                           int64_t B, int64_t totM, float eps, const float* shift, const float* scale, float* x,
                           hipStream_t s) {
  net::FeatNorm nm;
  for (int k = 0; k < kCloudFeatures; ++k) {
    nm.shift[k] = shift[k];
    nm.scale[k] = scale[k];
  }
  if (totM > 0)
    hipLaunchKernelGGL(net::k_cloud_assemble, dim3(net::cdiv(totM, net::kB)), dim3(net::kB), 0, s, prod, n_prod, logq,
                       offN, offM, B, totM, eps, nm, x);
}

void launch_problem_lse(const float* w, const int64_t* offC, const int64_t* offR, int64_t B, float* out,
                        hipStream_t s) {
  if (B > 0) hipLaunchKernelGGL(net::k_problem_lse, dim3((unsigned)B), dim3(net::kB), 0, s, w, offC, offR, out);
}

void launch_cloud_v0(const float* y, const float* q, int64_t n, float zeps, float out_scale, float out_shift,
                     float* v0, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(net::k_cloud_v0, dim3(net::cdiv(n, net::kB)), dim3(net::kB), 0, s, y, q, n, zeps, out_scale,
                       out_shift, v0);
}

}  // namespace uot

using namespace uot;
using namespace uot::net;

extern "C" {

int uot_net_param_count(const uot_net* n, int64_t* count) {
  int rc = check_net(n);
  if (rc) return rc;
  if (!count) return fail(UOT_E_INVALID, "count is NULL");
  *count = layout(n).total;
  return UOT_OK;
}

int uot_net_workspace_size(const uot_net* n, int64_t batch, size_t* bytes) {
  int rc = check_net(n);
  if (rc) return rc;
  if (batch < 1 || !bytes) return fail(UOT_E_INVALID, "batch >= 1 and bytes are required");
  *bytes = carve(n, batch, nullptr).total;
  return UOT_OK;
}

int uot_net_sync(uot_ctx* ctx, const uot_net* n) {
  int rc = check_net(n);
  if (rc) return rc;
  if (!ctx || !n->master || !n->wbf16) return fail(UOT_E_INVALID, "ctx, master and wbf16 are required");
  if ((rc = begin(ctx))) return rc;
  const int64_t tot = layout(n).total;
  hipLaunchKernelGGL(k_to_bf16, dim3(cdiv(tot, kB)), dim3(kB), 0, ctx->work, n->master, n->wbf16, tot);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

int uot_warmstart_infer(uot_ctx* ctx, const uot_net* n, const float* x, float* y, int64_t batch, void* ws,
                        size_t wsb) {
  int rc = check_net(n);
  if (rc) return rc;
  if (!ctx || !x || !y || batch < 1 || !n->master || !n->wbf16) return fail(UOT_E_INVALID, "bad arguments");
  const Act a0 = carve(n, batch, nullptr);
  if (!ws || wsb < a0.total) return fail(UOT_E_WORKSPACE, "workspace too small");
  if ((rc = begin(ctx))) return rc;
  const Layout L = layout(n);
  Act a = carve(n, batch, static_cast<char*>(ws));
  forward(n, L, a, x, batch, ctx->work, false);
  HIP_TRY(hipMemcpyAsync(y, a.y, 4 * batch * n->n_out, hipMemcpyDeviceToDevice, ctx->work));
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

int uot_net_grad(uot_ctx* ctx, const uot_net* n, const float* x, const float* t, int64_t batch, float* grad,
                 double* loss, void* ws, size_t wsb) {
  int rc = check_net(n);
  if (rc) return rc;
  if (!ctx || !x || !t || !grad || batch < 1 || !n->master || !n->wbf16) return fail(UOT_E_INVALID, "bad arguments");
  const Act a0 = carve(n, batch, nullptr);
  if (!ws || wsb < a0.total) return fail(UOT_E_WORKSPACE, "workspace too small");
  if ((rc = begin(ctx))) return rc;
  const Layout L = layout(n);
  Act a = carve(n, batch, static_cast<char*>(ws));
  forward(n, L, a, x, batch, ctx->work);
  backward(n, L, a, t, batch, ctx->work);
  HIP_TRY(hipMemcpyAsync(grad, a.grad, 4 * L.total, hipMemcpyDeviceToDevice, ctx->work));
  HIP_TRY(hipGetLastError());
  const double l = loss_from_parts(a, batch * n->n_out, ctx->work, &rc);
  if (rc) return rc;
  if (loss) *loss = l;
  return finish(ctx);
}

int uot_warmstart_train_step(uot_ctx* ctx, uot_net* n, const float* x, const float* t, int64_t batch, float lr,
                             double* loss, void* ws, size_t wsb) {
  int rc = check_net(n);
  if (rc) return rc;
  if (!ctx || !x || !t || batch < 1 || !n->master || !n->wbf16 || !n->adam_m || !n->adam_v)
    return fail(UOT_E_INVALID, "bad arguments");
  const Act a0 = carve(n, batch, nullptr);
  if (!ws || wsb < a0.total) return fail(UOT_E_WORKSPACE, "workspace too small");
  if ((rc = begin(ctx))) return rc;
  const Layout L = layout(n);
  Act a = carve(n, batch, static_cast<char*>(ws));
  forward(n, L, a, x, batch, ctx->work);
  backward(n, L, a, t, batch, ctx->work);
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
  hipLaunchKernelGGL(k_adam, dim3(cdiv(L.total, kB)), dim3(kB), 0, ctx->work, n->master, a.grad, n->adam_m, n->adam_v,
                     n->wbf16, L.total, lr, b1, b2, 1e-8f, c1, c2);
  HIP_TRY(hipGetLastError());
  if (loss) {
    *loss = loss_from_parts(a, batch * n->n_out, ctx->work, &rc);
    if (rc) return rc;
  }
  return finish(ctx);
}

int uot_warmstart_features(uot_ctx* ctx, const float* p, const float* q, int64_t nb, int R, int r, float* x) {
  if (!ctx || !p || !q || !x || nb < 1 || r < 1 || R < r || R % r) return fail(UOT_E_INVALID, "bad arguments");
  int rc = begin(ctx);
  if (rc) return rc;
  const int64_t tot = nb * (int64_t)r * r * 2;
  hipLaunchKernelGGL(k_features, dim3(cdiv(tot, kB)), dim3(kB), 0, ctx->work, p, q, nb, R, r, x);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

int uot_grid_upsample(uot_ctx* ctx, const float* y, int64_t nb, int r, int R, float* out) {
  if (!ctx || !y || !out || nb < 1 || r < 1 || R < 1) return fail(UOT_E_INVALID, "bad arguments");
  int rc = begin(ctx);
  if (rc) return rc;
  const int64_t tot = nb * (int64_t)R * R;
  hipLaunchKernelGGL(k_upsample, dim3(cdiv(tot, kB)), dim3(kB), 0, ctx->work, y, nb, r, R, out);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

int uot_bary_estimate(uot_ctx* ctx, const float* p, int n, int64_t size, const double* alpha, double eps,
                      const uot_div* F2, float* h) {
  if (!ctx || !p || !alpha || !F2 || !h || n < 1 || n > kMaxBary || size < 1) return fail(UOT_E_INVALID, "bad arguments");
  if (F2->kind != UOT_DIV_KL && F2->kind != UOT_DIV_EQ) return fail(UOT_E_UNSUPPORTED, "F2 must be KL or equality");
  BaryW la{};
  double asum = 0.0;
  for (int k = 0; k < n; ++k) {
    if (!(alpha[k] > 0)) return fail(UOT_E_INVALID, "alpha_k must be > 0");
    la.v[k] = std::log(alpha[k]);
    la.a[k] = alpha[k];
    asum += alpha[k];
  }
  int rc = begin(ctx);
  if (rc) return rc;
  hipLaunchKernelGGL(k_bary_estimate, dim3(cdiv(size, kB)), dim3(kB), 0, ctx->work, p, n, size, la, std::log(asum),
                     (float)eps, (float)F2->lambda, F2->kind == UOT_DIV_KL ? 1 : 0, h);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

int uot_bary_local_v0(uot_ctx* ctx, const float* p, const float* h0, int n, int n1, int n2, double h1, double h2,
                      double lam, double eps, float* v0) {
  if (!ctx || !p || !h0 || !v0 || n < 1 || n1 < 1 || n2 < 1 || !(h1 > 0) || !(h2 > 0) || !(lam > 0) || !(eps > 0))
    return fail(UOT_E_INVALID, "bad arguments");
  int rc = begin(ctx);
  if (rc) return rc;
  const int64_t tot = (int64_t)n * n1 * n2;
  hipLaunchKernelGGL(k_bary_local_v0, dim3(cdiv(tot, kB)), dim3(kB), 0, ctx->work, p, h0, n, n1, n2, (float)h1,
                     (float)h2, (float)lam, (float)eps, v0);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

int uot_gemm_workspace_size(int M, int N, int K, size_t* bytes) {
  if (!bytes || M < 1 || N < 1 || K < 1) return fail(UOT_E_INVALID, "bad arguments");
  *bytes = 4 * (size_t)gemm_partials(M, N, K, true);
  return UOT_OK;
}

static int gemm_ws_check(const void* ws, size_t wsb, float*& part, int64_t& floats) {
  part = nullptr;
  floats = 0;
  if (!ws) return UOT_OK;
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(UOT_E_WORKSPACE, "workspace must be 256-byte aligned");
  part = static_cast<float*>(const_cast<void*>(ws));
  floats = (int64_t)(wsb / 4);
  return UOT_OK;
}

int uot_gemm_bf16(uot_ctx* ctx, int ta, int tb, int M, int N, int K, const uint16_t* A, int64_t lda, const uint16_t* B,
                  int64_t ldb, float* C, int64_t ldc, void* ws, size_t wsb) {
  if (!ctx || !A || !B || !C || M < 1 || N < 1 || K < 1) return fail(UOT_E_INVALID, "bad arguments");
  float* part;
  int64_t pf;
  int rc = gemm_ws_check(ws, wsb, part, pf);
  if (rc) return rc;
  if ((rc = begin(ctx))) return rc;
  hipStream_t s = ctx->work;
  if (!ta && !tb) gemm<false, false>(A, lda, B, ldb, M, N, K, C, ldc, nullptr, nullptr, 0, s, part, pf);
  else if (!ta && tb) gemm<false, true>(A, lda, B, ldb, M, N, K, C, ldc, nullptr, nullptr, 0, s, part, pf);
  else if (ta && !tb) gemm<true, false>(A, lda, B, ldb, M, N, K, C, ldc, nullptr, nullptr, 0, s, part, pf);
  else gemm<true, true>(A, lda, B, ldb, M, N, K, C, ldc, nullptr, nullptr, 0, s, part, pf);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

int uot_time_gemm_bf16(uot_ctx* ctx, int ta, int tb, int M, int N, int K, const uint16_t* A, int64_t lda,
                       const uint16_t* B, int64_t ldb, float* C, int64_t ldc, int reps, double* ms, void* ws,
                       size_t wsb) {
  if (!ctx || !A || !B || !C || !ms || M < 1 || N < 1 || K < 1 || reps < 1) return fail(UOT_E_INVALID, "bad arguments");
  float* part;
  int64_t pf;
  int rc = gemm_ws_check(ws, wsb, part, pf);
  if (rc) return rc;
  if ((rc = begin(ctx))) return rc;
  hipStream_t s = ctx->work;
  auto run = [&] {
    if (!ta && !tb) gemm<false, false>(A, lda, B, ldb, M, N, K, C, ldc, nullptr, nullptr, 0, s, part, pf);
    else if (!ta && tb) gemm<false, true>(A, lda, B, ldb, M, N, K, C, ldc, nullptr, nullptr, 0, s, part, pf);
    else if (ta && !tb) gemm<true, false>(A, lda, B, ldb, M, N, K, C, ldc, nullptr, nullptr, 0, s, part, pf);
    else gemm<true, true>(A, lda, B, ldb, M, N, K, C, ldc, nullptr, nullptr, 0, s, part, pf);
  };
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  run();
  HIP_TRY(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) run();
  HIP_TRY(hipEventRecord(e1, s));
  HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  *ms = double(t) / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

}  // extern "C"
