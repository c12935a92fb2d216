// HIP kernels of libuot for gfx950 (MI355X).
//
// One half-step of the scaling iteration (S) is
//   (1) a Gibbs product in the log domain, S = log K(b dy), and
//   (2) a pointwise proxdiv epilogue (Table proximalexplicit), plus on the X
//       side the partial sums of the marginal residual.
// (1) has two forms:
//   * regular grids: K is a tensor product of 1-D Gaussian kernels (Sec. 4.4,
//     separable kernel); every 1-D pass is a batched log-sum-exp
//     out[a][i][b] = LSE2_j(g[i-j] + in[a][j][b]), with g = -C1/eps in log2
//     units taken from a per-stage table;
//   * point clouds: dense log-sum-exp over all columns, C_ij = |x_i - y_j|^2
//     recomputed from coordinates staged in LDS (Sec. 4.4, "Computing the
//     matrix multiplications"); columns are split across blocks and the
//     per-split (max, sum) pairs merged by the epilogue kernel.
#include <algorithm>
#include <cstdlib>

#include "uot_device.h"
#include "uot_epilogue.h"
#include "uot_launch.h"

namespace uot {

constexpr int kChunk = 8;       // terms per online-max rescale
static inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
constexpr int kMaxLine = 4096;  // longest grid axis (LDS table of the contiguous pass)

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// ---------------------------------------------------------------------------
// input preparation: log densities (-inf at 0), log reference weights
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_log(const T* __restrict__ src, T* __restrict__ dst, int64_t n, int zero_is_ninf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = src[i];
  dst[i] = (s > T(0)) ? Num<T>::log(s) : (zero_is_ninf ? Num<T>::ninf() : Num<T>::log(s));
}

// pot = v0 (or 0), w = (pot/eps + logd) * log2(e); a potential of +inf (left by
// a vanishing product: that point's row of the plan is zero) gives w = -inf
template <typename T>
__global__ void k_init_pot(const T* __restrict__ v0, const T* __restrict__ logd, T* __restrict__ pot,
                           T* __restrict__ w, int64_t n, int64_t size, const Ctrl* __restrict__ c,
                           int which_eps) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T eps = T(c->eps[which_eps & 1]);
  T p = v0 ? v0[i] : T(0);
  if (pot) pot[i] = p;
  if (w) w[i] = (p == Num<T>::pinf()) ? Num<T>::ninf() : (p / eps + logd[i % size]) * T(kLog2e);
}

// g tables of one grid axis for every eps stage, tab[s][k] = log2 of the 1-D
// kernel at offset d = (k - (n-1)) h:  -d^2 / eps_s log2(e) (squared
// Euclidean cost), or (2 / eps_s) log2 cos((pi/2) |d| / cut) for |d| < cut and
// -inf beyond (WF cost, 1-D grids)
template <typename T>
__global__ void k_gtab(T* __restrict__ tab, int n, double h, const Ctrl* __restrict__ c, int nst, CostArgs cost) {
  const int len = 2 * n - 1;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)len * nst) return;
  const int s = (int)(t / len), k = (int)(t % len);
  const double d = double(k - (n - 1)) * h;
  if (cost.kind == 1) {
    const double ad = ::fabs(d);
    tab[t] = ad < cost.cut ? T(2.0 / c->eps_tab[s] * ::log2(::cos(0.5 * M_PI * ad / cost.cut)))
                           : Num<T>::ninf();
  } else {
    tab[t] = T(-(d * d) / c->eps_tab[s] * kLog2e);
  }
}

// merge the per-wave partial LSEs of a block (4 waves split the taps); the
// merged value for (output r, lane) is returned to wave 0
template <typename T, int RI>
__device__ __forceinline__ void merge_waves(Lse2<T> (&acc)[RI]) {
  __shared__ T smm[4][RI][64], sms[4][RI][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    smm[wv][r][lane] = acc[r].m;
    sms[wv][r][lane] = acc[r].s;
  }
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int r = 0; r < RI; ++r)
#pragma unroll
      for (int k = 1; k < 4; ++k) acc[r].merge(smm[k][r][lane], sms[k][r][lane]);
  }
}

// ---------------------------------------------------------------------------
// grid pass along a strided axis:  out[a][i][b] = LSE2_j ( g[i - j] + in[a][j][b] )
// lanes over 64 consecutive b, RI outputs i per lane (uniform, so g[i-j] is a
// scalar load), the 4 waves of a block take a quarter of the taps j each.
// grid = (ceil(B/64), ceil(n/RI), A)
// ---------------------------------------------------------------------------
template <typename T, int RI>
__global__ __launch_bounds__(kBlock) void k_grid_strided(const T* __restrict__ in, int n, int64_t B,
                                                          const T* __restrict__ gtab, int side,
                                                          const Ctrl* __restrict__ c, EpiArgs<T> ep) {
  if (skip_side(c, side)) return;
  // the stage's table in LDS: the lookups g[i - j] are wave-uniform broadcasts
  extern __shared__ __align__(16) unsigned char gl_raw[];
  T* gl = reinterpret_cast<T*>(gl_raw);
  const int stage = stage_of(c, side);
  const T* __restrict__ gsrc = gtab + (int64_t)stage * (2 * n - 1);
  for (int k = threadIdx.x; k < 2 * n - 1; k += kBlock) gl[k] = gsrc[k];
  __syncthreads();
  const T* g = gl + (n - 1);    // g[d] for d in [-(n-1), n-1]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 64 + lane;
  const bool valid_b = b < B;
  const int64_t a = blockIdx.z;
  const int i0 = blockIdx.y * RI;
  int ii[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) ii[r] = (i0 + r < n) ? i0 + r : n - 1;
  const T* __restrict__ col = in + (a * n) * B + (valid_b ? b : 0);
  const int jq = (n + 3) >> 2;
  const int j0 = wv * jq;
  const int j1 = (j0 + jq < n) ? j0 + jq : n;
  Lse2<T> acc[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) acc[r].init();
  int j = j0;
  for (; j + kChunk <= j1; j += kChunk) {
    T w[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) w[k] = col[(int64_t)(j + k) * B];
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      T t[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) t[k] = g[ii[r] - (j + k)] + w[k];
      acc[r].template add<kChunk>(t);
    }
  }
  if (j < j1) {
    // tail: indices clamped into [j, j1), surplus terms replaced by -inf
    T w[kChunk];
    int jc[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      jc[k] = (j + k < j1) ? j + k : j1 - 1;
      w[k] = col[(int64_t)jc[k] * B];
    }
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      T t[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) {
        const T tk = g[ii[r] - jc[k]] + w[k];
        t[k] = (j + k < j1) ? tk : Num<T>::ninf();
      }
      acc[r].template add<kChunk>(t);
    }
  }
  merge_waves<T, RI>(acc);
  ResAcc<T> ra;
  ra.init();
  if (wv == 0 && valid_b) {
#pragma unroll
    for (int r = 0; r < RI; ++r)
      if (i0 + r < n) epi_elem<T>((a * n + i0 + r) * B + b, acc[r].result(), c, side, ep, ra);
  }
  epi_finish<T>(ep, ra, (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
}

// ---------------------------------------------------------------------------
// grid pass along the contiguous axis:  out[a][i] = LSE2_j ( g[i - j] + in[a][j] )
// lanes over 64 consecutive outputs i (RI groups of 64 per block), the line a
// uniform, so in[a][j] is a scalar load and g[i-j] comes from an LDS copy of
// the stage's table; the 4 waves split the taps j.
// grid = (ceil(n / (64 RI)), A_lo, A_hi) with a = blockIdx.z * gridDim.y + blockIdx.y
// ---------------------------------------------------------------------------
// taps j with |i - j| >= band are exact zeros of the kernel (a cut locus; band
// = n otherwise) and are skipped: a block reads only the taps within band of
// its outputs, and only the part of the g table they need.
// SPLIT: few long lines (1-D grids): blockIdx.z takes one of nsplit slices of
// the tap range and the block writes its partial LSE (m, s) per output to
// pm / ps[(z A + a) n + i]; k_dense_epi merges the slices and runs the
// epilogue.  grid = (ceil(n / 64 RI), A, nsplit) then, else (.., lines in y, z).
template <typename T, int RI, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_grid_contig(const T* __restrict__ in, int n, int64_t A,
                                                         const T* __restrict__ gtab, int side,
                                                         const Ctrl* __restrict__ c, EpiArgs<T> ep, int band,
                                                         T* __restrict__ pm, T* __restrict__ ps, int nsplit) {
  // block 0 of a launch that hosts the control step: partials loaded first
  const bool hosting = !SPLIT && ep.host_ctl != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0;
  const int par = par_of(side);
  CtrlSnap hsnap{};
  float hm = -__builtin_inff(), hden = 0.f, hnum = 0.f, hdu = 0.f;
  if (hosting) {
    hsnap = ctrl_snap(ep.host_ctl, par);
    ctl_load(ep.host_parts, ep.host_nparts, hm, hden, hnum, hdu);
  }
  if (skip_side(c, side)) {
    if (hosting && threadIdx.x == 0) control_skip(ep.host_ctl, par);
    return;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t a = SPLIT ? (int64_t)blockIdx.y : (int64_t)blockIdx.z * gridDim.y + blockIdx.y;
  const bool valid_a = a < A;
  const T* __restrict__ line = in + (valid_a ? a : 0) * (int64_t)n;
  // outputs [o0, o1) of the block, taps [ta, tb) within the band (one slice
  // of it when SPLIT)
  const int o0 = blockIdx.x * RI * 64;
  const int o1 = (o0 + RI * 64 < n) ? o0 + RI * 64 : n;
  int ta = (o0 - band + 1 > 0) ? o0 - band + 1 : 0;
  int tb = (o1 - 1 + band < n) ? o1 - 1 + band : n;
  if (SPLIT) {
    const int sl = (tb - ta + nsplit - 1) / nsplit;
    const int s0 = ta + (int)blockIdx.z * sl;
    ta = s0 < tb ? s0 : tb;
    tb = (s0 + sl < tb) ? s0 + sl : tb;
  }
  // the g entries the block reads: offsets i - j in [o0 - tb + 1, o1 - 1 - ta]
  extern __shared__ __align__(16) unsigned char gl_raw[];
  T* gl = reinterpret_cast<T*>(gl_raw);
  const int stage = stage_of(c, side);
  const T* __restrict__ g = gtab + (int64_t)stage * (2 * n - 1);
  const int wlo = o0 - tb + 1 + (n - 1);
  const int wlen = (tb > ta) ? (o1 - o0) + (tb - ta) - 1 : 0;
  for (int k = threadIdx.x; k < wlen; k += kBlock) gl[k] = g[wlo + k];
  __syncthreads();
  int ii[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    const int i = (blockIdx.x * RI + r) * 64 + lane;
    ii[r] = (i < n ? i : o1 - 1) + (n - 1) - wlo;   // window index of g[i - 0]
  }
  const int jq = (tb - ta + 3) >> 2;
  const int j0 = ta + wv * jq;
  const int j1 = (j0 + jq < tb) ? j0 + jq : tb;
  Lse2<T> acc[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) acc[r].init();
  int j = j0;
  for (; j + kChunk <= j1; j += kChunk) {
    T w[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) w[k] = line[j + k];
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      T t[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) t[k] = gl[ii[r] - (j + k)] + w[k];
      acc[r].template add<kChunk>(t);
    }
  }
  if (j < j1) {
    // tail: indices clamped into [j, j1), surplus terms replaced by -inf
    int jc[kChunk];
    T w[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; ++k) {
      jc[k] = (j + k < j1) ? j + k : j1 - 1;
      w[k] = line[jc[k]];
    }
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      T t[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) {
        const T tk = gl[ii[r] - jc[k]] + w[k];
        t[k] = (j + k < j1) ? tk : Num<T>::ninf();
      }
      acc[r].template add<kChunk>(t);
    }
  }
  merge_waves<T, RI>(acc);
  if (SPLIT) {
    if (wv == 0 && valid_a) {
#pragma unroll
      for (int r = 0; r < RI; ++r) {
        const int i = (blockIdx.x * RI + r) * 64 + lane;
        if (i < n) {
          const int64_t e = ((int64_t)blockIdx.z * A + a) * n + i;
          pm[e] = acc[r].m;
          ps[e] = acc[r].s;
        }
      }
    }
    return;
  }
  ResAcc<T> ra;
  ra.init();
  if (wv == 0 && valid_a) {
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int i = (blockIdx.x * RI + r) * 64 + lane;
      if (i < n) epi_elem<T>(a * n + i, acc[r].result(), c, side, ep, ra);
    }
  }
  epi_finish<T>(ep, ra, (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
  if (hosting) ctl_reduce_finish(ep.host_ctl, hsnap, hm, hden, hnum, hdu, ep.host_hist, par);
}

// ---------------------------------------------------------------------------
// dense point-cloud product: partial LSE over one column split.
//   part[split][i] = (m, s) with  m + log2 s = LSE2_{j in split}( w_j + log2 K_ij )
// rows: xr (DIM x Nr), columns: yc (DIM x Mc) and w (Mc, log2 units).
// COST 0: log2 K = -|x_i - y_j|^2 log2(e) / eps.
// COST 1: the WF cost with cut locus, log2 K = (2/eps) log2 cos((pi/2) d / cut)
//         for d < cut and -inf beyond (wf_log2k).  K then has exact zeros:
//         each wave holds 64 R consecutive rows (R = 1 for this cost) and
//         bounds them by a box, every 256-column chunk is bounded by 16 boxes
//         of 16 columns, and a
//         wave skips the column groups whose box lies at distance >= cut from
//         its rows' box (every entry there is zero).  This pays when the
//         points are stored in a spatially coherent order.
// grid = (ceil(Nr / (256 R)), splits)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T lanes_min(T v, int from) {
#pragma unroll
  for (int o = from; o >= 1; o >>= 1) v = Num<T>::fmin(v, __shfl_xor(v, o));
  return v;
}
template <typename T>
__device__ __forceinline__ T lanes_max(T v, int from) {
#pragma unroll
  for (int o = from; o >= 1; o >>= 1) v = Num<T>::fmax(v, __shfl_xor(v, o));
  return v;
}

template <typename T, int DIM, int R, int COST>
__global__ __launch_bounds__(kBlock) void k_dense_lse(const T* __restrict__ xr, int64_t Nr,
                                                       const T* __restrict__ yc, const T* __restrict__ w,
                                                       int64_t Mc, int64_t cols_per_split,
                                                       T* __restrict__ pm, T* __restrict__ ps, int side,
                                                       const Ctrl* __restrict__ c, T a2, T cut2) {
  if (skip_side(c, side)) return;
  using V4 = typename Vec4<T>::type;
  __shared__ V4 tile[kBlock];
  const T sc = T(kLog2e / eps_of(c, side));
  const T ewf = T(2.0 / eps_of(c, side));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  T xi[R][DIM];
  int64_t rows[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    // WF: the rows of a wave are consecutive, so its box is tight
    rows[r] = (int64_t)blockIdx.x * (kBlock * R) +
              (COST == 1 ? wv * (64 * R) + r * 64 + lane : r * kBlock + threadIdx.x);
    const int64_t rr = rows[r] < Nr ? rows[r] : 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[r][d] = xr[d * Nr + rr];
  }
  Lse2<T> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r].init();
  const int64_t cb = (int64_t)blockIdx.y * cols_per_split;
  const int64_t ce = (cb + cols_per_split < Mc) ? cb + cols_per_split : Mc;
  if constexpr (COST == 0) {
    for (int64_t c0 = cb; c0 < ce; c0 += kBlock) {
      const int64_t cc = c0 + threadIdx.x;
      V4 rec;
      rec.x = rec.y = rec.z = T(0);
      if (cc < ce) {
        rec.x = yc[cc];
        if (DIM > 1) rec.y = yc[Mc + cc];
        if (DIM > 2) rec.z = yc[2 * Mc + cc];
        rec.w = w[cc];
      } else {
        rec.w = Num<T>::ninf();
      }
      __syncthreads();
      tile[threadIdx.x] = rec;
      __syncthreads();
      const int64_t rem = ce - c0;
      const int cnt = rem < kBlock ? (int)rem : kBlock;
      for (int jj = 0; jj < cnt; jj += kChunk) {
        V4 q[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) q[k] = tile[jj + k];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          T t[kChunk];
#pragma unroll
          for (int k = 0; k < kChunk; ++k) {
            T d0 = xi[r][0] - q[k].x;
            T cst = d0 * d0;
            if (DIM > 1) { T d1 = xi[r][1] - q[k].y; cst = Num<T>::fma(d1, d1, cst); }
            if (DIM > 2) { T d2 = xi[r][2] - q[k].z; cst = Num<T>::fma(d2, d2, cst); }
            t[k] = Num<T>::fma(-sc, cst, q[k].w);
          }
          acc[r].template add<kChunk>(t);
        }
      }
    }
  } else {
    __shared__ T gbx[16][6];  // boxes of the 16 groups of 16 columns of a chunk
    T rlo[3], rhi[3];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      T lo = Num<T>::pinf(), hi = Num<T>::ninf();
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (rows[r] < Nr) {
          lo = Num<T>::fmin(lo, xi[r][d]);
          hi = Num<T>::fmax(hi, xi[r][d]);
        }
      rlo[d] = lanes_min<T>(lo, 32);
      rhi[d] = lanes_max<T>(hi, 32);
    }
    for (int64_t c0 = cb; c0 < ce; c0 += kBlock) {
      const int64_t cc = c0 + threadIdx.x;
      V4 rec;
      rec.x = rec.y = rec.z = T(0);
      if (cc < ce) {
        rec.x = yc[cc];
        if (DIM > 1) rec.y = yc[Mc + cc];
        if (DIM > 2) rec.z = yc[2 * Mc + cc];
        rec.w = w[cc];
      } else {
        rec.w = Num<T>::ninf();
      }
      __syncthreads();
      tile[threadIdx.x] = rec;
      // box of each group of 16 columns, over the columns that carry mass
      const bool live = rec.w != Num<T>::ninf();
      const T cx[3] = {rec.x, rec.y, rec.z};
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const T lo = lanes_min<T>(live ? cx[d] : Num<T>::pinf(), 8);
        const T hi = lanes_max<T>(live ? cx[d] : Num<T>::ninf(), 8);
        if ((lane & 15) == 0) {
          gbx[wv * 4 + (lane >> 4)][2 * d] = lo;
          gbx[wv * 4 + (lane >> 4)][2 * d + 1] = hi;
        }
      }
      __syncthreads();
      const int64_t rem = ce - c0;
      const int cnt = rem < kBlock ? (int)rem : kBlock;
      for (int gi = 0; gi < 16 && gi * 16 < cnt; ++gi) {
        T gap2 = T(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const T g = Num<T>::fmax(Num<T>::fmax(gbx[gi][2 * d] - rhi[d], rlo[d] - gbx[gi][2 * d + 1]), T(0));
          gap2 = Num<T>::fma(g, g, gap2);
        }
        // every entry of the group is beyond the cut (an empty box gives +inf)
        if (!(gap2 < cut2)) continue;
        const int je = (gi * 16 + 16 < cnt) ? gi * 16 + 16 : cnt;
        for (int jj = gi * 16; jj < je; jj += kChunk) {
          V4 q[kChunk];
#pragma unroll
          for (int k = 0; k < kChunk; ++k) q[k] = tile[jj + k];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            T t[kChunk];
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
              T d0 = xi[r][0] - q[k].x;
              T cst = d0 * d0;
              if (DIM > 1) { T d1 = xi[r][1] - q[k].y; cst = Num<T>::fma(d1, d1, cst); }
              if (DIM > 2) { T d2 = xi[r][2] - q[k].z; cst = Num<T>::fma(d2, d2, cst); }
              t[k] = q[k].w + wf_log2k<T>(cst, a2, cut2, ewf);
            }
            acc[r].template add<kChunk>(t);
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (rows[r] < Nr) {
      pm[blockIdx.y * Nr + rows[r]] = acc[r].m;
      ps[blockIdx.y * Nr + rows[r]] = acc[r].s;
    }
  }
}

// ---------------------------------------------------------------------------
// dense point-cloud product, tile-factored (FP32, squared Euclidean cost).
// Row tile I = the 64 R consecutive rows of a wave (centre xbar_I, radius
// r_I), column tile J = 16 consecutive columns of a staged chunk (ybar_J, r_J),
// e_i = x_i - xbar_I, f_j = y_j - ybar_J.  With c = log2(e) / eps,
//   w_j - c |x_i - y_j|^2 = beta_jI + alpha_iJ + 2 c e_i . f_j,
//   beta_jI  = w_j - c |y_j - xbar_I|^2,
//   alpha_iJ = -c |x_i - ybar_J|^2 + c |xbar_I - ybar_J|^2
// (exact), so the tile's share of row i is
//   2^{alpha_iJ + m_IJ} sum_j 2^{2c e_i.f_j + l_jI},  l_jI = beta_jI - m_IJ <= 0,
// m_IJ = max_j beta_jI: per pair DIM FMAs (the chain starts at l_jI), one exp2
// and one add, and no running maximum.  The exponent is summed before the
// exp2: 2^{l_jI} alone can fall below the FP32 normal range while the product
// with 2^{2c e.f} still matters.  The tile's largest term is at least 2^{-B},
// B = 2c r_I r_J, so terms that underflow are negligible.  Tile pairs where B
// exceeds kDenseTfBound (wide tiles: points not in a spatially coherent order)
// are summed directly instead, so the result never depends on the order.
// grid = (ceil(Nr / (256 R)), splits); partials as in k_dense_lse.
// ---------------------------------------------------------------------------
constexpr float kDenseTfBound = 64.f;

template <int DIM, int R>
__global__ __launch_bounds__(kBlock) void k_dense_tf(const float* __restrict__ xr, int64_t Nr,
                                                      const float* __restrict__ yc, const float* __restrict__ w,
                                                      int64_t Mc, int64_t cols_per_split,
                                                      float* __restrict__ pm, float* __restrict__ ps, int side,
                                                      const Ctrl* __restrict__ c) {
  if (skip_side(c, side)) return;
  __shared__ float4 tile[kBlock];        // (y, w) of the chunk, for directly summed tile pairs
  __shared__ float4 fe[4][kBlock];       // (f_j, l_jI) for the row tile I of each wave
  __shared__ float toff[4][16];          // m_IJ + c |xbar_I - ybar_J|^2  (-inf: no mass in J)
  __shared__ int tfac[4][16];            // tile pair factored (1) or summed directly (0)
  __shared__ float tyb[16][3];           // ybar_J
  __shared__ float xbs[4][3], xrs[4];    // xbar_I and r_I^2 of the 4 waves
  const float cc = float(kLog2e / eps_of(c, side));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float xi[R][3];
  int64_t rows[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    rows[r] = (int64_t)blockIdx.x * (kBlock * R) + wv * (64 * R) + r * 64 + lane;
    const int64_t rr = rows[r] < Nr ? rows[r] : 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) xi[r][d] = d < DIM ? xr[d * Nr + rr] : 0.f;
  }
  // the wave's row tile: box centre and radius over its valid rows
  float xb[3], e2[R][3];
  float rad2 = 0.f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float lo = __builtin_inff(), hi = -__builtin_inff();
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (d < DIM && rows[r] < Nr) {
        lo = fminf(lo, xi[r][d]);
        hi = fmaxf(hi, xi[r][d]);
      }
    lo = lanes_min<float>(lo, 32);
    hi = lanes_max<float>(hi, 32);
    xb[d] = lo <= hi ? 0.5f * (lo + hi) : 0.f;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    float q = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float e = xi[r][d] - xb[d];
      e2[r][d] = 2.f * cc * e;
      q = __builtin_fmaf(e, e, q);
    }
    if (rows[r] < Nr) rad2 = fmaxf(rad2, q);
  }
  rad2 = lanes_max<float>(rad2, 32);
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) xbs[wv][d] = xb[d];
    xrs[wv] = rad2;
  }
  __syncthreads();
  Lse2<float> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r].init();
  const int64_t cb = (int64_t)blockIdx.y * cols_per_split;
  const int64_t ce = (cb + cols_per_split < Mc) ? cb + cols_per_split : Mc;
  const int J = threadIdx.x >> 4;        // this thread's column tile within the chunk
  for (int64_t c0 = cb; c0 < ce; c0 += kBlock) {
    const int64_t col = c0 + threadIdx.x;
    float4 rec;
    rec.x = rec.y = rec.z = 0.f;
    if (col < ce) {
      rec.x = yc[col];
      if (DIM > 1) rec.y = yc[Mc + col];
      if (DIM > 2) rec.z = yc[2 * Mc + col];
      rec.w = w[col];
    } else {
      rec.w = -__builtin_inff();
    }
    __syncthreads();                     // the previous chunk's reads are done
    tile[threadIdx.x] = rec;
    // column tile: box centre and radius over its columns that carry mass
    const bool live = rec.w != -__builtin_inff();
    const float y[3] = {rec.x, rec.y, rec.z};
    float yb[3], f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float lo = lanes_min<float>(live && d < DIM ? y[d] : __builtin_inff(), 8);
      const float hi = lanes_max<float>(live && d < DIM ? y[d] : -__builtin_inff(), 8);
      yb[d] = lo <= hi ? 0.5f * (lo + hi) : 0.f;
      // columns without mass (padding, zero density) lie outside the box: f = 0
      // keeps 2c e.f bounded there, and their l is -inf
      f[d] = live ? y[d] - yb[d] : 0.f;
    }
    const float fr2 = lanes_max<float>(live ? __builtin_fmaf(f[0], f[0], __builtin_fmaf(f[1], f[1], f[2] * f[2])) : 0.f, 8);
    if ((threadIdx.x & 15) == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) tyb[J][d] = yb[d];
    }
#pragma unroll
    for (int I = 0; I < 4; ++I) {
      float dy2 = 0.f, dxy2 = 0.f;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float a = y[d] - xbs[I][d], b = xbs[I][d] - yb[d];
        dy2 = __builtin_fmaf(a, a, dy2);
        dxy2 = __builtin_fmaf(b, b, dxy2);
      }
      const float beta = live ? __builtin_fmaf(-cc, dy2, rec.w) : -__builtin_inff();
      const float m = lanes_max<float>(beta, 8);
      fe[I][threadIdx.x] = make_float4(f[0], f[1], f[2], beta - m);   // -inf for columns without mass
      if ((threadIdx.x & 15) == 0) {
        toff[I][J] = m == -__builtin_inff() ? m : __builtin_fmaf(cc, dxy2, m);
        tfac[I][J] = 2.f * cc * __builtin_sqrtf(xrs[I] * fr2) <= kDenseTfBound;
      }
    }
    __syncthreads();
    const int64_t rem = ce - c0;
    const int cnt = rem < kBlock ? (int)rem : kBlock;
    const int ntl = (cnt + 15) >> 4;
    // tile metadata for this wave's row tile in lanes 0..15, read per tile
    // into scalars (no LDS round trip inside the tile loop)
    const int li = lane & 15;
    const float moff = toff[wv][li];
    const int mfac = tfac[wv][li];
    const float myb0 = tyb[li][0], myb1 = tyb[li][1], myb2 = tyb[li][2];
    for (int jt = 0; jt < ntl; ++jt) {
      const float off = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(moff), jt));
      if (off == -__builtin_inff()) continue;     // no mass in this column tile
      if (__builtin_amdgcn_readlane(mfac, jt)) {
        // each staged column feeds the R rows of the thread
        float sm[R];
#pragma unroll
        for (int r = 0; r < R; ++r) sm[r] = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const float4 q = fe[wv][jt * 16 + k];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            float t = __builtin_fmaf(e2[r][0], q.x, q.w);
            if (DIM > 1) t = __builtin_fmaf(e2[r][1], q.y, t);
            if (DIM > 2) t = __builtin_fmaf(e2[r][2], q.z, t);
            sm[r] += __builtin_amdgcn_exp2f(t);
          }
        }
        const float ybj[3] = {__int_as_float(__builtin_amdgcn_readlane(__float_as_int(myb0), jt)),
                              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(myb1), jt)),
                              __int_as_float(__builtin_amdgcn_readlane(__float_as_int(myb2), jt))};
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float a = off;
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            const float dd = xi[r][d] - ybj[d];
            a = __builtin_fmaf(-cc * dd, dd, a);
          }
          // branch-free merge of (a, sm[r]) into the running (m, s)
          const float mn = fmaxf(acc[r].m, a);
          const float sh = mn == -__builtin_inff() ? 0.f : mn;
          acc[r].s = acc[r].s * __builtin_amdgcn_exp2f(acc[r].m - sh) + sm[r] * __builtin_amdgcn_exp2f(a - sh);
          acc[r].m = mn;
        }
      } else {
        const float sc = cc;
        for (int jj = jt * 16; jj < jt * 16 + 16; jj += kChunk) {
          float4 q[kChunk];
#pragma unroll
          for (int k = 0; k < kChunk; ++k) q[k] = tile[jj + k];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            float t[kChunk];
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
              float d0 = xi[r][0] - q[k].x;
              float cst = d0 * d0;
              if (DIM > 1) { float d1 = xi[r][1] - q[k].y; cst = __builtin_fmaf(d1, d1, cst); }
              if (DIM > 2) { float d2 = xi[r][2] - q[k].z; cst = __builtin_fmaf(d2, d2, cst); }
              t[k] = __builtin_fmaf(-sc, cst, q[k].w);
            }
            acc[r].template add<kChunk>(t);
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (rows[r] < Nr) {
      pm[blockIdx.y * Nr + rows[r]] = acc[r].m;
      ps[blockIdx.y * Nr + rows[r]] = acc[r].s;
    }
  }
}

// ---------------------------------------------------------------------------
// spatial order of a point cloud (Z-order / Morton), for the tile-factored
// dense product: box, codes, then the permutation by counting ranks
// ---------------------------------------------------------------------------
// bx[d] = min, bx[3 + d] = max of coordinate d (one block)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_point_box(const T* __restrict__ x, int64_t n, int dim, T* __restrict__ bx) {
  __shared__ T smin[kBlock], smax[kBlock];
  for (int d = 0; d < dim; ++d) {
    T lo = Num<T>::pinf(), hi = Num<T>::ninf();
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      const T v = x[d * n + i];
      lo = Num<T>::fmin(lo, v);
      hi = Num<T>::fmax(hi, v);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int o = kBlock / 2; o >= 1; o >>= 1) {
      if ((int)threadIdx.x < o) {
        smin[threadIdx.x] = Num<T>::fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
        smax[threadIdx.x] = Num<T>::fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      bx[d] = smin[0];
      bx[3 + d] = smax[0];
    }
    __syncthreads();
  }
}

// Morton code: coordinates quantised over the box to 2^bits levels
// (bits = 30 / dim), their bits interleaved; xp: the point's first
// coordinate, stride: between coordinates
template <typename T>
__device__ __forceinline__ uint32_t morton_code(const T* __restrict__ xp, int64_t stride, int dim,
                                                const T* __restrict__ bx) {
  const int bits = 30 / dim;
  const uint32_t top = (1u << bits) - 1u;
  uint32_t out = 0;
  for (int d = 0; d < dim; ++d) {
    const double lo = double(bx[d]), ext = double(bx[3 + d]) - lo;
    double t = ext > 0 ? (double(xp[d * stride]) - lo) / ext : 0.0;
    uint32_t q = (uint32_t)(t * double(top) + 0.5);
    q = q > top ? top : q;
    for (int b = 0; b < bits; ++b) out |= ((q >> b) & 1u) << (b * dim + d);
  }
  return out;
}
template <typename T>
__global__ void k_morton(const T* __restrict__ x, int64_t n, int dim, const T* __restrict__ bx,
                         uint32_t* __restrict__ code) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  code[i] = morton_code<T>(x + i, n, dim, bx);
}

// perm[rank_i] = i with rank_i = #{j : code_j < code_i, or code_j = code_i and j < i}
// (a stable order; O(n^2) comparisons, once per solve, through LDS tiles)
__global__ __launch_bounds__(kBlock) void k_rank(const uint32_t* __restrict__ code, int64_t n,
                                                  int32_t* __restrict__ perm) {
  __shared__ uint32_t sc[kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint32_t ci = i < n ? code[i] : 0u;
  int64_t rank = 0;
  for (int64_t j0 = 0; j0 < n; j0 += kBlock) {
    __syncthreads();
    sc[threadIdx.x] = (j0 + threadIdx.x < n) ? code[j0 + threadIdx.x] : 0xffffffffu;
    __syncthreads();
    const int cnt = (n - j0 < kBlock) ? (int)(n - j0) : kBlock;
    for (int k = 0; k < cnt; ++k) {
      const uint32_t cj = sc[k];
      rank += (cj < ci || (cj == ci && j0 + k < i)) ? 1 : 0;
    }
  }
  if (i < n) perm[rank] = (int32_t)i;
}

// out[r][k] = in[r][perm[k]] for rows r < nrow of length n
template <typename T>
__global__ void k_gather(const T* __restrict__ in, const int32_t* __restrict__ perm, int64_t n, int nrow,
                         T* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t src = perm[k];
  for (int r = 0; r < nrow; ++r) out[r * n + k] = in[r * n + src];
}

// out[perm[k]] = in[k]
template <typename T>
__global__ void k_scatter(const T* __restrict__ in, const int32_t* __restrict__ perm, int64_t n, T* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  out[perm[k]] = in[k];
}

// The same per problem of a batch: problem b holds the points off[b] ..
// off[b + 1] - 1 of x (coordinate stride tot); its box goes to bx[6 b ..],
// and perm maps within the problem's range (perm[off[b] + rank] = off[b] + i).
// grid: blockIdx.x = problem (box: one block each; codes and ranks: blocks
// (b, t) step over the problem's tiles of 256 points by gridDim.y)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_point_box_batch(const T* __restrict__ x, int64_t tot,
                                                             const int64_t* __restrict__ off, int dim,
                                                             T* __restrict__ bx) {
  __shared__ T smin[kBlock], smax[kBlock];
  const int64_t o = off[blockIdx.x], n = off[blockIdx.x + 1] - o;
  for (int d = 0; d < dim; ++d) {
    T lo = Num<T>::pinf(), hi = Num<T>::ninf();
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      const T v = x[d * tot + o + i];
      lo = Num<T>::fmin(lo, v);
      hi = Num<T>::fmax(hi, v);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int h = kBlock / 2; h >= 1; h >>= 1) {
      if ((int)threadIdx.x < h) {
        smin[threadIdx.x] = Num<T>::fmin(smin[threadIdx.x], smin[threadIdx.x + h]);
        smax[threadIdx.x] = Num<T>::fmax(smax[threadIdx.x], smax[threadIdx.x + h]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      bx[6 * blockIdx.x + d] = smin[0];
      bx[6 * blockIdx.x + 3 + d] = smax[0];
    }
    __syncthreads();
  }
}
template <typename T>
__global__ void k_morton_batch(const T* __restrict__ x, int64_t tot, const int64_t* __restrict__ off, int dim,
                               const T* __restrict__ bx, uint32_t* __restrict__ code) {
  const int64_t o = off[blockIdx.x], n = off[blockIdx.x + 1] - o;
  for (int64_t i = (int64_t)blockIdx.y * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.y * kBlock)
    code[o + i] = morton_code<T>(x + o + i, tot, dim, bx + 6 * blockIdx.x);
}
__global__ __launch_bounds__(kBlock) void k_rank_batch(const uint32_t* __restrict__ code,
                                                        const int64_t* __restrict__ off, int32_t* __restrict__ perm) {
  __shared__ uint32_t sc[kBlock];
  const int64_t o = off[blockIdx.x], n = off[blockIdx.x + 1] - o;
  for (int64_t t0 = (int64_t)blockIdx.y * kBlock; t0 < n; t0 += (int64_t)gridDim.y * kBlock) {
    const int64_t i = t0 + threadIdx.x;
    const uint32_t ci = i < n ? code[o + i] : 0u;
    int64_t rank = 0;
    for (int64_t j0 = 0; j0 < n; j0 += kBlock) {
      __syncthreads();
      sc[threadIdx.x] = (j0 + threadIdx.x < n) ? code[o + j0 + threadIdx.x] : 0xffffffffu;
      __syncthreads();
      const int cnt = (n - j0 < kBlock) ? (int)(n - j0) : kBlock;
      for (int k = 0; k < cnt; ++k) {
        const uint32_t cj = sc[k];
        rank += (cj < ci || (cj == ci && j0 + k < i)) ? 1 : 0;
      }
    }
    if (i < n) perm[o + rank] = (int32_t)(o + i);
  }
}

// the same permutation for problems of at most kSortLds points: a bitonic
// sort of (code, index) pairs in LDS, one block per problem (the index
// breaks ties, so the order is the stable one of k_rank_batch)
constexpr int kSortLds = 4096;
__global__ __launch_bounds__(kBlock) void k_sort_batch(const uint32_t* __restrict__ code,
                                                        const int64_t* __restrict__ off, int32_t* __restrict__ perm) {
  __shared__ uint32_t sk[kSortLds];
  __shared__ int32_t si[kSortLds];
  const int64_t o = off[blockIdx.x];
  const int n = (int)(off[blockIdx.x + 1] - o);
  int P = 1;
  while (P < n) P <<= 1;
  for (int i = threadIdx.x; i < P; i += kBlock) {
    sk[i] = i < n ? code[o + i] : 0xffffffffu;
    si[i] = i;   // padding sorts last: largest code, then largest index
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += kBlock) {
        // pair (a, b = a + j) of the j-step: a has bit j clear
        const int a = ((t / j) * 2 * j) + (t % j), b = a + j;
        const bool up = (a & k) == 0;
        const uint32_t ka = sk[a], kb = sk[b];
        const int32_t ia = si[a], ib = si[b];
        const bool gt = ka > kb || (ka == kb && ia > ib);
        if (gt == up) {
          sk[a] = kb;
          sk[b] = ka;
          si[a] = ib;
          si[b] = ia;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += kBlock) perm[o + i] = (int32_t)(o + si[i]);
}

template <typename T>
void launch_spatial_order_batch(const T* x, int64_t tot, const int64_t* off, int64_t B, int64_t nmax, int dim,
                                T* box, uint32_t* code, int32_t* perm, hipStream_t s) {
  const unsigned ty = (unsigned)std::min<int64_t>(ceil_div(nmax, kBlock), 1024);
  hipLaunchKernelGGL(k_point_box_batch<T>, dim3((unsigned)B), dim3(kBlock), 0, s, x, tot, off, dim, box);
  hipLaunchKernelGGL(k_morton_batch<T>, dim3((unsigned)B, ty), dim3(kBlock), 0, s, x, tot, off, dim, box, code);
  if (nmax <= kSortLds)
    hipLaunchKernelGGL(k_sort_batch, dim3((unsigned)B), dim3(kBlock), 0, s, code, off, perm);
  else
    hipLaunchKernelGGL(k_rank_batch, dim3((unsigned)B, ty), dim3(kBlock), 0, s, code, off, perm);
}
template void launch_spatial_order_batch<float>(const float*, int64_t, const int64_t*, int64_t, int64_t, int, float*,
                                                uint32_t*, int32_t*, hipStream_t);

template <typename T>
void launch_spatial_order(const T* x, int64_t n, int dim, T* box, uint32_t* code, int32_t* perm, hipStream_t s) {
  hipLaunchKernelGGL(k_point_box<T>, dim3(1), dim3(kBlock), 0, s, x, n, dim, box);
  hipLaunchKernelGGL(k_morton<T>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, x, n, dim, box, code);
  hipLaunchKernelGGL(k_rank, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, code, n, perm);
}
template <typename T>
void launch_gather(const T* in, const int32_t* perm, int64_t n, int nrow, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather<T>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, in, perm, n, nrow, out);
}
template <typename T>
void launch_scatter(const T* in, const int32_t* perm, int64_t n, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter<T>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, in, perm, n, out);
}
template void launch_spatial_order<float>(const float*, int64_t, int, float*, uint32_t*, int32_t*, hipStream_t);
template void launch_spatial_order<double>(const double*, int64_t, int, double*, uint32_t*, int32_t*, hipStream_t);
template void launch_gather<float>(const float*, const int32_t*, int64_t, int, float*, hipStream_t);
template void launch_gather<double>(const double*, const int32_t*, int64_t, int, double*, hipStream_t);
template void launch_scatter<float>(const float*, const int32_t*, int64_t, float*, hipStream_t);
template void launch_scatter<double>(const double*, const int32_t*, int64_t, double*, hipStream_t);

void launch_dense_tf(int dim, const float* xr, int64_t Nr, const float* yc, const float* w, int64_t Mc, int nsplit,
                     int64_t cps, float* pm, float* ps, int side, const Ctrl* c, hipStream_t s) {
  dim3 grid(ceil_div(Nr, kBlock * 2), (unsigned)nsplit);
  if (dim == 1) hipLaunchKernelGGL((k_dense_tf<1, 2>), grid, dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, cps, pm, ps, side, c);
  else if (dim == 2)
    hipLaunchKernelGGL((k_dense_tf<2, 2>), grid, dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, cps, pm, ps, side, c);
  else hipLaunchKernelGGL((k_dense_tf<3, 2>), grid, dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, cps, pm, ps, side, c);
}

// log2 of the sum of n partials (m, s) of one row (2^m s each, partial k at
// base + k stride), in order of k: chunks of 16 partials are loaded together
// (one memory round trip per chunk; lanes past n read partial 0 again, in
// bounds, and drop it), the chunk's maximum taken, and the running sum
// rescaled once per chunk; -inf when n = 0 or every partial is -inf
template <typename T>
__device__ __forceinline__ T merge_parts(const T* __restrict__ pm, const T* __restrict__ ps, int64_t stride,
                                         int64_t base, int n) {
  constexpr int C = 16;
  T m = Num<T>::ninf(), acc = T(0);
  for (int k0 = 0; k0 < n; k0 += C) {
    T a[C], b[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const bool ok = k0 + k < n;
      const int64_t off = base + (int64_t)(ok ? k0 + k : 0) * stride;
      const T pa = pm[off], pb = ps[off];
      a[k] = ok ? pa : Num<T>::ninf();
      b[k] = ok ? pb : T(0);
    }
    T cm = a[0];
#pragma unroll
    for (int k = 1; k < C; ++k) cm = Num<T>::fmax(cm, a[k]);
    const T mn = Num<T>::fmax(m, cm);
    if (mn != Num<T>::ninf()) {
      T sum = acc * Num<T>::exp2(m - mn);
#pragma unroll
      for (int k = 0; k < C; ++k) sum += b[k] * Num<T>::exp2(a[k] - mn);
      acc = sum;
      m = mn;
    }
  }
  return m == Num<T>::ninf() ? m : m + Num<T>::log2(acc);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_epi(const T* __restrict__ pm, const T* __restrict__ ps,
                                                       int nsplit, int64_t Nr, int side,
                                                       const Ctrl* __restrict__ c, EpiArgs<T> ep) {
  if (skip_side(c, side)) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < Nr;
  ResAcc<T> ra;
  ra.init();
  // the column splits of k_dense_lse (partial k of row i at k Nr + i)
  if (valid) epi_elem<T>(i, merge_parts<T>(pm, ps, Nr, i, nsplit), c, side, ep, ra);
  epi_finish<T>(ep, ra, blockIdx.x);
}

// ---------------------------------------------------------------------------
// control kernel (one block), between the X and the Y half-step: reduce the
// residual partials, count the iteration, pick the next eps, set stop flags.
// ---------------------------------------------------------------------------
// control step (one block of 256 threads): reduce the residual partials,
// count the iteration, pick the next eps, set the stop flag.  (Folding this
// step into the last block of the final pass needs a device-scope fence in
// every block, which on a multi-XCD MI355X costs more than the launch.)
__device__ void control_step(Ctrl* __restrict__ c, const ResPart* __restrict__ part, int nparts,
                             double* __restrict__ hist, int nfields, int par) {
  // nfields > 0: the partials form nfields equal contiguous ranges (one per
  // field) and r is the largest per-field residual
  __shared__ float smax[kBlock], sdu[kBlock];
  const CtrlSnap snap = ctrl_snap(c, par);
  float rmax = -1.0f, du = 0.f;
  const int per = nparts / nfields;
  for (int f = threadIdx.x; f < nfields; f += kBlock) {
    float m = -__builtin_inff(), den = 0.f, num = 0.f;
    for (int k = f * per; k < (f + 1) * per; ++k) {
      res_merge<float>(m, den, num, part[k].m, part[k].den, part[k].num);
      du = fmaxf(du, part[k].du);
    }
    const float rf = float(res_ratio(double(num), double(den)));
    rmax = (rf != rf || rmax != rmax) ? rf : (rf > rmax ? rf : rmax);
  }
  smax[threadIdx.x] = rmax;
  sdu[threadIdx.x] = du;
  __syncthreads();
  for (int off = kBlock / 2; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const float a = smax[threadIdx.x], b = smax[threadIdx.x + off];
      smax[threadIdx.x] = (a != a || b != b) ? (a != a ? a : b) : (a > b ? a : b);
      sdu[threadIdx.x] = fmaxf(sdu[threadIdx.x], sdu[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) control_finish(c, snap, double(smax[0]), double(sdu[0]), hist, par);
}

// control step of iteration parity par as its own launch.  Single problem:
// the partials and the control fields are loaded before the skip flag is
// tested, then reduced with wave exchanges.
__global__ __launch_bounds__(kBlock) void k_control(Ctrl* __restrict__ c, const ResPart* __restrict__ part,
                                                     int nparts, double* __restrict__ hist, int nfields, int par) {
  if (nfields > 0) {
    if (c->skip[par]) {
      if (threadIdx.x == 0) control_skip(c, par);
      return;
    }
    control_step(c, part, nparts, hist, nfields, par);
    return;
  }
  const CtrlSnap snap = ctrl_snap(c, par);
  float m, den, num, du;
  ctl_load(part, nparts, m, den, num, du);
  asm volatile("" ::"v"(m), "v"(den), "v"(num), "v"(du));
  if (c->skip[par]) {
    if (threadIdx.x == 0) control_skip(c, par);
    return;
  }
  ctl_reduce_finish(c, snap, m, den, num, du, hist, par);
}

// plain reduction of residual partials into out[0] (single half-step entry)
__global__ void k_res_reduce(const ResPart* __restrict__ part, int nparts, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double m = -__builtin_inf(), den = 0.0, num = 0.0;
  for (int k = 0; k < nparts; ++k) res_merge<double>(m, den, num, part[k].m, part[k].den, part[k].num);
  out[0] = res_ratio(num, den);
}

// continue a stopped solve with a new tolerance (the second phase of a
// mixed-precision grid solve): clear the stop and skip flags, keep the
// iteration count, residual history and eps slots
// ---------------------------------------------------------------------------
// barycentric projection (colour transfer): T_i = sum_j R_ij dy_j y_j /
// sum_j R_ij dy_j as a ratio of two Gibbs products of the same row, the
// numerator's input weighted by one coordinate of y_j (log domain: its log2
// added to w).  Grid coordinates (cell centres) are positive; point
// coordinates are split into positive and negative parts.
// ---------------------------------------------------------------------------
// out[j] = w[j] + log2 y_j^(k): grid cell centre (j_k + 1/2) h_k with
// j_k = (j / stride) % nk, or, for points (yk != null), log2 max(sign yk[j], 0)
template <typename T>
__global__ void k_coord_weight(const T* __restrict__ w, T* __restrict__ out, int64_t M, int64_t stride, int64_t nk,
                               double hk, const T* __restrict__ yk, int sign) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  T lc;
  if (yk) {
    const T y = T(sign) * yk[j];
    lc = y > T(0) ? Num<T>::log2(y) : Num<T>::ninf();
  } else {
    const int64_t jk = (j / stride) % nk;
    lc = T(::log2((double(jk) + 0.5) * hk));
  }
  out[j] = w[j] + lc;
}

// T[i] = 2^{num[i] - den[i]} (- 2^{neg[i] - den[i]}); NaN where the row of
// the plan vanishes (den = -inf)
template <typename T>
__global__ void k_map_finish(T* __restrict__ num, const T* __restrict__ den, const T* __restrict__ neg, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const T d = den[i];
  if (d == Num<T>::ninf()) {
    num[i] = T(__builtin_nan(""));
    return;
  }
  T t = Num<T>::exp2(num[i] - d);
  if (neg) t -= Num<T>::exp2(neg[i] - d);
  num[i] = t;
}

template <typename T>
void launch_coord_weight(const T* w, T* out, int64_t M, int64_t stride, int64_t nk, double hk, const T* yk, int sign,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_coord_weight<T>, dim3(ceil_div(M, kBlock)), dim3(kBlock), 0, s, w, out, M, stride, nk, hk, yk,
                     sign);
}
template <typename T>
void launch_map_finish(T* num, const T* den, const T* neg, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(k_map_finish<T>, dim3(ceil_div(N, kBlock)), dim3(kBlock), 0, s, num, den, neg, N);
}
template void launch_coord_weight<float>(const float*, float*, int64_t, int64_t, int64_t, double, const float*, int,
                                         hipStream_t);
template void launch_coord_weight<double>(const double*, double*, int64_t, int64_t, int64_t, double, const double*, int,
                                          hipStream_t);
template void launch_map_finish<float>(float*, const float*, const float*, int64_t, hipStream_t);
template void launch_map_finish<double>(double*, const double*, const double*, int64_t, hipStream_t);

// after a stopped solve, slot 0 is made valid again for one more product at
// the eps of the last iteration (a stopped solve marks its slots skipped)
__global__ void k_ctrl_post(Ctrl* __restrict__ c) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t l = c->iter > 0 ? c->iter - 1 : 0;
  int64_t sn = c->iters_per_stage > 0 ? l / c->iters_per_stage : c->n_stages;
  if (sn > c->n_stages) sn = c->n_stages;
  c->stage[0] = (int)sn;
  c->eps[0] = c->eps_tab[sn];
  c->skip[0] = 0;
}

__global__ void k_ctrl_resume(Ctrl* __restrict__ c, double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  c->stop = 0;
  c->status = 1;
  c->skip[0] = c->skip[1] = 0;
  c->tol = tol;
}

// total-mass step of Algorithm 4 (one block): log m from the mass partials of
// the Y half-step, then log z = log proxdiv_F3(m) with p = m0 on the
// one-point space, at the eps of the iteration
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mass_update(Ctrl* __restrict__ c, const T* __restrict__ mm,
                                                         const T* __restrict__ ms, int nparts, DivDev F3,
                                                         double log_m0, int par) {
  if (c->skip[par]) return;
  Lse2<T> a;
  a.init();
  for (int k = threadIdx.x; k < nparts; k += kBlock) a.merge(mm[k], ms[k]);
  __shared__ T om, os;
  block_lse_reduce<T>(a.m, a.s, &om, &os);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double logm = (double(om) + ::log2(double(os))) * kLn2;
    const double eps = c->eps[par];
    c->zeta = proxdiv_pot<double>(F3, log_m0, logm, eps) / eps;
  }
}

__global__ void k_ctrl_init(Ctrl* __restrict__ c, Ctrl init) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = init;
}

// ---------------------------------------------------------------------------
// barycentre combine (Table estimatebary rows (i)/(ii), log form) after the
// Y Gibbs product: T2 (n x size, log2 units) ->  log h (natural), and
//   v_k = eps log proxdiv_{F2(.|h)}(e^{T_k}),  w_k = (v_k/eps_next + log dy) log2(e)
// ---------------------------------------------------------------------------
// Table estimatebary (iii) lam TV / (iv) RG[b1, b2]: log h is a root of
//   TV: A0 + sum_{k: s_k>0} alpha_k clamp((x - log s_k) eps/lam, -1, 1)   (A0: weight of s_k = 0)
//   RG: sum_k alpha_k [b2 min(x + log b2 - log s_k, 0) + b1 max(x + log b1 - log s_k, 0)]
// in x = log h; both are non-decreasing and linear between their breakpoints
// (log s_k -+ lam/eps, log s_k - log b_i).  The smallest root is taken: the
// first breakpoint where the function is >= 0, linear interpolation from the
// breakpoint before it.  h = 0 (TV: A0 >= weight of the others; RG: some
// s_k = 0).  t2: log2 s_k at stride `stride`.

// breakpoint w (0, 1) of input k, natural log t: TV t -+ d, RG t - log b2 / t - log b1
template <typename T>
__device__ __forceinline__ T bary_break(bool tv, T t, int w, T d, T lb1, T lb2) {
  return tv ? (w == 0 ? t - d : t + d) : (w == 0 ? t - lb2 : t - lb1);
}

// TV / RG barycentre combine with L lanes per cell (L a power of two, 2..64):
// each lane evaluates f at its share of the cell's breakpoints, segmented
// shuffle reductions over the L lanes find the smallest breakpoint with
// f >= 0 and the largest one below it, and f is linear in between.  Spreading
// the breakpoints over lanes replaces one long dependent loop per cell, which
// left a launch of a few blocks waiting on memory.
template <typename T>
__device__ __forceinline__ T bary_fa(const T* __restrict__ t2, int64_t stride, int n, const BaryW& la, bool tv, T a0,
                                     T d, T lb1, T lb2, T b1, T b2, bool has_lo, T x) {
  T acc = tv ? a0 : T(0);
  for (int k = 0; k < n; ++k) {
    const T t = t2[k * stride] * T(kLn2);
    if (t == Num<T>::ninf()) continue;
    const T al = T(la.a[k]);
    if (tv) {
      const T y = (x - t) / d;
      acc += al * (y < T(-1) ? T(-1) : (y > T(1) ? T(1) : y));
    } else {
      const T up = x + lb2 - t, dn = x + lb1 - t;
      T term = b2 * (up < T(0) ? up : T(0));
      if (has_lo) term += b1 * (dn > T(0) ? dn : T(0));
      acc += al * term;
    }
  }
  return acc;
}

template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_bary_root(const T* __restrict__ T2, int nm, int64_t size, BaryW la,
                                                       DivDev F2, const T* __restrict__ logdy, T* __restrict__ v,
                                                       T* __restrict__ w, T* __restrict__ logh_out,
                                                       const Ctrl* __restrict__ c, int side) {
  if (skip_side(c, side)) return;
  const int sub = threadIdx.x & (L - 1);
  const int64_t j = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / L;
  const bool valid = j < size;
  const T* __restrict__ t2 = T2 + (valid ? j : size - 1);   // every lane takes part in the shuffles
  const T eps = T(eps_of(c, side));
  const T eps_w = T(eps_next_of(c, side));
  const bool tv = F2.kind == 2;
  const bool lo = F2.has_lo != 0;
  T a0 = T(0), a1 = T(0), tmax = Num<T>::ninf(), tmin = Num<T>::pinf();
  for (int k = 0; k < nm; ++k) {
    const T t = t2[k * size] * T(kLn2);
    const T al = T(la.a[k]);
    if (t == Num<T>::ninf()) {
      a0 += al;
    } else {
      a1 += al;
      tmax = t > tmax ? t : tmax;
      tmin = t < tmin ? t : tmin;
    }
  }
  // the cases with a closed answer: no mass (-inf), or RG with every input in
  // one band (the left end of the zero interval, exactly)
  bool closed = false;
  T logh = T(0);
  if (tv ? (a0 >= a1) : (a0 > T(0))) {
    closed = true;
    logh = Num<T>::ninf();
  } else if (!tv) {
    const T left = tmax - T(F2.log_beta);
    if (!lo || left <= tmin - T(F2.log_alpha)) {
      closed = true;
      logh = left;
    }
  }
  const T d = tv ? T(F2.lam) / eps : T(0);
  const T lb1 = lo ? T(F2.log_alpha) : T(0), lb2 = T(F2.log_beta);
  const T b1 = lo ? T(::exp(F2.log_alpha)) : T(0), b2 = T(::exp(F2.log_beta));
  const int per = tv ? 2 : (lo ? 2 : 1);
  const int nbp = nm * per;
  // smallest breakpoint with f >= 0 (and f there)
  T bhi = Num<T>::pinf(), fhi = T(0);
  for (int q = sub; q < nbp; q += L) {
    const int k = q / per, wq = q % per;
    const T t = t2[k * size] * T(kLn2);
    if (t == Num<T>::ninf()) continue;
    const T b = bary_break<T>(tv, t, wq, d, lb1, lb2);
    const T fb = bary_fa<T>(t2, size, nm, la, tv, a0, d, lb1, lb2, b1, b2, lo, b);
    if (fb >= T(0) && b < bhi) {
      bhi = b;
      fhi = fb;
    }
  }
#pragma unroll
  for (int o = L / 2; o >= 1; o >>= 1) {
    const T ob = __shfl_xor(bhi, o), of = __shfl_xor(fhi, o);
    if (ob < bhi || (ob == bhi && of < fhi)) {
      bhi = ob;
      fhi = of;
    }
  }
  // largest breakpoint below it
  T blo = Num<T>::ninf();
  for (int q = sub; q < nbp; q += L) {
    const int k = q / per, wq = q % per;
    const T t = t2[k * size] * T(kLn2);
    if (t == Num<T>::ninf()) continue;
    const T b = bary_break<T>(tv, t, wq, d, lb1, lb2);
    if (b < bhi && b > blo) blo = b;
  }
#pragma unroll
  for (int o = L / 2; o >= 1; o >>= 1) {
    const T ob = __shfl_xor(blo, o);
    blo = ob > blo ? ob : blo;
  }
  if (!closed) {
    if (blo == Num<T>::ninf()) {
      logh = bhi;
    } else {
      const T flo = bary_fa<T>(t2, size, nm, la, tv, a0, d, lb1, lb2, b1, b2, lo, blo);
      logh = blo + (T(0) - flo) * (bhi - blo) / (fhi - flo);
    }
  }
  if (!valid) return;
  if (sub == 0 && logh_out) logh_out[j] = logh;
  const T ld = logdy[j];
  for (int k = sub; k < nm; k += L) {
    const T S = T2[k * size + j] * T(kLn2);
    const T vn = proxdiv_pot<T>(F2, logh, S, eps);
    v[k * size + j] = vn;
    w[k * size + j] = (S == Num<T>::ninf()) ? Num<T>::ninf() : (vn / eps_w + ld) * T(kLog2e);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bary_combine(const T* __restrict__ T2, int nm, int64_t size,
                                                          BaryW log_alpha, double log_sum_alpha,
                                                          DivDev F2, const T* __restrict__ logdy,
                                                          T* __restrict__ v, T* __restrict__ w, T* __restrict__ logh_out,
                                                          const Ctrl* __restrict__ c, int side) {
  if (skip_side(c, side)) return;
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= size) return;
  const T eps = T(eps_of(c, side));
  const T eps_w = T(eps_next_of(c, side));
  T logh;   // (TV and RG barycentres run in k_bary_root)
  if (F2.kind == 0) {
    double acc = 0.0, asum = 0.0;
    for (int k = 0; k < nm; ++k) {
      const double al = ::exp(log_alpha.v[k]);
      acc += al * double(T2[k * size + j]) * kLn2;
      asum += al;
    }
    logh = T(acc / asum);
  } else {
    const T gam = eps / (eps + T(F2.lam));           // eps/(eps+lam)
    Lse2<T> a;
    a.init();
    for (int k = 0; k < nm; ++k) {
      T t[1] = {T(log_alpha.v[k] * kLog2e) + gam * T2[k * size + j]};
      a.template add<1>(t);
    }
    logh = (a.result() * T(kLn2) - T(log_sum_alpha)) / gam;
  }
  if (logh_out) logh_out[j] = logh;
  const T ld = logdy[j];
  for (int k = 0; k < nm; ++k) {
    const T S = T2[k * size + j] * T(kLn2);
    const T vn = proxdiv_pot<T>(F2, logh, S, eps);
    v[k * size + j] = vn;
    w[k * size + j] = (S == Num<T>::ninf()) ? Num<T>::ninf() : (vn / eps_w + ld) * T(kLog2e);
  }
}

// ---------------------------------------------------------------------------
// gradient flows (Sec. 5.3)
// ---------------------------------------------------------------------------
// Y update of the multi-species growth step: the joint proxdiv of the growth
// functional (F, kind 4, cap q) at the sum of the species' products,
// L = log sum_k e^{T_k}; the potential v is the same for every species.
// T2: nm x size in log2 units.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_growth_combine(const T* __restrict__ T2, int nm, int64_t size,
                                                            DivDev F, const T* __restrict__ logq,
                                                            const T* __restrict__ logdy, T* __restrict__ v,
                                                            T* __restrict__ w, const Ctrl* __restrict__ c, int side) {
  if (skip_side(c, side)) return;
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= size) return;
  const T eps = T(eps_of(c, side));
  const T eps_w = T(eps_next_of(c, side));
  Lse2<T> a;
  a.init();
  for (int k = 0; k < nm; ++k) {
    T t[1] = {T2[k * size + j]};
    a.template add<1>(t);
  }
  const T vn = proxdiv_pot<T>(F, logq[j], a.result() * T(kLn2), eps);
  const T wn = (vn / eps_w + logdy[j]) * T(kLog2e);
  for (int k = 0; k < nm; ++k) {
    v[k * size + j] = vn;
    w[k * size + j] = (T2[k * size + j] == Num<T>::ninf()) ? Num<T>::ninf() : wn;
  }
}

// next densities of a gradient-flow step from the final potentials: the
// second marginals y_k = e^{T_k + v_k/eps} of the couplings (T2: log2 of
// K^T(a_k dx)), as they are (heat, crowd) or, for growth, the inner
// minimiser of the growth functional, y_k / max(kappa, sum_k y_k / q)
template <typename T>
__device__ __forceinline__ T flow_logy(const T* __restrict__ T2, const T* __restrict__ v, int64_t e, T eps) {
  const T t = T2[e];
  return t == Num<T>::ninf() ? Num<T>::ninf() : t * T(kLn2) + v[e] / eps;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_flow_next(const T* __restrict__ T2, const T* __restrict__ v,
                                                       const T* __restrict__ logq, int nm, int64_t size, int growth,
                                                       double log_kappa, const Ctrl* __restrict__ c,
                                                       T* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= size) return;
  const T eps = T(c->eps[0]);
  T den = T(0);
  if (growth) {
    T m = Num<T>::ninf();
    for (int k = 0; k < nm; ++k) m = Num<T>::fmax(m, flow_logy<T>(T2, v, k * size + j, eps));
    T sum = T(0);
    if (m != Num<T>::ninf())
      for (int k = 0; k < nm; ++k) sum += Num<T>::exp(flow_logy<T>(T2, v, k * size + j, eps) - m);
    const T L = m == Num<T>::ninf() ? m : m + Num<T>::log(sum);
    const T lq = logq[j];
    den = lq == Num<T>::ninf() ? Num<T>::pinf() : Num<T>::fmax(T(log_kappa), L - lq);
  }
  for (int k = 0; k < nm; ++k) out[k * size + j] = Num<T>::exp(flow_logy<T>(T2, v, k * size + j, eps) - den);
}

// ---------------------------------------------------------------------------
// objective terms in FP64 (Thm. duality at the plan R = e^{(u+v-C)/eps}):
// per element of one side, with S = log of the Gibbs product of the other
// side's scaling (natural log):
//   pi = e^{pot/eps + S};  acc[0] += d pi; acc[1] += d pot pi;
//   acc[2] += d f(pi | p); acc[3] += d f*(-pot | p)
// written as per-block partials (4 doubles each).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_obj_side(const T* __restrict__ pot, const T* __restrict__ S,
                                                      const T* __restrict__ p, const T* __restrict__ d,
                                                      int64_t n, double eps, DivDev F, T* __restrict__ pi_out,
                                                      double* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  if (i < n) {
    const double u = double(pot[i]);
    const double s = double(S[i]) * kLn2;   // S arrives in log2 units
    const double pp = double(p[i]);
    const double dd = double(d[i]);
    // no mass where the potential or the product vanishes (0 times any potential)
    const double pi = (u == -__builtin_inf() || s == -__builtin_inf()) ? 0.0 : ::exp(u / eps + s);
    if (pi_out) pi_out[i] = T(pi);
    a0 = dd * pi;
    a1 = (pi > 0) ? dd * u * pi : 0.0;
    const double w = -u;   // conjugate argument
    const double lam = F.lam;
    switch (F.kind) {
      case 1:  // lam KL
        a2 = dd * lam * ((pi > 0 ? pi * ::log(pi / pp) : 0.0) - pi + pp);
        if (pp == 0.0 && pi > 0) a2 = __builtin_inf();
        a3 = (pp > 0) ? dd * lam * pp * ::expm1(w / lam) : 0.0;
        break;
      case 2:  // lam TV
        a2 = dd * lam * ::fabs(pi - pp);
        a3 = (w > lam * (1 + 1e-6)) ? __builtin_inf() : dd * pp * ::fmax(w, -lam);
        break;
      case 4: {  // growth, cap pp: F = s log kappa below kappa pp, s log(s/pp) - s + kappa pp above
        const double kap = 1.0 - lam;
        if (pp == 0.0) a2 = pi > 0 ? __builtin_inf() : 0.0;
        else a2 = dd * (pi <= kap * pp ? pi * ::log(kap) : pi * ::log(pi / pp) - pi + kap * pp);
        a3 = dd * pp * ::fmax(::exp(w) - kap, 0.0);
        break;
      }
      default:  // = / RG: indicator terms are not finite-valued; gap reported as NaN by the host
        a2 = 0.0;
        a3 = 0.0;
        if (F.kind == 0) a3 = (pp > 0) ? dd * pp * w : 0.0;
        else {
          const double al = F.has_lo ? ::exp(F.log_alpha) : 0.0;
          const double be = F.has_hi ? ::exp(F.log_beta) : __builtin_inf();
          a3 = (pp > 0) ? dd * pp * ((w > 0) ? be * w : al * w) : 0.0;
        }
        break;
    }
  }
  __shared__ double sm[4][kBlock];
  sm[0][threadIdx.x] = a0;
  sm[1][threadIdx.x] = a1;
  sm[2][threadIdx.x] = a2;
  sm[3][threadIdx.x] = a3;
  __syncthreads();
  for (int off = kBlock / 2; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int q = 0; q < 4; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sm[threadIdx.x][0];
}

// sum_i exp2(a_i + b_i) (or exp2(b_i) when a is null) in FP64, per-block partials
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sum_exp2(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                                      double* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double x = (a ? double(a[i]) : 0.0) + double(b[i]);
    v = (x == -__builtin_inf()) ? 0.0 : ::exp2(x);
  }
  __shared__ double sm[kBlock];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int off = kBlock / 2; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) sm[threadIdx.x] += sm[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// dense transport-cost moment: for row i, log2 sum_j C_ij 2^{w_j - sc C_ij}
// (single block column loop; one thread per row; used once per objective)
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_dense_cost(const T* __restrict__ xr, int64_t Nr,
                                                        const T* __restrict__ yc, const T* __restrict__ w,
                                                        int64_t Mc, double eps, T* __restrict__ out, CostArgs cost) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= Nr) return;
  const double sc = kLog2e / eps;
  double xi[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) xi[d] = double(xr[d * Nr + i]);
  double m = -__builtin_inf(), s = 0.0;
  for (int64_t j = 0; j < Mc; ++j) {
    double cst = 0.0;
    for (int d = 0; d < DIM; ++d) {
      const double dd = xi[d] - double(yc[d * Mc + j]);
      cst += dd * dd;
    }
    if (cost.kind == 1) {
      // WF: c = -2 log cos((pi/2) d / cut); no mass beyond the cut
      if (cst >= cost.cut * cost.cut) continue;
      cst = -2.0 * ::log(::cos(0.5 * M_PI * ::sqrt(cst) / cost.cut));
    }
    const double t = double(w[j]) - sc * cst;
    if (t == -__builtin_inf() || cst == 0.0) continue;
    const double tt = t + ::log2(cst);
    if (tt > m) {
      s = s * ::exp2(m - tt) + 1.0;
      m = tt;
    } else {
      s += ::exp2(tt - m);
    }
  }
  out[i] = T(m + ::log2(s));
}

// grid cost table: tab[k] = g_s[k] + log2(C1(k)) at the current X stage (-inf at 0 offset)
template <typename T>
__global__ void k_gtab_cost(T* __restrict__ tab, int n, double h, double eps, CostArgs cost) {
  const int len = 2 * n - 1;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  const double d = double(k - (n - 1)) * h;
  double cst = d * d;
  if (cost.kind == 1) {
    const double ad = ::fabs(d);
    cst = ad < cost.cut ? -2.0 * ::log(::cos(0.5 * M_PI * ad / cost.cut)) : __builtin_inf();
  }
  tab[k] = (cst == 0.0 || cst == __builtin_inf()) ? T(-__builtin_inf()) : T(-cst / eps * kLog2e + ::log2(cst));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T>
void launch_log(const T* src, T* dst, int64_t n, int zero_is_ninf, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_log<T>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, src, dst, n, zero_is_ninf);
}

template <typename T>
void launch_init_pot(const T* v0, const T* logd, T* pot, T* w, int64_t n, int64_t size, const Ctrl* c, int which,
                     hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_init_pot<T>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, v0, logd, pot, w, n, size, c, which);
}

template <typename T>
void launch_gtab(T* tab, int n, double h, const Ctrl* c, int nst, const CostArgs& cost, hipStream_t s) {
  const int64_t tot = (int64_t)(2 * n - 1) * nst;
  hipLaunchKernelGGL(k_gtab<T>, dim3(ceil_div(tot, kBlock)), dim3(kBlock), 0, s, tab, n, h, c, nst, cost);
}

template <typename T>
void launch_gtab_cost(T* tab, int n, double h, double eps, const CostArgs& cost, hipStream_t s) {
  hipLaunchKernelGGL(k_gtab_cost<T>, dim3(ceil_div(2 * n - 1, kBlock)), dim3(kBlock), 0, s, tab, n, h, eps, cost);
}

// outputs per lane: 2 when one output per lane would already give more than
// 8 waves per SIMD, else 1 (latency hiding for small grids)
static int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v ? atoi(v) : dflt;
}
static inline int strided_ri(int n, int64_t A, int64_t B) {
  static const int forced = env_int("UOT_STRIDED_RI", 0);
  if (forced == 1 || forced == 2) return forced;
  const int64_t blocks1 = (int64_t)ceil_div(B, 64) * n * A;
  return blocks1 * 4 > 8 * 1024 ? 2 : 1;
}
static inline int contig_ri(int n, int64_t A) {
  const int64_t blocks1 = (int64_t)ceil_div(n, 64) * A;
  return blocks1 * 4 > 8 * 1024 ? 2 : 1;
}
static inline void contig_grid(int n, int64_t A, int ri, unsigned& gx, unsigned& gy, unsigned& gz) {
  const int64_t ylim = 65535;
  const int64_t y = A < ylim ? A : ylim;
  gx = ceil_div(n, 64 * ri);
  gy = (unsigned)y;
  gz = (unsigned)((A + y - 1) / y);
}

template <typename T>
int grid_strided_parts(int n, int64_t A, int64_t B) {
  const int ri = strided_ri(n, A, B);
  return (int)(ceil_div(B, 64) * (int64_t)ceil_div(n, ri) * A);
}

template <typename T>
int grid_contig_parts(int n, int64_t A) {
  unsigned gx, gy, gz;
  contig_grid(n, A, contig_ri(n, A), gx, gy, gz);
  return (int)((int64_t)gx * gy * gz);
}

template <typename T>
void launch_grid_strided(const T* in, int64_t A, int n, int64_t B, const T* gtab, int side, const Ctrl* c,
                         const EpiArgs<T>& ep, hipStream_t s) {
  const int ri = strided_ri(n, A, B);
  dim3 grid(ceil_div(B, 64), ceil_div(n, ri), (unsigned)A);
  const size_t lds = (size_t)(2 * n - 1) * sizeof(T);
  if (ri == 2) hipLaunchKernelGGL((k_grid_strided<T, 2>), grid, dim3(kBlock), lds, s, in, n, B, gtab, side, c, ep);
  else hipLaunchKernelGGL((k_grid_strided<T, 1>), grid, dim3(kBlock), lds, s, in, n, B, gtab, side, c, ep);
}

template <typename T>
void launch_grid_contig(const T* in, int64_t A, int n, const T* gtab, int side, const Ctrl* c,
                        const EpiArgs<T>& ep, int band, hipStream_t s) {
  const int ri = contig_ri(n, A);
  unsigned gx, gy, gz;
  contig_grid(n, A, ri, gx, gy, gz);
  const size_t lds = (size_t)(2 * n - 1) * sizeof(T);
  const int bd = (band < 1 || band > n) ? n : band;
  if (ri == 2)
    hipLaunchKernelGGL((k_grid_contig<T, 2, false>), dim3(gx, gy, gz), dim3(kBlock), lds, s, in, n, A, gtab, side, c,
                       ep, bd, (T*)nullptr, (T*)nullptr, 1);
  else
    hipLaunchKernelGGL((k_grid_contig<T, 1, false>), dim3(gx, gy, gz), dim3(kBlock), lds, s, in, n, A, gtab, side, c,
                       ep, bd, (T*)nullptr, (T*)nullptr, 1);
}

// tap slices for few long lines (A x ceil(n/64) blocks well below the chip's
// width): enough slices for ~2048 blocks, each slice at least 256 taps
int grid_contig_splits(int n, int64_t A, int band) {
  const int bd = (band < 1 || band > n) ? n : band;
  const int64_t blocks1 = (int64_t)ceil_div(n, 64) * A;
  if (blocks1 >= 1024 || A > 65535) return 1;
  const int taps = std::min(n, 2 * bd - 1);
  int64_t sp = (2048 + blocks1 - 1) / blocks1;
  const int64_t maxsp = std::max(1, taps / 256);
  return (int)std::max<int64_t>(1, std::min(sp, maxsp));
}

template <typename T>
void launch_grid_contig_split(const T* in, int64_t A, int n, const T* gtab, int side, const Ctrl* c, int band,
                              int nsplit, T* pm, T* ps, hipStream_t s) {
  const int bd = (band < 1 || band > n) ? n : band;
  const size_t lds = (size_t)(2 * n - 1) * sizeof(T);
  EpiArgs<T> none{};
  hipLaunchKernelGGL((k_grid_contig<T, 1, true>), dim3(ceil_div(n, 64), (unsigned)A, (unsigned)nsplit), dim3(kBlock),
                     lds, s, in, n, A, gtab, side, c, none, bd, pm, ps, nsplit);
}

template <typename T, int DIM, int R>
static void launch_dense_lse_t(const T* xr, int64_t Nr, const T* yc, const T* w, int64_t Mc, int nsplit,
                               int64_t cps, T* pm, T* ps, int side, const Ctrl* c, const CostArgs& cost,
                               hipStream_t s) {
  dim3 grid(ceil_div(Nr, kBlock * R), (unsigned)nsplit);
  if (cost.kind == 1) {
    const T a2 = T(0.25 * M_PI * M_PI / (cost.cut * cost.cut)), cut2 = T(cost.cut * cost.cut);
    hipLaunchKernelGGL((k_dense_lse<T, DIM, R, 1>), grid, dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, cps, pm, ps, side,
                       c, a2, cut2);
  } else {
    hipLaunchKernelGGL((k_dense_lse<T, DIM, R, 0>), grid, dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, cps, pm, ps, side,
                       c, T(0), T(0));
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_chunk_boxes(const T* __restrict__ pts, int64_t n, int64_t per, int dim,
                                                         T* __restrict__ out) {
  __shared__ T red[2][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < n ? b0 + per : n;
  for (int d = 0; d < 3; ++d) {
    T lo = Num<T>::pinf(), hi = Num<T>::ninf();
    if (d < dim)
      for (int64_t i = b0 + threadIdx.x; i < b1; i += kBlock) {
        lo = Num<T>::fmin(lo, pts[d * n + i]);
        hi = Num<T>::fmax(hi, pts[d * n + i]);
      }
    lo = lanes_min<T>(lo, 32);
    hi = lanes_max<T>(hi, 32);
    __syncthreads();                       // the previous coordinate's reads are done
    if (lane == 0) {
      red[0][wv] = lo;
      red[1][wv] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      lo = Num<T>::fmin(Num<T>::fmin(red[0][0], red[0][1]), Num<T>::fmin(red[0][2], red[0][3]));
      hi = Num<T>::fmax(Num<T>::fmax(red[1][0], red[1][1]), Num<T>::fmax(red[1][2], red[1][3]));
      out[6 * (int64_t)blockIdx.x + 2 * d] = d < dim ? lo : T(0);
      out[6 * (int64_t)blockIdx.x + 2 * d + 1] = d < dim ? hi : T(0);
    }
  }
}

template <typename T>
void launch_chunk_boxes(const T* pts, int64_t n, int64_t per, int dim, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_chunk_boxes<T>, dim3(ceil_div(n, per)), dim3(kBlock), 0, s, pts, n, per, dim, out);
}

// ---------------------------------------------------------------------------
// WF point clouds on work lists.  K is exactly zero beyond the cut, so a
// product only needs the (row wave of 64 rows, group of 16 columns) pairs
// whose boxes lie within the cut of each other.  Once per solve (the
// geometry is fixed): the boxes of the row waves and of the column groups,
// one mask bit per (row wave, group) pair within the cut (k_wf_mask), and
// the work units of every row wave: consecutive ranges [g0, g1) of its
// groups that hold kWfUnitGroups groups within the cut, the last one
// possibly fewer (k_wf_units).  Per half-step one wave per unit stages the
// unit's columns in its own LDS and sums its row wave's 64 rows (one per
// lane) over them (k_wf_lse), and k_wf_epi merges each row's units in unit
// order and applies the epilogue.  Unit k of row wave rw sits in slot
// k nrw + rw (at most ceil(groups / kWfUnitGroups) units per row wave), so
// the busy slots come first in the launch.
// ---------------------------------------------------------------------------
constexpr int kWfUnitGroups = 16;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_wf_mask(const T* __restrict__ rbox, int64_t nrw,
                                                     const T* __restrict__ gbox, int64_t ngr, int nwd, int dim, T cut2,
                                                     uint32_t* __restrict__ mask) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= nrw * nwd) return;
  const int64_t rw = t / nwd;
  const int wd = (int)(t % nwd);
  const T* rb = rbox + 6 * rw;
  uint32_t bits = 0;
  for (int b = 0; b < 32; ++b) {
    const int64_t g = (int64_t)wd * 32 + b;
    if (g >= ngr) break;
    const T* cb = gbox + 6 * g;
    T gap2 = T(0);
    for (int d = 0; d < dim; ++d) {
      const T e = Num<T>::fmax(Num<T>::fmax(cb[2 * d] - rb[2 * d + 1], rb[2 * d] - cb[2 * d + 1]), T(0));
      gap2 = Num<T>::fma(e, e, gap2);
    }
    if (gap2 < cut2) bits |= 1u << b;
  }
  mask[t] = bits;
}

__global__ __launch_bounds__(kBlock) void k_wf_units(const uint32_t* __restrict__ mask, int64_t nrw, int nwd,
                                                      int2* __restrict__ units, int* __restrict__ ucnt,
                                                      int* __restrict__ umax) {
  const int64_t rw = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (rw >= nrw) return;
  const uint32_t* m = mask + rw * nwd;
  int n = 0, g0 = -1, cnt = 0, last = 0;
  for (int wd = 0; wd < nwd; ++wd) {
    uint32_t bits = m[wd];
    while (bits) {
      const int g = wd * 32 + __builtin_ctz(bits);
      bits &= bits - 1;
      if (g0 < 0) g0 = g;
      last = g + 1;
      if (++cnt == kWfUnitGroups) {
        units[(int64_t)n++ * nrw + rw] = make_int2(g0, last);
        g0 = -1;
        cnt = 0;
      }
    }
  }
  if (g0 >= 0) units[(int64_t)n++ * nrw + rw] = make_int2(g0, last);
  ucnt[rw] = n;
  atomicMax(umax, n);
}

__global__ void k_zero_int(int* p) { *p = 0; }


template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_wf_lse(const T* __restrict__ xr, int64_t Nr, const T* __restrict__ yc,
                                                    const T* __restrict__ w, int64_t Mc,
                                                    const uint32_t* __restrict__ mask, const int2* __restrict__ units,
                                                    const int* __restrict__ ucnt, int nwd, T* __restrict__ pm,
                                                    T* __restrict__ ps, int side, const Ctrl* __restrict__ c, T a2,
                                                    T cut2) {
  using V4 = typename Vec4<T>::type;
  // per wave: its unit's groups and their columns (x, y, z, w)
  __shared__ int glist[kBlock / 64][kWfUnitGroups];
  __shared__ V4 cols[kBlock / 64][kWfUnitGroups * 16];
  if (skip_side(c, side)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nrw = (Nr + 63) / 64;
  const int64_t slot = (int64_t)blockIdx.x * (kBlock / 64) + wv;
  const int64_t rw = slot % nrw, k = slot / nrw;
  // a wave past its row wave's units has no work, but takes part in the
  // block's two barriers (wave-uniform)
  const bool has = k < ucnt[rw];
  int ng = 0;
  if (has) {
    const int2 un = units[slot];
    for (int wd = un.x >> 5; wd <= (un.y - 1) >> 5; ++wd) {
      uint32_t bits = mask[rw * nwd + wd];
      while (bits) {
        const int g = wd * 32 + __builtin_ctz(bits);
        bits &= bits - 1;
        if (g < un.x || g >= un.y) continue;
        if (lane == 0) glist[wv][ng] = g;
        ++ng;
      }
    }
  }
  __syncthreads();
  // stage the unit's columns: every load in flight at once, then LDS
  constexpr int NR = kWfUnitGroups * 16 / 64;
  V4 rec[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int k = r * 64 + lane;
    V4 q;
    q.x = q.y = q.z = T(0);
    q.w = Num<T>::ninf();
    if (k < ng * 16) {
      const int64_t col = (int64_t)glist[wv][k >> 4] * 16 + (k & 15);
      if (col < Mc) {
        q.x = yc[col];
        if (DIM > 1) q.y = yc[Mc + col];
        if (DIM > 2) q.z = yc[2 * Mc + col];
        q.w = w[col];
      }
    }
    rec[r] = q;
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r * 64 + lane < ng * 16) cols[wv][r * 64 + lane] = rec[r];
  __syncthreads();
  if (!has) return;
  const T ewf = T(2.0 / eps_of(c, side));
  const int64_t i = rw * 64 + lane < Nr ? rw * 64 + lane : Nr - 1;
  T xi[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int d = 0; d < DIM; ++d) xi[d] = xr[d * Nr + i];
  Lse2<T> acc;
  acc.init();
  for (int g = 0; g < ng; ++g) {
    T t[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const V4 q = cols[wv][g * 16 + j];
      T d2 = (xi[0] - q.x) * (xi[0] - q.x);
      if (DIM > 1) d2 = Num<T>::fma(xi[1] - q.y, xi[1] - q.y, d2);
      if (DIM > 2) d2 = Num<T>::fma(xi[2] - q.z, xi[2] - q.z, d2);
      t[j] = q.w + wf_log2k<T>(d2, a2, cut2, ewf);
    }
    acc.template add<16>(t);
  }
  pm[slot * 64 + lane] = acc.m;
  ps[slot * 64 + lane] = acc.s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_wf_epi(const T* __restrict__ pm, const T* __restrict__ ps,
                                                    const int* __restrict__ ucnt, int64_t Nr, int side,
                                                    const Ctrl* __restrict__ c, EpiArgs<T> ep) {
  if (skip_side(c, side)) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  ResAcc<T> ra;
  ra.init();
  if (i < Nr) {
    // the units of the row's wave (unit k at slot k nrw + rw, row i at lane
    // i % 64); a row with no unit, or no term within the cut, gets -inf
    const int64_t rw = i / 64, nrw = (Nr + 63) / 64;
    epi_elem<T>(i, merge_parts<T>(pm, ps, 64 * nrw, rw * 64 + i % 64, ucnt[rw]), c, side, ep, ra);
  }
  epi_finish<T>(ep, ra, blockIdx.x);
}

template <typename T>
void launch_wf_lists(const T* rows, int64_t Nr, const T* cols, int64_t Mc, int dim, double cut, const WfLists<T>& L,
                     hipStream_t s) {
  const int64_t nrw = (Nr + 63) / 64, ngr = (Mc + 15) / 16;
  const int nwd = (int)((ngr + 31) / 32);
  launch_chunk_boxes<T>(rows, Nr, 64, dim, L.rbox, s);
  launch_chunk_boxes<T>(cols, Mc, 16, dim, L.gbox, s);
  hipLaunchKernelGGL(k_wf_mask<T>, dim3(ceil_div(nrw * nwd, kBlock)), dim3(kBlock), 0, s, L.rbox, nrw, L.gbox, ngr,
                     nwd, dim, T(cut * cut), L.mask);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, L.umax);
  hipLaunchKernelGGL(k_wf_units, dim3(ceil_div(nrw, kBlock)), dim3(kBlock), 0, s, L.mask, nrw, nwd, L.units, L.ucnt,
                     L.umax);
}

template <typename T>
void launch_wf_lse(int dim, const T* xr, int64_t Nr, const T* yc, const T* w, int64_t Mc, double cut,
                   const WfLists<T>& L, int umax, T* pm, T* ps, int side, const Ctrl* c, hipStream_t s) {
  const int64_t nrw = (Nr + 63) / 64, ngr = (Mc + 15) / 16;
  const int nwd = (int)((ngr + 31) / 32);
  // the slots of the first umax units of every row wave (unit-major): the
  // rest are empty
  if (umax < 1) umax = 1;
  const dim3 grid(ceil_div(nrw * umax, kBlock / 64));
  const T a2 = T(0.25 * M_PI * M_PI / (cut * cut)), cut2 = T(cut * cut);
#define UOT_WF(D)                                                                                                 \
  hipLaunchKernelGGL((k_wf_lse<T, D>), grid, dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, L.mask, L.units, L.ucnt, nwd, \
                     pm, ps, side, c, a2, cut2)
  if (dim == 1) UOT_WF(1);
  else if (dim == 2) UOT_WF(2);
  else UOT_WF(3);
#undef UOT_WF
}

template <typename T>
void launch_wf_epi(const T* pm, const T* ps, const WfLists<T>& L, int64_t Nr, int64_t Mc, int side, const Ctrl* c,
                   const EpiArgs<T>& ep, hipStream_t s) {
  (void)Mc;
  hipLaunchKernelGGL(k_wf_epi<T>, dim3(ceil_div(Nr, kBlock)), dim3(kBlock), 0, s, pm, ps, L.ucnt, Nr, side, c, ep);
}

template <typename T>
void launch_dense_lse(int dim, int R, const T* xr, int64_t Nr, const T* yc, const T* w, int64_t Mc, int nsplit,
                      int64_t cps, T* pm, T* ps, int side, const Ctrl* c, const CostArgs& cost, hipStream_t s) {
#define UOT_DL(D, RR) launch_dense_lse_t<T, D, RR>(xr, Nr, yc, w, Mc, nsplit, cps, pm, ps, side, c, cost, s)
  if (R == 1) {
    if (dim == 1) UOT_DL(1, 1); else if (dim == 2) UOT_DL(2, 1); else UOT_DL(3, 1);
  } else if (R == 2) {
    if (dim == 1) UOT_DL(1, 2); else if (dim == 2) UOT_DL(2, 2); else UOT_DL(3, 2);
  } else {
    if (dim == 1) UOT_DL(1, 4); else if (dim == 2) UOT_DL(2, 4); else UOT_DL(3, 4);
  }
#undef UOT_DL
}

template <typename T>
void launch_dense_epi(const T* pm, const T* ps, int nsplit, int64_t Nr, int side, const Ctrl* c,
                      const EpiArgs<T>& ep, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_epi<T>, dim3(ceil_div(Nr, kBlock)), dim3(kBlock), 0, s, pm, ps, nsplit, Nr, side, c, ep);
}

void launch_control(Ctrl* c, const ResPart* part, int nparts, double* hist, hipStream_t s, int nfields, int par) {
  hipLaunchKernelGGL(k_control, dim3(1), dim3(kBlock), 0, s, c, part, nparts, hist, nfields, par);
}

void launch_res_reduce(const ResPart* part, int nparts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_res_reduce, dim3(1), dim3(64), 0, s, part, nparts, out);
}

void launch_ctrl_resume(Ctrl* c, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_resume, dim3(1), dim3(64), 0, s, c, tol);
}

void launch_ctrl_post(Ctrl* c, hipStream_t s) { hipLaunchKernelGGL(k_ctrl_post, dim3(1), dim3(64), 0, s, c); }

template <typename T>
void launch_growth_combine(const T* T2, int nm, int64_t size, const DivDev& F, const T* logq, const T* logdy, T* v,
                           T* w, const Ctrl* c, int side, hipStream_t s) {
  hipLaunchKernelGGL(k_growth_combine<T>, dim3(ceil_div(size, kBlock)), dim3(kBlock), 0, s, T2, nm, size, F, logq,
                     logdy, v, w, c, side);
}
template void launch_growth_combine<float>(const float*, int, int64_t, const DivDev&, const float*, const float*,
                                           float*, float*, const Ctrl*, int, hipStream_t);
template void launch_growth_combine<double>(const double*, int, int64_t, const DivDev&, const double*,
                                            const double*, double*, double*, const Ctrl*, int, hipStream_t);

template <typename T>
void launch_flow_next(const T* T2, const T* v, const T* logq, int nm, int64_t size, int growth, double log_kappa,
                      const Ctrl* c, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_flow_next<T>, dim3(ceil_div(size, kBlock)), dim3(kBlock), 0, s, T2, v, logq, nm, size, growth,
                     log_kappa, c, out);
}
template void launch_flow_next<float>(const float*, const float*, const float*, int, int64_t, int, double,
                                      const Ctrl*, float*, hipStream_t);
template void launch_flow_next<double>(const double*, const double*, const double*, int, int64_t, int, double,
                                       const Ctrl*, double*, hipStream_t);

template <typename T>
void launch_mass_update(Ctrl* c, const T* mass_m, const T* mass_s, int nparts, const DivDev& F3, double log_m0, int par,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_mass_update<T>, dim3(1), dim3(kBlock), 0, s, c, mass_m, mass_s, nparts, F3, log_m0, par);
}
template void launch_mass_update<float>(Ctrl*, const float*, const float*, int, const DivDev&, double, int, hipStream_t);
template void launch_mass_update<double>(Ctrl*, const double*, const double*, int, const DivDev&, double, int,
                                         hipStream_t);

void launch_ctrl_init(Ctrl* c, const Ctrl& init, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, s, c, init);
}

template <typename T>
void launch_bary_combine(const T* T2, int nm, int64_t size, const BaryW& log_alpha, double log_sum_alpha,
                         const DivDev& F2, const T* logdy, T* v, T* w, T* logh, const Ctrl* c, int side,
                         hipStream_t s) {
  if (F2.kind == 2 || F2.kind == 3) {
    const int nbp = nm * ((F2.kind == 2 || F2.has_lo) ? 2 : 1);
    int L = 2;
    while (L < nbp && L < 64) L *= 2;
    const unsigned blocks = ceil_div(size * L, kBlock);
#define UOT_BR(LL)                                                                                               \
  hipLaunchKernelGGL((k_bary_root<T, LL>), dim3(blocks), dim3(kBlock), 0, s, T2, nm, size, log_alpha, F2, logdy, v, w, \
                     logh, c, side)
    switch (L) {
      case 2: UOT_BR(2); break;
      case 4: UOT_BR(4); break;
      case 8: UOT_BR(8); break;
      case 16: UOT_BR(16); break;
      case 32: UOT_BR(32); break;
      default: UOT_BR(64); break;
    }
#undef UOT_BR
    return;
  }
  hipLaunchKernelGGL(k_bary_combine<T>, dim3(ceil_div(size, kBlock)), dim3(kBlock), 0, s, T2, nm, size, log_alpha,
                     log_sum_alpha, F2, logdy, v, w, logh, c, side);
}

template <typename T>
int launch_obj_side(const T* pot, const T* S, const T* p, const T* d, int64_t n, double eps, const DivDev& F,
                    T* pi_out, double* part, hipStream_t s) {
  const unsigned nb = ceil_div(n, kBlock);
  hipLaunchKernelGGL(k_obj_side<T>, dim3(nb), dim3(kBlock), 0, s, pot, S, p, d, n, eps, F, pi_out, part);
  return (int)nb;
}

template <typename T>
int launch_sum_exp2(const T* a, const T* b, int64_t n, double* part, hipStream_t s) {
  const unsigned nb = ceil_div(n, kBlock);
  hipLaunchKernelGGL(k_sum_exp2<T>, dim3(nb), dim3(kBlock), 0, s, a, b, n, part);
  return (int)nb;
}

template <typename T>
void launch_dense_cost(int dim, const T* xr, int64_t Nr, const T* yc, const T* w, int64_t Mc, double eps, T* out,
                       const CostArgs& cost, hipStream_t s) {
  dim3 grid(ceil_div(Nr, kBlock));
  if (dim == 1) hipLaunchKernelGGL((k_dense_cost<T, 1>), grid, dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, eps, out, cost);
  else if (dim == 2)
    hipLaunchKernelGGL((k_dense_cost<T, 2>), grid, dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, eps, out, cost);
  else hipLaunchKernelGGL((k_dense_cost<T, 3>), grid, dim3(kBlock), 0, s, xr, Nr, yc, w, Mc, eps, out, cost);
}

#define UOT_INSTANTIATE(T)                                                                                         \
  template void launch_log<T>(const T*, T*, int64_t, int, hipStream_t);                                           \
  template void launch_init_pot<T>(const T*, const T*, T*, T*, int64_t, int64_t, const Ctrl*, int, hipStream_t);  \
  template void launch_gtab<T>(T*, int, double, const Ctrl*, int, const CostArgs&, hipStream_t);                  \
  template void launch_gtab_cost<T>(T*, int, double, double, const CostArgs&, hipStream_t);                       \
  template int grid_strided_parts<T>(int, int64_t, int64_t);                                                      \
  template int grid_contig_parts<T>(int, int64_t);                                                                \
  template void launch_grid_strided<T>(const T*, int64_t, int, int64_t, const T*, int, const Ctrl*,              \
                                       const EpiArgs<T>&, hipStream_t);                                          \
  template void launch_grid_contig<T>(const T*, int64_t, int, const T*, int, const Ctrl*, const EpiArgs<T>&,     \
                                      int, hipStream_t);                                                          \
  template void launch_grid_contig_split<T>(const T*, int64_t, int, const T*, int, const Ctrl*, int, int, T*, T*, \
                                            hipStream_t);                                                         \
  template void launch_dense_lse<T>(int, int, const T*, int64_t, const T*, const T*, int64_t, int, int64_t, T*,  \
                                    T*, int, const Ctrl*, const CostArgs&, hipStream_t);                          \
  template void launch_chunk_boxes<T>(const T*, int64_t, int64_t, int, T*, hipStream_t);                        \
  template void launch_wf_lists<T>(const T*, int64_t, const T*, int64_t, int, double, const WfLists<T>&,          \
                                   hipStream_t);                                                                  \
  template void launch_wf_lse<T>(int, const T*, int64_t, const T*, const T*, int64_t, double, const WfLists<T>&, \
                                 int, T*, T*, int, const Ctrl*, hipStream_t);                                     \
  template void launch_wf_epi<T>(const T*, const T*, const WfLists<T>&, int64_t, int64_t, int, const Ctrl*,      \
                                 const EpiArgs<T>&, hipStream_t);                                                 \
  template void launch_dense_epi<T>(const T*, const T*, int, int64_t, int, const Ctrl*, const EpiArgs<T>&,       \
                                    hipStream_t);                                                                 \
  template void launch_bary_combine<T>(const T*, int, int64_t, const BaryW&, double, const DivDev&, const T*,    \
                                       T*, T*, T*, const Ctrl*, int, hipStream_t);                               \
  template int launch_obj_side<T>(const T*, const T*, const T*, const T*, int64_t, double, const DivDev&, T*,    \
                                  double*, hipStream_t);                                                          \
  template int launch_sum_exp2<T>(const T*, const T*, int64_t, double*, hipStream_t);                            \
  template void launch_dense_cost<T>(int, const T*, int64_t, const T*, const T*, int64_t, double, T*,             \
                                     const CostArgs&, hipStream_t);

UOT_INSTANTIATE(float)
UOT_INSTANTIATE(double)

}  // namespace uot

// ---------------------------------------------------------------------------
// throughput probes for the roofline of the log-sum-exp passes: 8 independent
// dependency chains per lane of v_exp_f32 (x <- 2^-x stays in [0.5, 1]) or of
// v_add_f32; each lane writes its sum so nothing is optimised away.
// ---------------------------------------------------------------------------
namespace uot {

__global__ __launch_bounds__(kBlock) void k_probe_exp(float* __restrict__ out, int iters) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 0.01f * (threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_exp2f(-x[k]);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_probe_add(float* __restrict__ out, int iters, float c) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 0.01f * (threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = x[k] + c;
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

void launch_probe(int which, float* out, int blocks, int iters, hipStream_t s) {
  if (which == 0) hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(kBlock), 0, s, out, iters);
  else hipLaunchKernelGGL(k_probe_add, dim3(blocks), dim3(kBlock), 0, s, out, iters, 1e-7f);
}

}  // namespace uot

// ---------------------------------------------------------------------------
// ragged batches of independent point-cloud problems.  One persistent launch
// per half-step over the item list (problem, row tile), *count items long:
// each block pulls items from an atomic cursor until the list is exhausted
// (a greedy list schedule: along a list that runs from the costliest items
// down, the blocks finish within about one small item of each other).
// Items of problems that stopped since the list was built are skipped.
// ---------------------------------------------------------------------------
namespace uot {

template <typename T, int DIM, int R>
__global__ __launch_bounds__(kBlock) void k_batch_lse(const BItem* __restrict__ items, const int* __restrict__ count,
                                                       int* __restrict__ cursor, const int64_t* __restrict__ offR,
                                                       const int64_t* __restrict__ offC, const T* __restrict__ xr,
                                                       int64_t totR, const T* __restrict__ yc, int64_t totC,
                                                       const T* __restrict__ w, const BCtrl* __restrict__ bc,
                                                       const Ctrl* __restrict__ c, int side, EpiArgs<T> ep) {
  using V4 = typename Vec4<T>::type;
  __shared__ V4 tile[kBlock];
  __shared__ int item_sh;
  const T sc = T(kLog2e / eps_of(c, side));
  const int n_items = *count;
  const int32_t* __restrict__ skip = half_of(side) == 0 ? bc->stop : bc->yskip;
  while (true) {
    __syncthreads();   // the previous item's reads of the tile and item_sh are done
    if (threadIdx.x == 0) item_sh = atomicAdd(cursor, 1);
    __syncthreads();
    const int it = item_sh;
    if (it >= n_items) break;
    const BItem I = items[it];
    if (skip[I.prob]) continue;
    const int64_t rb = offR[I.prob];
    const int64_t cb = offC[I.prob], ce = offC[I.prob + 1];
    T xi[R][DIM];
    bool vr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int lr = I.row0 + r * kBlock + threadIdx.x;
      vr[r] = lr < I.row0 + I.nrows;
      const int64_t g = rb + (vr[r] ? lr : I.row0);
#pragma unroll
      for (int d = 0; d < DIM; ++d) xi[r][d] = xr[d * totR + g];
    }
    Lse2<T> acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r].init();
    for (int64_t c0 = cb; c0 < ce; c0 += kBlock) {
      const int64_t cc = c0 + threadIdx.x;
      V4 rec;
      rec.x = rec.y = rec.z = T(0);
      if (cc < ce) {
        rec.x = yc[cc];
        if (DIM > 1) rec.y = yc[totC + cc];
        if (DIM > 2) rec.z = yc[2 * totC + cc];
        rec.w = w[cc];
      } else {
        rec.w = Num<T>::ninf();
      }
      __syncthreads();
      tile[threadIdx.x] = rec;
      __syncthreads();
      const int64_t rem = ce - c0;
      const int cnt = rem < kBlock ? (int)rem : kBlock;
      for (int jj = 0; jj < cnt; jj += kChunk) {
        V4 q[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) q[k] = tile[jj + k];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          T t[kChunk];
#pragma unroll
          for (int k = 0; k < kChunk; ++k) {
            T d0 = xi[r][0] - q[k].x;
            T cst = d0 * d0;
            if (DIM > 1) { T d1 = xi[r][1] - q[k].y; cst = Num<T>::fma(d1, d1, cst); }
            if (DIM > 2) { T d2 = xi[r][2] - q[k].z; cst = Num<T>::fma(d2, d2, cst); }
            t[k] = Num<T>::fma(-sc, cst, q[k].w);
          }
          acc[r].template add<kChunk>(t);
        }
      }
    }
    ResAcc<T> ra;
    ra.init();
    const bool bal = bal_on<T>(ep, c);   // (block-uniform)
    MassAcc<T> mb;
    mb.init();
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (vr[r]) {
        const int64_t e = rb + I.row0 + r * kBlock + threadIdx.x;
        const T S2 = acc[r].result();
        epi_elem<T>(e, S2, c, side, ep, ra);
        if (bal) bal_elem<T>(e, S2, c, side, ep, mb);
      }
    epi_finish<T>(ep, ra, I.part);
    if (bal) block_lse_reduce<T>(mb.m, mb.s, ep.bal_m + I.part, ep.bal_s + I.part);
  }
}

// log2 of the sum of the partials (m, s)[k0 .. k1) over a wave, in FP64:
// lane-strided merge, then a butterfly over the 64 lanes (every lane gets it)
template <typename T>
__device__ __forceinline__ double wave_lse_parts(const T* __restrict__ pm, const T* __restrict__ ps, int k0, int k1,
                                                 int lane) {
  double m = -__builtin_inf(), s = 0.0;
  for (int k = k0 + lane; k < k1; k += 64) {
    const double m2 = double(pm[k]), s2 = double(ps[k]);
    const double mn = fmax(m, m2);
    if (mn == -__builtin_inf()) continue;
    s = s * exp2(m - mn) + s2 * exp2(m2 - mn);
    m = mn;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double m2 = __shfl_xor(m, o), s2 = __shfl_xor(s, o);
    const double mn = fmax(m, m2);
    if (mn != -__builtin_inf()) {
      s = s * exp2(m - mn) + s2 * exp2(m2 - mn);
      m = mn;
    }
  }
  return m + log2(s);
}

// per-problem control between the X and Y half-steps, one wave per problem:
// the residual of the X half-step from the problem's partials (Sec. 4.4's
// stopping rule on the X marginal), its iteration count, and the stop
// decision; a stopped problem leaves the item lists at the next compaction
template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_control(Ctrl* __restrict__ c, BCtrl* __restrict__ bc, int B,
                                                           const ResPart* __restrict__ part,
                                                           const int32_t* __restrict__ pstart, int par,
                                                           BatchBalance<T> bal) {
  const int lane = threadIdx.x & 63;
  const int64_t b = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;   // uniform over the wave
  if (b >= B) return;
  if (bc->stop[b]) {
    if (lane == 0) bc->yskip[b] = 1;
    return;
  }
  float m = -__builtin_inff(), den = 0.f, num = 0.f, du = 0.f;
  for (int k = pstart[b] + lane; k < pstart[b + 1]; k += 64) res_merge<float>(m, den, num, part[k].m, part[k].den, part[k].num);
  wave_res_reduce(m, den, num, du);
  // (every lane holds the totals and takes the same decision; lane 0 writes)
  const double r = res_ratio(double(num), double(den));
  const int64_t l = bc->iters[b];
  const bool final_stage = c->iters_per_stage <= 0 || l >= (int64_t)c->n_stages * c->iters_per_stage;
  int stop = 0, status = 1;
  if (r != r) { stop = 1; status = -3; }
  else if (final_stage && r <= c->tol && l >= 1) { stop = 1; status = 0; }
  else if (l + 1 >= c->max_iter) { stop = 1; status = 1; }
  if (lane == 0) {
    bc->res[b] = r;
    bc->iters[b] = l + 1;
    if (stop) {
      bc->status[b] = status;
      bc->stop[b] = 1;
      bc->clock[b] = wall_clock64();
      atomicAdd(&c->nstop, 1);   // a few problems per iteration
    }
  }
  if (stop || bal.pxm == nullptr || c->iter != bal.iter) return;
  // the in-solve mass balance: P from this X half-step's items, Q from the
  // previous Y half-step's (log2 sums, merged in FP64)
  const double lP = wave_lse_parts<T>(bal.pxm, bal.pxs, pstart[b], pstart[b + 1], lane);
  const double lQ = wave_lse_parts<T>(bal.pym, bal.pys, bal.pstartY[b], bal.pstartY[b + 1], lane);
  if (!(__builtin_isfinite(lP) && __builtin_isfinite(lQ))) return;
  const double eps = c->eps[par];
  const double th1 = double(bal.lam1) / (double(bal.lam1) + eps);
  const double sh = (lP - lQ) * kLn2 / (th1 / double(bal.lam1) + 1.0 / double(bal.lam2));
  const T du_ = T(th1 * sh), dw = T(th1 * sh / eps * kLog2e);
  for (int64_t i = bal.offN[b] + lane; i < bal.offN[b + 1]; i += 64) {
    bal.pot[i] += du_;
    bal.w[i] += dw;
  }
}

// After the control step of the iteration of parity par (advance = 1), or
// at the start of a solve (advance = 0, every problem listed): reset the
// work cursors, and rebuild both item lists (block 0: rows X, block 1: rows
// Y) when at least 1/16 of the problems listed at the last rebuild have
// stopped since, keeping each side's problem order (an exclusive scan of the
// listed problems' item counts gives each problem its first position).  The
// X list (next iteration) holds the problems not stopped, the Y list (this
// iteration) also those that stopped in this iteration's control step
// (yskip).  With advance, block 0 also records the number of active problems
// for the host and does the global eps bookkeeping.
constexpr int kCompactBlock = 1024;
constexpr int kCompactPer = 4;   // problems per thread and pass
__global__ __launch_bounds__(kCompactBlock) void k_batch_compact(Ctrl* __restrict__ c, const BCtrl* __restrict__ bc,
                                                                 int B, BatchLists L, int par, int advance) {
  const int side = blockIdx.x;
  // (both blocks read the same counters; only the slot par ^ 1 is written)
  const int nstop = c->nstop, built = c->built[par];
  const bool rebuild = !advance || (nstop > built && (int64_t)(nstop - built) * 16 >= (int64_t)(B - built));
  if (threadIdx.x == 0) {
    *L.cursor[side] = 0;
    if (side == 0 && advance) {
      const int64_t l = c->iter;
      c->active[l & 1] = B - nstop;
      c->built[par ^ 1] = rebuild ? nstop : built;
      c->iter = l + 1;
      int64_t sn = c->iters_per_stage > 0 ? (l + 1) / c->iters_per_stage : c->n_stages;
      if (sn > c->n_stages) sn = c->n_stages;
      c->stage[par ^ 1] = (int)sn;
      c->eps[par ^ 1] = c->eps_tab[sn];
    }
  }
  if (!rebuild) return;
  const int32_t* __restrict__ ord = L.ord[side];
  const int64_t* __restrict__ off = L.off[side];
  const int32_t* __restrict__ stop = side == 0 ? bc->stop : bc->yskip;
  BItem* __restrict__ out = L.items[side];
  constexpr int kWaves = kCompactBlock / 64;
  __shared__ int wtot[kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t carry = 0;
  for (int64_t base = 0; base < B; base += (int64_t)kCompactBlock * kCompactPer) {
    int prob[kCompactPer], cnt[kCompactPer];
    int64_t nrow[kCompactPer];
    int mine = 0;
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) {
      const int64_t k = base + (int64_t)threadIdx.x * kCompactPer + j;
      prob[j] = 0;
      cnt[j] = 0;
      nrow[j] = 0;
      if (k < B) {
        const int b = ord[k];
        prob[j] = b;
        if (!stop[b]) {
          nrow[j] = off[b + 1] - off[b];
          cnt[j] = (int)((nrow[j] + L.rows - 1) / L.rows);
        }
      }
      mine += cnt[j];
    }
    // inclusive scan of the item counts over the wave, then over the waves
    int incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      before += w < wv ? wtot[w] : 0;
      total += wtot[w];
    }
    int64_t p = carry + before + incl - mine;
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j)
      for (int q = 0; q < cnt[j]; ++q) {
        BItem it;
        it.prob = prob[j];
        it.row0 = q * L.rows;
        it.nrows = (int)(nrow[j] - it.row0 < L.rows ? nrow[j] - it.row0 : L.rows);
        it.part = (side == 0 ? L.pstart[prob[j]] : L.pstartY[prob[j]]) + q;
        out[p++] = it;
      }
    carry += total;
    __syncthreads();   // wtot is rewritten by the next pass
  }
  if (threadIdx.x == 0) *L.count[side] = (int)carry;
}

// column weights of the X half-step's product from a starting potential:
// w_j = v0_j / eps + log dy_j (natural log)
__global__ void k_balance_w(const float* __restrict__ v0, const float* __restrict__ dy, int64_t n, float inv_eps,
                            float* __restrict__ w) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < n) w[j] = v0[j] * inv_eps + logf(dy[j]);
}

// Mass balance of a starting potential v0 (KL on both marginals), one block
// per problem.  S: log K(e^{v0/eps} dy) at every X point (natural log, from
// the batch Gibbs product).  u1 = theta1 eps (log p - S) is the X half-step
// from v0 (Table proximalexplicit, KL row); P = sum p e^{-u1/lam1} dx is the
// mass of the plan's first marginal after it, Q = sum q e^{-v0/lam2} dy the
// mass v0 gives the second; s = log(P/Q) / (theta1/lam1 + 1/lam2) makes them
// agree once v0 is replaced by v0 - s (u1 then moves by theta1 s).  Points
// of zero density carry no mass; s = 0 when P or Q is 0.
__global__ __launch_bounds__(kBlock) void k_batch_balance(const float* __restrict__ S, const float* __restrict__ p,
                                                           const float* __restrict__ dx,
                                                           const int64_t* __restrict__ offN,
                                                           const float* __restrict__ q, const float* __restrict__ dy,
                                                           const int64_t* __restrict__ offM, float th1_eps,
                                                           float inv_lam1, float inv_lam2, float inv_denom,
                                                           float* __restrict__ v0, float* __restrict__ shift) {
  const int64_t b = blockIdx.x;
  __shared__ float lm[2], ls[2];
  Lse2<float> a, c;
  a.init();
  c.init();
  for (int64_t i = offN[b] + threadIdx.x; i < offN[b + 1]; i += kBlock) {
    const float pi = p[i];
    if (pi > 0.f) {
      const float lp = logf(pi);
      const float u1 = th1_eps * (lp - S[i]);
      const float t = float(kLog2e) * (lp - u1 * inv_lam1 + logf(dx[i]));
      a.add<1>(&t);
    }
  }
  for (int64_t j = offM[b] + threadIdx.x; j < offM[b + 1]; j += kBlock) {
    const float qj = q[j];
    if (qj > 0.f) {
      const float t = float(kLog2e) * (logf(qj) - v0[j] * inv_lam2 + logf(dy[j]));
      c.add<1>(&t);
    }
  }
  block_lse_reduce<float>(a.m, a.s, &lm[0], &ls[0]);
  block_lse_reduce<float>(c.m, c.s, &lm[1], &ls[1]);
  __syncthreads();   // (also: every thread's reads of v0 are done)
  const float lP = lm[0] + log2f(ls[0]), lQ = lm[1] + log2f(ls[1]);
  float sh = (lP - lQ) * float(kLn2) * inv_denom;
  if (!(lP > -__builtin_inff() && lQ > -__builtin_inff()) || sh != sh) sh = 0.f;
  for (int64_t j = offM[b] + threadIdx.x; j < offM[b + 1]; j += kBlock) v0[j] -= sh;
  if (shift && threadIdx.x == 0) shift[b] = sh;
}

__global__ void k_batch_init(BCtrl* __restrict__ bc, int B, Ctrl* __restrict__ c) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) {
    c->t0_clock = wall_clock64();
    c->active[0] = c->active[1] = B;
  }
  if (b >= B) return;
  bc->stop[b] = 0;
  bc->yskip[b] = 0;
  bc->iters[b] = 0;
  bc->status[b] = 1;
  bc->res[b] = __builtin_inf();
  bc->clock[b] = 0;
}

__global__ void k_set_int(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
void launch_batch_lse(int dim, int R, int blocks, const BItem* items, const int* count, int* cursor,
                      const int64_t* offR, const int64_t* offC, const T* xr, int64_t totR, const T* yc, int64_t totC,
                      const T* w, const BCtrl* bc, const Ctrl* c, int side, const EpiArgs<T>& ep, hipStream_t s) {
#define UOT_BL(D, RR)                                                                                          \
  hipLaunchKernelGGL((k_batch_lse<T, D, RR>), dim3(blocks), dim3(kBlock), 0, s, items, count, cursor, offR, offC, \
                     xr, totR, yc, totC, w, bc, c, side, ep)
  if (R == 1) {
    if (dim == 1) UOT_BL(1, 1); else if (dim == 2) UOT_BL(2, 1); else UOT_BL(3, 1);
  } else if (R == 2) {
    if (dim == 1) UOT_BL(1, 2); else if (dim == 2) UOT_BL(2, 2); else UOT_BL(3, 2);
  } else {
    if (dim == 1) UOT_BL(1, 4); else if (dim == 2) UOT_BL(2, 4); else UOT_BL(3, 4);
  }
#undef UOT_BL
}

template <typename T>
void launch_batch_control(Ctrl* c, BCtrl* bc, int B, const ResPart* part, const int32_t* pstart,
                          const BatchLists& L, int par, const BatchBalance<T>& bal, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_control<T>, dim3((unsigned)ceil_div((int64_t)B * 64, kBlock)), dim3(kBlock), 0, s, c, bc,
                     B, part, pstart, par, bal);
  hipLaunchKernelGGL(k_batch_compact, dim3(2), dim3(kCompactBlock), 0, s, c, bc, B, L, par, 1);
}
template void launch_batch_control<float>(Ctrl*, BCtrl*, int, const ResPart*, const int32_t*, const BatchLists&, int,
                                          const BatchBalance<float>&, hipStream_t);
template void launch_batch_control<double>(Ctrl*, BCtrl*, int, const ResPart*, const int32_t*, const BatchLists&,
                                           int, const BatchBalance<double>&, hipStream_t);

void launch_batch_compact(Ctrl* c, const BCtrl* bc, int B, const BatchLists& L, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_compact, dim3(2), dim3(kCompactBlock), 0, s, c, bc, B, L, 0, 0);
}

void launch_balance_w(const float* v0, const float* dy, int64_t n, double eps, float* w, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_balance_w, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, v0, dy, n, float(1.0 / eps), w);
}

void launch_batch_balance(const float* S, const float* p, const float* dx, const int64_t* offN, const float* q,
                          const float* dy, const int64_t* offM, int64_t B, double eps, double lam1, double lam2,
                          float* v0, float* shift, hipStream_t s) {
  const double th1 = lam1 / (lam1 + eps);
  hipLaunchKernelGGL(k_batch_balance, dim3((unsigned)B), dim3(kBlock), 0, s, S, p, dx, offN, q, dy, offM,
                     float(th1 * eps), float(1.0 / lam1), float(1.0 / lam2), float(1.0 / (th1 / lam1 + 1.0 / lam2)),
                     v0, shift);
}

void launch_batch_init(BCtrl* bc, int B, Ctrl* c, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_init, dim3(ceil_div(B, kBlock)), dim3(kBlock), 0, s, bc, B, c);
}

void launch_set_int(int* p, int n, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, p, n, v);
}

template <typename T>
__global__ void k_scale(T* __restrict__ a, int64_t n, T f) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] *= f;
}

template <typename T> void launch_scale(T* a, int64_t n, double f, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale<T>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, a, n, T(f));
}
template void launch_scale<float>(float*, int64_t, double, hipStream_t);
template void launch_scale<double>(double*, int64_t, double, hipStream_t);

template void launch_batch_lse<float>(int, int, int, const BItem*, const int*, int*, const int64_t*, const int64_t*,
                                      const float*, int64_t, const float*, int64_t, const float*, const BCtrl*,
                                      const Ctrl*, int, const EpiArgs<float>&, hipStream_t);
template void launch_batch_lse<double>(int, int, int, const BItem*, const int*, int*, const int64_t*,
                                       const int64_t*, const double*, int64_t, const double*, int64_t, const double*,
                                       const BCtrl*, const Ctrl*, int, const EpiArgs<double>&, hipStream_t);

}  // namespace uot
