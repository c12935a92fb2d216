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
#include <cstdlib>

#include "uot_device.h"
#include "uot_launch.h"

namespace uot {

constexpr int kBlock = 256;
constexpr int kChunk = 8;       // terms per online-max rescale
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

// ---------------------------------------------------------------------------
// epilogue shared by every Gibbs product.  epi_elem handles one element with
// S2 = log2 of the product; epi_finish reduces the residual partials of the
// block (every thread of the block must call it).
// ---------------------------------------------------------------------------
template <typename T> struct ResAcc {
  T m, den, num;
  __device__ __forceinline__ void init() {
    m = Num<T>::ninf();
    den = T(0);
    num = T(0);
  }
  __device__ __forceinline__ void add(T m2, T d2, T n2) { res_merge<T>(m, den, num, m2, d2, n2); }
};

// operands of one element's epilogue, loadable ahead of the product
template <typename T> struct EpiIn {
  T ld, uo, lp;
};

template <typename T>
__device__ __forceinline__ EpiIn<T> epi_load(int64_t e, const EpiArgs<T>& ep) {
  EpiIn<T> x;
  if (ep.mode == EPI_RAW) {
    x.ld = x.uo = x.lp = T(0);
    return x;
  }
  x.ld = ep.logd[e < ep.size ? e : e % ep.size];
  x.uo = ep.pot[e];
  x.lp = ep.logp[e];
  return x;
}

template <typename T>
__device__ __forceinline__ void epi_apply(int64_t e, T S2, const EpiIn<T>& x, const Ctrl* __restrict__ c, int side,
                                          const EpiArgs<T>& ep, ResAcc<T>& ra) {
  if (ep.mode == EPI_RAW) {
    ep.out[e] = S2;
    return;
  }
  const T eps = T(eps_of(c, side));
  const T eps_w = T(eps_next_of(c, side));   // w feeds the next half-step
  const T Sraw = S2 * T(kLn2);
  const T S = Sraw + T(c->zeta);              // z K(.): log z of a total-mass penalty, else 0
  const T ld = x.ld;
  const T uo = x.uo;
  const T un = proxdiv_pot<T>(ep.F, x.lp, S, eps);
  // a vanishing product (K b = 0 here, possible with exact zeros of K): the
  // row of the plan is zero whatever the potential, so the point carries no
  // marginal mass and enters the next product as -inf
  const bool vanish = Sraw == Num<T>::ninf();
  ep.pot[e] = un;
  if (ep.wnext) ep.wnext[e] = vanish ? Num<T>::ninf() : (un / eps_w + ld) * T(kLog2e);
  if (ep.lse_out) ep.lse_out[e] = S;
  if (vanish) return;
  if (ep.part) {
    if (un == Num<T>::ninf()) {
      if (uo != Num<T>::ninf()) ra.add((S + uo / eps + ld) * T(kLog2e), T(0), T(1));
    } else {
      const T d = Num<T>::expm1((uo - un) / eps);
      ra.add((S + un / eps + ld) * T(kLog2e), T(1), Num<T>::fmax(d, -d));
    }
  } else if (ep.mass_m) {
    // mass of the plan without z: the (m, den) pair of ra carries it
    ra.add((Sraw + un / eps + ld) * T(kLog2e), T(1), T(0));
  }
}

template <typename T>
__device__ __forceinline__ void epi_elem(int64_t e, T S2, const Ctrl* __restrict__ c, int side,
                                         const EpiArgs<T>& ep, ResAcc<T>& ra) {
  epi_apply<T>(e, S2, epi_load<T>(e, ep), c, side, ep, ra);
}

// log2-sum-exp (m, s) over a block in T precision (every thread calls it);
// thread 0 writes the result
template <typename T>
__device__ __forceinline__ void block_lse_reduce(T m, T s, T* out_m, T* out_s) {
  __shared__ T sm[kBlock], ss[kBlock];
  sm[threadIdx.x] = m;
  ss[threadIdx.x] = s;
  __syncthreads();
  for (int off = kBlock / 2; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) {
      Lse2<T> a;
      a.m = sm[threadIdx.x];
      a.s = ss[threadIdx.x];
      a.merge(sm[threadIdx.x + off], ss[threadIdx.x + off]);
      sm[threadIdx.x] = a.m;
      ss[threadIdx.x] = a.s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *out_m = sm[0];
    *out_s = ss[0];
  }
}

template <typename T>
__device__ __forceinline__ void epi_finish(const EpiArgs<T>& ep, const ResAcc<T>& ra, int part_index) {
  if (ep.mode == EPI_RAW) return;
  if (ep.part) block_res_reduce<T>(ra.m, ra.den, ra.num, ep.part + part_index);
  else if (ep.mass_m) block_lse_reduce<T>(ra.m, ra.den, ep.mass_m + part_index, ep.mass_s + part_index);
}

// ---------------------------------------------------------------------------
// control step of an iteration: reduce the residual partials of the X
// half-step, count the iteration, pick the next eps, stop when done.  It runs
// as its own launch (k_control) or in block 0 of the first pass of the Y
// half-step (grid solves of one problem: that pass only reads the slot of
// the current iteration, the step writes the slot of the next).
// ---------------------------------------------------------------------------
// what the control step of an iteration of parity par reads of the control
// block, loaded before the residual reduction so those loads overlap the
// loads of the partials
struct CtrlSnap {
  int64_t l, max_iter;
  int stage, n_stages, sn;
  double tol, eps_next;
};

__device__ __forceinline__ CtrlSnap ctrl_snap(const Ctrl* c, int par) {
  CtrlSnap s;
  s.l = c->iter;
  s.max_iter = c->max_iter;
  s.stage = c->stage[par];
  s.n_stages = c->n_stages;
  s.tol = c->tol;
  int64_t sn = c->iters_per_stage > 0 ? (s.l + 1) / c->iters_per_stage : s.n_stages;
  if (sn > s.n_stages) sn = s.n_stages;
  s.sn = (int)sn;
  s.eps_next = c->eps_tab[sn];
  return s;
}

// one thread: record r, count the iteration, fill the slot of the next
// iteration (parity par ^ 1) with its eps stage, stop when done.  A stopped
// solve skips the next iteration; the control step of a skipped iteration
// passes the skip on (control_skip), so every later iteration skips too.
__device__ void control_finish(Ctrl* c, const CtrlSnap& s, double r, double* __restrict__ hist, int par) {
  if (hist) hist[s.l] = r;
  c->res = r;
  c->iter = s.l + 1;
  c->stage[par ^ 1] = s.sn;
  c->eps[par ^ 1] = s.eps_next;
  const bool final_stage = s.stage >= s.n_stages;
  int status = 0;
  bool stop = false;
  if (r != r) {
    stop = true;
    status = -3;
  } else if (final_stage && r <= s.tol && s.l >= 1) {
    // (the first residual compares with the initial u and is not used to stop)
    stop = true;
    status = 0;
  } else if (s.l + 1 >= s.max_iter) {
    stop = true;
    status = 1;
  }
  if (stop) {
    c->status = status;
    c->stop = 1;
    c->skip[par ^ 1] = 1;
  }
}

__device__ __forceinline__ void control_skip(Ctrl* c, int par) { c->skip[par ^ 1] = 1; }

// this thread's share of the residual partials of one problem
__device__ __forceinline__ void ctl_load(const ResPart* __restrict__ part, int nparts, float& m, float& den,
                                         float& num) {
  m = -__builtin_inff();
  den = num = 0.f;
  for (int k = threadIdx.x; k < nparts; k += kBlock) res_merge<float>(m, den, num, part[k].m, part[k].den, part[k].num);
}

// block reduction of the shares and the control step (every thread of the
// block calls it)
__device__ __forceinline__ void ctl_reduce_finish(Ctrl* c, const CtrlSnap& snap, float m, float den, float num,
                                                  double* __restrict__ hist, int par) {
  __shared__ ResPart tot;
  __syncthreads();   // the block's own reductions before this one are complete
  block_res_reduce<float>(m, den, num, &tot);
  __syncthreads();
  if (threadIdx.x == 0) control_finish(c, snap, res_ratio(double(tot.num), double(tot.den)), hist, par);
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
// its outputs
template <typename T, int RI>
__global__ __launch_bounds__(kBlock) void k_grid_contig(const T* __restrict__ in, int n, int64_t A,
                                                         const T* __restrict__ gtab, int side,
                                                         const Ctrl* __restrict__ c, EpiArgs<T> ep, int band) {
  // block 0 of a launch that hosts the control step: partials loaded first
  const bool hosting = ep.host_ctl != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0;
  const int par = par_of(side);
  CtrlSnap hsnap{};
  float hm = -__builtin_inff(), hden = 0.f, hnum = 0.f;
  if (hosting) {
    hsnap = ctrl_snap(ep.host_ctl, par);
    ctl_load(ep.host_parts, ep.host_nparts, hm, hden, hnum);
  }
  if (skip_side(c, side)) {
    if (hosting && threadIdx.x == 0) control_skip(ep.host_ctl, par);
    return;
  }
  extern __shared__ __align__(16) unsigned char gl_raw[];
  T* gl = reinterpret_cast<T*>(gl_raw);
  const int stage = stage_of(c, side);
  const T* __restrict__ g = gtab + (int64_t)stage * (2 * n - 1);
  for (int k = threadIdx.x; k < 2 * n - 1; k += kBlock) gl[k] = g[k];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t a = (int64_t)blockIdx.z * gridDim.y + blockIdx.y;
  const bool valid_a = a < A;
  const T* __restrict__ line = in + (valid_a ? a : 0) * (int64_t)n;
  int ii[RI];
#pragma unroll
  for (int r = 0; r < RI; ++r) {
    const int i = (blockIdx.x * RI + r) * 64 + lane;
    ii[r] = (i < n ? i : n - 1) + (n - 1);          // index of g[i - 0] in the LDS table
  }
  const int o0 = blockIdx.x * RI * 64;
  const int o1 = (o0 + RI * 64 < n) ? o0 + RI * 64 : n;
  const int ta = (o0 - band + 1 > 0) ? o0 - band + 1 : 0;
  const int tb = (o1 - 1 + band < n) ? o1 - 1 + band : n;
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
  if (hosting) ctl_reduce_finish(ep.host_ctl, hsnap, hm, hden, hnum, ep.host_hist, par);
}

// ---------------------------------------------------------------------------
// dense point-cloud product: partial LSE over one column split.
//   part[split][i] = (m, s) with  m + log2 s = LSE2_{j in split}( w_j + log2 K_ij )
// rows: xr (DIM x Nr), columns: yc (DIM x Mc) and w (Mc, log2 units).
// COST 0: log2 K = -|x_i - y_j|^2 log2(e) / eps.
// COST 1: the WF cost with cut locus, log2 K = (2/eps) log2 cos((pi/2) d / cut)
//         for d < cut and -inf beyond (wf_log2k).  K then has exact zeros:
//         each block bounds its rows and every 256-column chunk by boxes and
//         skips a chunk whose box lies at distance >= cut from the rows' box
//         (every entry of that tile is zero; the skip is block-uniform).
// grid = (ceil(Nr / (256 R)), splits)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = Num<T>::fmin(v, __shfl_xor(v, o));
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = Num<T>::fmax(v, __shfl_xor(v, o));
  return v;
}

// bounding box of the points a block's threads hold (invalid ones pass
// lo = +inf, hi = -inf); every thread receives it.  Uses bx[4][2 DIM].
template <typename T, int DIM>
__device__ __forceinline__ void block_box(const T (&lo)[3], const T (&hi)[3], T (*bx)[6], T (&blo)[3],
                                          T (&bhi)[3]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const T a = wave_min<T>(lo[d]), b = wave_max<T>(hi[d]);
    if (lane == 0) {
      bx[wv][2 * d] = a;
      bx[wv][2 * d + 1] = b;
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    blo[d] = Num<T>::fmin(Num<T>::fmin(bx[0][2 * d], bx[1][2 * d]), Num<T>::fmin(bx[2][2 * d], bx[3][2 * d]));
    bhi[d] = Num<T>::fmax(Num<T>::fmax(bx[0][2 * d + 1], bx[1][2 * d + 1]),
                          Num<T>::fmax(bx[2][2 * d + 1], bx[3][2 * d + 1]));
  }
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
  __shared__ T rbx[4][6], cbx[4][6];
  const T sc = T(kLog2e / eps_of(c, side));
  const T ewf = T(2.0 / eps_of(c, side));
  T xi[R][DIM];
  int64_t rows[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    rows[r] = (int64_t)blockIdx.x * (kBlock * R) + r * kBlock + threadIdx.x;
    const int64_t rr = rows[r] < Nr ? rows[r] : 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[r][d] = xr[d * Nr + rr];
  }
  T rlo[3], rhi[3];
  if (COST == 1) {
    T lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      lo[d] = Num<T>::pinf();
      hi[d] = Num<T>::ninf();
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (rows[r] < Nr) {
          lo[d] = Num<T>::fmin(lo[d], xi[r][d]);
          hi[d] = Num<T>::fmax(hi[d], xi[r][d]);
        }
    }
    block_box<T, DIM>(lo, hi, rbx, rlo, rhi);
  }
  Lse2<T> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r].init();
  const int64_t cb = (int64_t)blockIdx.y * cols_per_split;
  const int64_t ce = (cb + cols_per_split < Mc) ? cb + cols_per_split : Mc;
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
    if (COST == 1) {
      // box of the chunk's columns that carry mass
      const bool live = rec.w != Num<T>::ninf();
      const T cx[3] = {rec.x, rec.y, rec.z};
      T lo[3], hi[3], clo[3], chi[3];
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        lo[d] = live ? cx[d] : Num<T>::pinf();
        hi[d] = live ? cx[d] : Num<T>::ninf();
      }
      block_box<T, DIM>(lo, hi, cbx, clo, chi);   // includes the barrier that publishes the tile
      T gap2 = T(0);
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const T g = Num<T>::fmax(Num<T>::fmax(clo[d] - rhi[d], rlo[d] - chi[d]), T(0));
        gap2 = Num<T>::fma(g, g, gap2);
      }
      // every entry of the tile is beyond the cut (an empty chunk gives nan
      // or +inf here and is skipped as well)
      if (!(gap2 < cut2)) continue;
    } else {
      __syncthreads();
    }
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
          if (COST == 1) t[k] = q[k].w + wf_log2k<T>(cst, a2, cut2, ewf);
          else t[k] = Num<T>::fma(-sc, cst, q[k].w);
        }
        acc[r].template add<kChunk>(t);
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

// merge the column splits of k_dense_lse, then the epilogue; grid = ceil(Nr/256)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_epi(const T* __restrict__ pm, const T* __restrict__ ps,
                                                       int nsplit, int64_t Nr, int side,
                                                       const Ctrl* __restrict__ c, EpiArgs<T> ep) {
  if (skip_side(c, side)) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < Nr;
  ResAcc<T> ra;
  ra.init();
  if (valid) {
    Lse2<T> acc;
    acc.init();
    for (int s = 0; s < nsplit; ++s) acc.merge(pm[s * Nr + i], ps[s * Nr + i]);
    epi_elem<T>(i, acc.result(), c, side, ep, ra);
  }
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
  __shared__ float smax[kBlock];
  const CtrlSnap snap = ctrl_snap(c, par);
  float rmax = -1.0f;
  const int per = nparts / nfields;
  for (int f = threadIdx.x; f < nfields; f += kBlock) {
    float m = -__builtin_inff(), den = 0.f, num = 0.f;
    for (int k = f * per; k < (f + 1) * per; ++k) res_merge<float>(m, den, num, part[k].m, part[k].den, part[k].num);
    const float rf = float(res_ratio(double(num), double(den)));
    rmax = (rf != rf || rmax != rmax) ? rf : (rf > rmax ? rf : rmax);
  }
  smax[threadIdx.x] = rmax;
  __syncthreads();
  for (int off = kBlock / 2; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const float a = smax[threadIdx.x], b = smax[threadIdx.x + off];
      smax[threadIdx.x] = (a != a || b != b) ? (a != a ? a : b) : (a > b ? a : b);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) control_finish(c, snap, double(smax[0]), hist, par);
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
  float m, den, num;
  ctl_load(part, nparts, m, den, num);
  asm volatile("" ::"v"(m), "v"(den), "v"(num));
  if (c->skip[par]) {
    if (threadIdx.x == 0) control_skip(c, par);
    return;
  }
  ctl_reduce_finish(c, snap, m, den, num, hist, par);
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
template <typename T>
__device__ T bary_f(const T* __restrict__ t2, int64_t stride, int n, const double* lav, bool tv, T a0, T d, T lb1,
                    T lb2, T b1, T b2, bool has_lo, T x) {
  T acc = tv ? a0 : T(0);
  for (int k = 0; k < n; ++k) {
    const T t = t2[k * stride] * T(kLn2);
    if (t == Num<T>::ninf()) continue;
    const T al = T(::exp(lav[k]));
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

// breakpoint w (0, 1) of input k, natural log t: TV t -+ d, RG t - log b2 / t - log b1
template <typename T>
__device__ __forceinline__ T bary_break(bool tv, T t, int w, T d, T lb1, T lb2) {
  return tv ? (w == 0 ? t - d : t + d) : (w == 0 ? t - lb2 : t - lb1);
}

template <typename T>
__device__ T bary_root(const T* __restrict__ t2, int64_t stride, int n, const BaryW& la, const DivDev& F, T eps) {
  const bool tv = F.kind == 2;
  T a0 = T(0), a1 = T(0);
  for (int k = 0; k < n; ++k) {
    const T al = T(::exp(la.v[k]));
    if (t2[k * stride] == Num<T>::ninf()) a0 += al;
    else a1 += al;
  }
  if (tv ? (a0 >= a1) : (a0 > T(0))) return Num<T>::ninf();
  if (!tv) {
    // every input within one band [b1 h, b2 h]: the function is zero on
    // [max log s_k - log b2, min log s_k - log b1]; return its left end
    // exactly (at a breakpoint the sum may round to -0)
    T tmax = Num<T>::ninf(), tmin = Num<T>::pinf();
    for (int k = 0; k < n; ++k) {
      const T t = t2[k * stride] * T(kLn2);
      tmax = t > tmax ? t : tmax;
      tmin = t < tmin ? t : tmin;
    }
    const T left = tmax - T(F.log_beta);
    if (!F.has_lo || left <= tmin - T(F.log_alpha)) return left;
  }
  const T d = tv ? T(F.lam) / eps : T(0);
  const T lb1 = F.has_lo ? T(F.log_alpha) : T(0), lb2 = T(F.log_beta);
  const T b1 = F.has_lo ? T(::exp(F.log_alpha)) : T(0), b2 = T(::exp(F.log_beta));
  const bool lo = F.has_lo != 0;
  const int per = tv ? 2 : (lo ? 2 : 1);
  // first breakpoint (in value) where the function is >= 0 ...
  T bhi = Num<T>::pinf(), fhi = T(0);
  for (int q = 0; q < n * per; ++q) {
    const int k = q / per, w = q % per;
    const T t = t2[k * stride] * T(kLn2);
    if (t == Num<T>::ninf()) continue;
    const T b = bary_break<T>(tv, t, w, d, lb1, lb2);
    if (b < bhi) {
      const T fb = bary_f<T>(t2, stride, n, la.v, tv, a0, d, lb1, lb2, b1, b2, lo, b);
      if (fb >= T(0)) {
        bhi = b;
        fhi = fb;
      }
    }
  }
  // ... and the breakpoint before it; the function is linear in between
  T blo = Num<T>::ninf();
  for (int q = 0; q < n * per; ++q) {
    const int k = q / per, w = q % per;
    const T t = t2[k * stride] * T(kLn2);
    if (t == Num<T>::ninf()) continue;
    const T b = bary_break<T>(tv, t, w, d, lb1, lb2);
    if (b < bhi && b > blo) blo = b;
  }
  if (blo == Num<T>::ninf()) return bhi;
  const T flo = bary_f<T>(t2, stride, n, la.v, tv, a0, d, lb1, lb2, b1, b2, lo, blo);
  return blo + (T(0) - flo) * (bhi - blo) / (fhi - flo);
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
  T logh;
  if (F2.kind == 2 || F2.kind == 3) {
    logh = bary_root<T>(T2 + j, size, nm, log_alpha, F2, eps);
  } else if (F2.kind == 0) {
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
static inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

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
    hipLaunchKernelGGL((k_grid_contig<T, 2>), dim3(gx, gy, gz), dim3(kBlock), lds, s, in, n, A, gtab, side, c, ep, bd);
  else
    hipLaunchKernelGGL((k_grid_contig<T, 1>), dim3(gx, gy, gz), dim3(kBlock), lds, s, in, n, A, gtab, side, c, ep, bd);
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
  template void launch_dense_lse<T>(int, int, const T*, int64_t, const T*, const T*, int64_t, int, int64_t, T*,  \
                                    T*, int, const Ctrl*, const CostArgs&, hipStream_t);                          \
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
// per half-step: each block pulls work items (problem, row tile) from an
// atomic cursor until the list is exhausted; items of problems that already
// stopped are skipped.  Items are pre-sorted by cost (rows x columns),
// largest first, so the tail of the launch is made of small items.
// ---------------------------------------------------------------------------
namespace uot {

template <typename T, int DIM, int R>
__global__ __launch_bounds__(kBlock) void k_batch_lse(const BItem* __restrict__ items, int n_items,
                                                       int* __restrict__ cursor, const int64_t* __restrict__ offR,
                                                       const int64_t* __restrict__ offC, const T* __restrict__ xr,
                                                       int64_t totR, const T* __restrict__ yc, int64_t totC,
                                                       const T* __restrict__ w, const BCtrl* __restrict__ bc,
                                                       const Ctrl* __restrict__ c, int side, EpiArgs<T> ep) {
  using V4 = typename Vec4<T>::type;
  __shared__ V4 tile[kBlock];
  __shared__ int item_sh;
  const T sc = T(kLog2e / eps_of(c, side));
  const int32_t* __restrict__ skip = half_of(side) == 0 ? bc->stop : bc->yskip;
  while (true) {
    __syncthreads();
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
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (vr[r]) epi_elem<T>(rb + I.row0 + r * kBlock + threadIdx.x, acc[r].result(), c, side, ep, ra);
    epi_finish<T>(ep, ra, I.part);
  }
}

// per-problem control (one thread per problem) between the X and Y half-steps
__global__ __launch_bounds__(kBlock) void k_batch_control(Ctrl* __restrict__ c, BCtrl* __restrict__ bc, int B,
                                                           const ResPart* __restrict__ part,
                                                           const int32_t* __restrict__ pstart, int* __restrict__ cursors) {
  const int b = blockIdx.x * kBlock + threadIdx.x;
  const int64_t l_glob = c->iter;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // cursors of the next launches, the global eps schedule and the counter slot
    cursors[0] = 0;
    cursors[1] = 0;
    c->active[(l_glob + 1) & 1] = 0;
  }
  if (b >= B) return;
  if (bc->stop[b]) {
    bc->yskip[b] = 1;
    return;
  }
  bc->yskip[b] = 0;
  float m = -__builtin_inff(), den = 0.f, num = 0.f;
  for (int k = pstart[b]; k < pstart[b + 1]; ++k) res_merge<float>(m, den, num, part[k].m, part[k].den, part[k].num);
  const double r = res_ratio(double(num), double(den));
  const int64_t l = bc->iters[b];
  bc->res[b] = r;
  bc->iters[b] = l + 1;
  const bool final_stage = c->iters_per_stage <= 0 || l >= (int64_t)c->n_stages * c->iters_per_stage;
  int stop = 0;
  if (r != r) { stop = 1; bc->status[b] = -3; }
  else if (final_stage && r <= c->tol && l >= 1) { stop = 1; bc->status[b] = 0; }
  else if (l + 1 >= c->max_iter) { stop = 1; bc->status[b] = 1; }
  if (stop) {
    bc->stop[b] = 1;
    bc->clock[b] = wall_clock64();
  } else {
    atomicAdd(&c->active[l & 1], 1);
  }
}

// global eps bookkeeping after the per-problem control (single thread)
__global__ void k_batch_advance(Ctrl* __restrict__ c, int par) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t l = c->iter;
  c->iter = l + 1;
  int64_t sn = c->iters_per_stage > 0 ? (l + 1) / c->iters_per_stage : c->n_stages;
  if (sn > c->n_stages) sn = c->n_stages;
  c->stage[par ^ 1] = (int)sn;
  c->eps[par ^ 1] = c->eps_tab[sn];
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
void launch_batch_lse(int dim, int R, int blocks, const BItem* items, int n_items, int* cursor, const int64_t* offR,
                      const int64_t* offC, const T* xr, int64_t totR, const T* yc, int64_t totC, const T* w,
                      const BCtrl* bc, const Ctrl* c, int side, const EpiArgs<T>& ep, hipStream_t s) {
#define UOT_BL(D, RR)                                                                                          \
  hipLaunchKernelGGL((k_batch_lse<T, D, RR>), dim3(blocks), dim3(kBlock), 0, s, items, n_items, cursor, offR, \
                     offC, xr, totR, yc, totC, w, bc, c, side, ep)
  if (R == 1) {
    if (dim == 1) UOT_BL(1, 1); else if (dim == 2) UOT_BL(2, 1); else UOT_BL(3, 1);
  } else if (R == 2) {
    if (dim == 1) UOT_BL(1, 2); else if (dim == 2) UOT_BL(2, 2); else UOT_BL(3, 2);
  } else {
    if (dim == 1) UOT_BL(1, 4); else if (dim == 2) UOT_BL(2, 4); else UOT_BL(3, 4);
  }
#undef UOT_BL
}

void launch_batch_control(Ctrl* c, BCtrl* bc, int B, const ResPart* part, const int32_t* pstart, int* cursors,
                          int par, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_control, dim3(ceil_div(B, kBlock)), dim3(kBlock), 0, s, c, bc, B, part, pstart, cursors);
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, c, par);
}

void launch_batch_init(BCtrl* bc, int B, Ctrl* c, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_init, dim3(ceil_div(B, kBlock)), dim3(kBlock), 0, s, bc, B, c);
}

void launch_set_int(int* p, int n, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, p, n, v);
}

template void launch_batch_lse<float>(int, int, int, const BItem*, int, int*, const int64_t*, const int64_t*,
                                      const float*, int64_t, const float*, int64_t, const float*, const BCtrl*,
                                      const Ctrl*, int, const EpiArgs<float>&, hipStream_t);
template void launch_batch_lse<double>(int, int, int, const BItem*, int, int*, const int64_t*, const int64_t*,
                                       const double*, int64_t, const double*, int64_t, const double*, const BCtrl*,
                                       const Ctrl*, int, const EpiArgs<double>&, hipStream_t);

}  // namespace uot

// ---------------------------------------------------------------------------
// Tile-factored separable pass on FP32 MFMA.  For output tile I and tap tile J
// of 16 cells each (centres cI, cJ, offsets e = i - cI, f = j - cJ, D = cI -
// cJ, all in cells) the 1-D kernel g(i - j) = -c (i - j)^2 (c = h^2 log2(e) /
// eps) splits exactly as
//   g = [-c e (e + 2D)] + [-c f (f - 2D)] - c D^2 + 2 c e f,
// so  sum_j 2^{g + w_j} = 2^{-c e (e+2D) - c D^2 + m} * sum_j Khat[e][f] E_j,
//   Khat[e][f] = 2^{2 c e f}  (one 16 x 16 matrix, |2 c e f| <= 2 c 7.5^2),
//   E_j = 2^{w_j - c f (f - 2D) - m},  m = max_j (w_j - c f (f - 2D)),
// and the inner sums of 16 lines at once are one 16x16x16 FP32 MFMA product.
// The J tiles of an output are combined by an online log-sum-exp.  Exact up
// to FP32 rounding; exp2 count per output: 16/16 (E) + 2 per J tile instead of
// 16 per J tile.  Requires n % 16 == 0.
// HALF: Khat and E in FP16, one v_mfma_f32_16x16x16f16 per J tile (FP32
// accumulation); lane (li, q) then holds taps 4 q .. 4 q + 3 of a tile.  The
// inputs carry FP16 rounding (2^-11 relative), so results are good to ~1e-3;
// Khat stays finite in FP16 while 2 c 7.5^2 <= 15.
//   STRIDED = false: in[a][j], lines a (16 per group);  out[a][i]
//   STRIDED = true : in[a][j][b], lines (a, b), 16 consecutive b per group
// grid = (n/16 output tiles, line groups (y, z)), 4 waves split the J tiles.
// ---------------------------------------------------------------------------
namespace uot {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));

template <bool STRIDED, int TPC, bool MULTI, bool HALF>
__global__ __launch_bounds__(kBlock) void k_grid_tf(const float* __restrict__ in, int n, int64_t A, int64_t B,
                                                     int opb, double h, int side, const Ctrl* __restrict__ c,
                                                     EpiArgs<float> ep) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane >> 4, li = lane & 15;
  const int nt = n / 16;
  // logical block -> (block of opb output tiles, line group of 16 lines)
  const int64_t lid = blockIdx.x;
  const int nob = MULTI ? opb : 1;         // output tiles of this block
  const int tpb = nt / nob;                // output-tile blocks per line group
  const int64_t grp = lid / tpb;
  const int ob = (int)(lid % tpb);
  int64_t a, bb;
  bool valid;
  if (STRIDED) {
    const int64_t gpa = (B + 15) / 16;     // groups per a
    a = grp / gpa;
    bb = (grp % gpa) * 16 + li;
    valid = (a < A) && (bb < B);
  } else {
    a = grp * 16 + li;
    bb = 0;
    valid = a < A;
  }
  const int64_t base = valid ? (STRIDED ? a * (int64_t)n * B + bb : a * (int64_t)n) : 0;
  const int64_t tstride = STRIDED ? B : 1;
  // The wave's tap tiles jt = wv, wv + 4, ... are taken in chunks of TPC
  // (4 TPC loads issued together).  The first chunk and the operands of the
  // first epilogue this wave finishes (outputs i = I0 + 4 q + wv of line li)
  // are loaded before the control block is read, so the latencies overlap.
  // Tap (jt, s) of the lane's line is cell jt * 16 + f(q, s), f = 4 s + q
  // (FP32 operand layout) or 4 q + s (FP16); tiles past the end are read at
  // the last tile (in bounds) and replaced by -inf.  Lanes of
  // a line past the end read line 0 unconditionally: lines never mix (MFMA
  // columns and the max exchanges stay within a line) and their outputs are
  // dropped, while a masked load would serialise the loads.
  auto tapf = [&](int s) -> int { return HALF ? 4 * q + s : 4 * s + q; };
  const float* __restrict__ pl = in + base;
  auto load_chunk = [&](float (&w)[TPC][4], int jc) {
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      const int jt = jc + 4 * t;
      const int jtc = jt < nt ? jt : nt - 1;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float x = pl[(int64_t)(jtc * 16 + tapf(s)) * tstride];
        w[t][s] = jt < nt ? x : -__builtin_inff();
      }
    }
  };
  // output element of lane (li, q) in output tile o of the block, row wv
  auto out_elem = [&](int o) -> int64_t {
    const int ie = (ob * nob + o) * 16 + 4 * q + wv;
    return valid ? (STRIDED ? (a * (int64_t)n + ie) * B + bb : a * (int64_t)n + ie) : 0;
  };
  float wv4[TPC][4];
  load_chunk(wv4, wv);
  int64_t eo = out_elem(0);
  EpiIn<float> xin = epi_load<float>(eo, ep);
  // block 0 of a launch that hosts the control step loads the residual
  // partials and control fields now, and finishes the step at the end
  const bool hosting = ep.host_ctl != nullptr && blockIdx.x == 0;
  const int par = par_of(side);
  CtrlSnap hsnap{};
  float hm = -__builtin_inff(), hden = 0.f, hnum = 0.f;
  if (hosting) {
    hsnap = ctrl_snap(ep.host_ctl, par);
    ctl_load(ep.host_parts, ep.host_nparts, hm, hden, hnum);
  }
  // keep those loads ahead of the branch (otherwise they may be moved past it)
#pragma unroll
  for (int t = 0; t < TPC; ++t)
#pragma unroll
    for (int s = 0; s < 4; ++s) asm volatile("" ::"v"(wv4[t][s]));
  asm volatile("" ::"v"(xin.ld), "v"(xin.uo), "v"(xin.lp));
  if (skip_side(c, side)) {
    if (hosting && threadIdx.x == 0) control_skip(ep.host_ctl, par);
    return;
  }
  const float cc = float(h * h * kLog2e / eps_of(c, side));
  // Khat as MFMA A operands: entry s of the lane is Khat[i = li][k = f(q, s)]
  float kh[4];
  f16x4_t kh16;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float e = float(li) - 7.5f, f = float(tapf(s)) - 7.5f;
    kh[s] = __builtin_amdgcn_exp2f(2.f * cc * e * f);
    kh16[s] = (_Float16)kh[s];
  }
  // opb > 1 only when one chunk holds all of a wave's tap tiles (the host
  // picks opb so), so the taps stay in registers across the output tiles
  __shared__ float smM[2][4][4][64], smS[2][4][4][64];
  ResAcc<float> ra;
  ra.init();
  for (int o = 0; o < nob; ++o) {
    const int I0 = (ob * nob + o) * 16;
    // epilogue operands of the next output tile, in flight during this one
    const bool more = MULTI && o + 1 < nob;
    const int64_t eo_next = more ? out_elem(o + 1) : eo;
    const EpiIn<float> xin_next = more ? epi_load<float>(eo_next, ep) : xin;
    // running LSE of the 4 outputs i = 4q + r of this lane's line li (D layout)
    float M[4], S[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      M[r] = -__builtin_inff();
      S[r] = 0.f;
    }
    for (int jc = wv; jc < nt; jc += 4 * TPC) {
      if (jc != wv) load_chunk(wv4, jc);
      // the TPC tiles of a chunk are independent until the final merge:
      // column factors and their line maxima first, then the products, so
      // the exchanges and the MFMA chains of different tiles overlap
      float D[TPC], mloc[TPC], beta[TPC][4];
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        D[t] = float(I0 - (jc + 4 * t) * 16);
        mloc[t] = -__builtin_inff();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float f = float(tapf(s)) - 7.5f;
          beta[t][s] = wv4[t][s] - cc * (f * (f - 2.f * D[t]));
          mloc[t] = fmaxf(mloc[t], beta[t][s]);
        }
      }
      // max over the 16 taps of the line: the four lane rows q share a line
#pragma unroll
      for (int t = 0; t < TPC; ++t) mloc[t] = max_over_rows(mloc[t]);
      f32x4_t acc[TPC];
      float E[TPC][4];
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        const float msh = (mloc[t] == -__builtin_inff()) ? 0.f : mloc[t];
#pragma unroll
        for (int s = 0; s < 4; ++s) E[t][s] = __builtin_amdgcn_exp2f(beta[t][s] - msh);
      }
      if (HALF) {
#pragma unroll
        for (int t = 0; t < TPC; ++t) {
          f16x4_t e16;
#pragma unroll
          for (int s = 0; s < 4; ++s) e16[s] = (_Float16)E[t][s];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(kh16, e16, acc[t], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int t = 0; t < TPC; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(kh[s], E[t][s], acc[t], 0, 0, 0);
      }
      // acc[t][r] = sum_f Khat[e_i][f] E_f for output i = 4 q + r of line li;
      // one rescale of the running sum per chunk
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float e = float(4 * q + r) - 7.5f;
        float al[TPC];
        float mn = M[r];
#pragma unroll
        for (int t = 0; t < TPC; ++t) {
          al[t] = (mloc[t] == -__builtin_inff()) ? -__builtin_inff()
                                                 : (mloc[t] - cc * (e * (e + 2.f * D[t])) - cc * D[t] * D[t]);
          mn = fmaxf(mn, al[t]);
        }
        const float sh = (mn == -__builtin_inff()) ? 0.f : mn;
        float sum = S[r] * __builtin_amdgcn_exp2f(M[r] - sh);
#pragma unroll
        for (int t = 0; t < TPC; ++t) sum += acc[t][r] * __builtin_amdgcn_exp2f(al[t] - sh);
        S[r] = sum;
        M[r] = mn;
      }
    }
    // merge the four waves (each saw a quarter of the J tiles); wave w then
    // finishes output row r = w of every lane.  Two LDS buffers alternate
    // over the output tiles, so one barrier per tile suffices.
    const int pb = o & 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      smM[pb][wv][r][lane] = M[r];
      smS[pb][wv][r][lane] = S[r];
    }
    __syncthreads();
    Lse2<float> tot;
    tot.m = smM[pb][0][wv][lane];
    tot.s = smS[pb][0][wv][lane];
#pragma unroll
    for (int k = 1; k < 4; ++k) tot.merge(smM[pb][k][wv][lane], smS[pb][k][wv][lane]);
    if (valid) epi_apply<float>(eo, tot.result(), xin, c, side, ep, ra);
    eo = eo_next;
    xin = xin_next;
  }
  epi_finish<float>(ep, ra, (int)lid);
  if (hosting) ctl_reduce_finish(ep.host_ctl, hsnap, hm, hden, hnum, ep.host_hist, par);
}

// output tiles per block: 1 unless there are enough line groups to fill the
// chip with fewer, longer blocks, and only while one chunk of tap tiles
// holds all of a wave's tiles (so the taps are loaded once per block)
static inline int tf_tpc(int n) {
  const int per_wave = (n / 16 + 3) / 4;
  return per_wave >= 4 ? 4 : (per_wave >= 2 ? 2 : 1);
}

static inline int tf_opb(int n, int64_t groups) {
  const int nt = n / 16;
  if (nt > 4 * tf_tpc(n)) return 1;
  int opb = 1;
  while (nt % (opb * 2) == 0 && (int64_t)(nt / (opb * 2)) * groups >= 2048) opb *= 2;
  return opb;
}

static inline int64_t tf_groups(int64_t A, int64_t B, bool strided) {
  return strided ? A * ((B + 15) / 16) : (A + 15) / 16;
}

int grid_tf_parts(int n, int64_t A, int64_t B, bool strided) {
  const int64_t g = tf_groups(A, B, strided);
  return (int)((n / 16) / tf_opb(n, g) * g);
}

template <bool ST, int TP, bool HF>
static void launch_tf_t(unsigned blocks, int opb, const float* in, int64_t A, int n, int64_t B, double h, int side,
                        const Ctrl* c, const EpiArgs<float>& ep, hipStream_t s) {
  if (opb > 1)
    hipLaunchKernelGGL((k_grid_tf<ST, TP, true, HF>), dim3(blocks), dim3(kBlock), 0, s, in, n, A, B, opb, h, side, c,
                       ep);
  else
    hipLaunchKernelGGL((k_grid_tf<ST, TP, false, HF>), dim3(blocks), dim3(kBlock), 0, s, in, n, A, B, 1, h, side, c,
                       ep);
}

template <bool ST, bool HF>
static void launch_tf_tpc(int tpc, unsigned blocks, int opb, const float* in, int64_t A, int n, int64_t B, double h,
                          int side, const Ctrl* c, const EpiArgs<float>& ep, hipStream_t s) {
  if (tpc == 4) launch_tf_t<ST, 4, HF>(blocks, opb, in, A, n, B, h, side, c, ep, s);
  else if (tpc == 2) launch_tf_t<ST, 2, HF>(blocks, opb, in, A, n, B, h, side, c, ep, s);
  else launch_tf_t<ST, 1, HF>(blocks, opb, in, A, n, B, h, side, c, ep, s);
}

void launch_grid_tf(const float* in, int64_t A, int n, int64_t B, bool strided, bool half, double h, int side,
                    const Ctrl* c, const EpiArgs<float>& ep, hipStream_t s) {
  const int64_t g = tf_groups(A, B, strided);
  const int opb = tf_opb(n, g);
  const unsigned blocks = (unsigned)((n / 16) / opb * g);
  const int tpc = tf_tpc(n);
  if (strided) {
    if (half) launch_tf_tpc<true, true>(tpc, blocks, opb, in, A, n, B, h, side, c, ep, s);
    else launch_tf_tpc<true, false>(tpc, blocks, opb, in, A, n, B, h, side, c, ep, s);
  } else {
    if (half) launch_tf_tpc<false, true>(tpc, blocks, opb, in, A, n, B, h, side, c, ep, s);
    else launch_tf_tpc<false, false>(tpc, blocks, opb, in, A, n, B, h, side, c, ep, s);
  }
}

}  // namespace uot
