// Epilogue and control-step device helpers shared by the Gibbs-product
// kernels of libuot (uot_kernels.hip, uot_grid_tf.hip): the pointwise proxdiv
// epilogue with the residual partials, and the control step of an iteration.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "uot_device.h"
#include "uot_launch.h"

namespace uot {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// epilogue shared by every Gibbs product.  epi_elem handles one element with
// S2 = log2 of the product; epi_finish reduces the residual partials of the
// block (every thread of the block must call it).
// ---------------------------------------------------------------------------
template <typename T> struct ResAcc {
  T m, den, num, du;   // du: largest |u_new - u_old| seen
  __device__ __forceinline__ void init() {
    m = Num<T>::ninf();
    den = T(0);
    num = T(0);
    du = T(0);
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
      if (uo != Num<T>::ninf()) {
        ra.add((S + uo / eps + ld) * T(kLog2e), T(0), T(1));
        ra.du = Num<T>::pinf();           // a potential that jumped to -inf
      }
    } else {
      const T d = Num<T>::expm1((uo - un) / eps);
      ra.add((S + un / eps + ld) * T(kLog2e), T(1), Num<T>::fmax(d, -d));
      const T a = uo - un;
      ra.du = Num<T>::fmax(ra.du, uo == Num<T>::ninf() ? Num<T>::pinf() : Num<T>::fmax(a, -a));
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

// Ragged batches, the in-solve mass balance: in the half-steps that run
// while the iteration counter equals ep.bal_iter, the plan's marginal mass
// over an item's rows (log2 units: S2 + (pot/eps + log d) log2(e), the row's
// a K b d, once its epilogue wrote the new potential) goes to one more
// block partial.  Rows with no mass (p = 0, or a vanishing product) add
// nothing.
template <typename T>
__device__ __forceinline__ bool bal_on(const EpiArgs<T>& ep, const Ctrl* __restrict__ c) {
  return ep.bal_m != nullptr && c->iter == ep.bal_iter;
}
// (m, s): a running log2-sum-exp in T precision, m + log2 s
template <typename T> struct MassAcc {
  T m, s;
  __device__ __forceinline__ void init() { m = Num<T>::ninf(); s = T(0); }
  __device__ __forceinline__ void add(T t) {
    if (t == Num<T>::ninf()) return;
    const T mn = Num<T>::fmax(m, t);
    s = s * Num<T>::exp2(m - mn) + Num<T>::exp2(t - mn);
    m = mn;
  }
};
template <typename T>
__device__ __forceinline__ void bal_elem(int64_t e, T S2, const Ctrl* __restrict__ c, int side, const EpiArgs<T>& ep,
                                         MassAcc<T>& mb) {
  if (S2 == Num<T>::ninf()) return;
  const T un = ep.pot[e];
  if (un == Num<T>::ninf() || un == Num<T>::pinf()) return;
  const T ld = ep.logd[e < ep.size ? e : e % ep.size];
  mb.add(S2 + (un / T(eps_of(c, side)) + ld) * T(kLog2e));
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
  if (ep.part) block_res_reduce<T>(ra.m, ra.den, ra.num, ra.du, ep.part + part_index);
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
static __device__ void control_finish(Ctrl* c, const CtrlSnap& s, double r, double du, double* __restrict__ hist,
                                      int par) {
  if (hist) hist[s.l] = r;
  c->res = r;
  c->du = du;
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
                                         float& num, float& du) {
  m = -__builtin_inff();
  den = num = du = 0.f;
  for (int k = threadIdx.x; k < nparts; k += kBlock) {
    res_merge<float>(m, den, num, part[k].m, part[k].den, part[k].num);
    du = fmaxf(du, part[k].du);
  }
}

// block reduction of the shares and the control step (every thread of the
// block calls it)
__device__ __forceinline__ void ctl_reduce_finish(Ctrl* c, const CtrlSnap& snap, float m, float den, float num,
                                                  float du, double* __restrict__ hist, int par) {
  __shared__ ResPart tot;
  __syncthreads();   // the block's own reductions before this one are complete
  block_res_reduce<float>(m, den, num, du, &tot);
  __syncthreads();
  if (threadIdx.x == 0)
    control_finish(c, snap, res_ratio(double(tot.num), double(tot.den)), double(tot.du), hist, par);
}

}  // namespace uot
