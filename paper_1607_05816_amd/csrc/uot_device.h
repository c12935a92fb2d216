// Device-side building blocks of libuot (gfx950, wave64).
//
// All log-sum-exps run in base 2 (v_exp_f32 / v_log_f32 are base-2
// instructions): a field w stored "in log2 units" means w = (pot/eps + log d)
// * log2(e), and a pass returns log2 of the Gibbs product.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace uot {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.6931471805599453094;
constexpr int kMaxStages = 32;

// ---------------------------------------------------------------------------
// scalar math per precision
// ---------------------------------------------------------------------------
template <typename T> struct Num;

template <> struct Num<float> {
  static __device__ __forceinline__ float ninf() { return -__builtin_inff(); }
  static __device__ __forceinline__ float pinf() { return __builtin_inff(); }
  // hardware v_exp_f32 / v_log_f32 (base 2); inputs below -126 give 0
  static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
  static __device__ __forceinline__ float log2(float x) { return __builtin_amdgcn_logf(x); }
  static __device__ __forceinline__ float expm1(float x) { return ::expm1f(x); }
  static __device__ __forceinline__ float exp(float x) { return ::expf(x); }
  static __device__ __forceinline__ float log(float x) { return ::logf(x); }
  static __device__ __forceinline__ float fmax(float a, float b) { return __builtin_fmaxf(a, b); }
  static __device__ __forceinline__ float fmin(float a, float b) { return __builtin_fminf(a, b); }
  static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};

template <> struct Num<double> {
  static __device__ __forceinline__ double ninf() { return -__builtin_inf(); }
  static __device__ __forceinline__ double pinf() { return __builtin_inf(); }
  static __device__ __forceinline__ double exp2(double x) { return ::exp2(x); }
  static __device__ __forceinline__ double log2(double x) { return ::log2(x); }
  static __device__ __forceinline__ double expm1(double x) { return ::expm1(x); }
  static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
  static __device__ __forceinline__ double log(double x) { return ::log(x); }
  static __device__ __forceinline__ double fmax(double a, double b) { return __builtin_fmax(a, b); }
  static __device__ __forceinline__ double fmin(double a, double b) { return __builtin_fmin(a, b); }
  static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
};

// ---------------------------------------------------------------------------
// cos(sqrt(z)) on 0 <= z <= (pi/2)^2 from the Taylor series of cos in
// z = theta^2, sum_k (-z)^k / (2k)!, in Horner form.  FP32 stops after z^6
// (remainder z^7/14! < 6.5e-9 at the end of the range), FP64 after z^10
// (remainder z^11/22! < 1.9e-17).  The WF cost -log cos^2(theta) only needs
// theta^2, so no square root and no range reduction are taken.
// ---------------------------------------------------------------------------
template <typename T> struct CosSqrt;
template <> struct CosSqrt<float> {
  static __device__ __forceinline__ float eval(float z) {
    float r = 1.0f / 479001600.0f;                 // 1/12!
    r = __builtin_fmaf(r, -z, 1.0f / 3628800.0f);  // 1/10!
    r = __builtin_fmaf(r, -z, 1.0f / 40320.0f);
    r = __builtin_fmaf(r, -z, 1.0f / 720.0f);
    r = __builtin_fmaf(r, -z, 1.0f / 24.0f);
    r = __builtin_fmaf(r, -z, 0.5f);
    return __builtin_fmaf(r, -z, 1.0f);
  }
};
template <> struct CosSqrt<double> {
  static __device__ __forceinline__ double eval(double z) {
    // 1/(2k)! for k = 10 .. 1
    constexpr double c[10] = {1.0 / 2432902008176640000.0, 1.0 / 6402373705728000.0, 1.0 / 20922789888000.0,
                              1.0 / 87178291200.0,         1.0 / 479001600.0,        1.0 / 3628800.0,
                              1.0 / 40320.0,               1.0 / 720.0,              1.0 / 24.0,
                              0.5};
    double r = c[0];
#pragma unroll
    for (int k = 1; k < 10; ++k) r = __builtin_fma(r, -z, c[k]);
    return __builtin_fma(r, -z, 1.0);
  }
};

// log2 of the WF kernel entry cos_+^{2/eps}(theta), theta = (pi/2) d / cut:
// ewf log2 cos(theta) with z = theta^2 = a2 d^2 (a2 = (pi / (2 cut))^2) while
// d^2 < cut^2; -inf from the cut locus on (the entry is exactly zero)
template <typename T>
__device__ __forceinline__ T wf_log2k(T d2, T a2, T cut2, T ewf) {
  const T cv = CosSqrt<T>::eval(d2 * a2);
  return (d2 < cut2 && cv > T(0)) ? ewf * Num<T>::log2(cv) : Num<T>::ninf();
}

// ---------------------------------------------------------------------------
// running log2-sum-exp2 with a chunked online maximum: the value is
// m + log2(s).  add<C>() folds C terms with one rescale, so the per-term
// cost is one max, one subtract, one exp2 and one add.
// ---------------------------------------------------------------------------
template <typename T> struct Lse2 {
  T m, s;
  __device__ __forceinline__ void init() { m = Num<T>::ninf(); s = T(0); }

  template <int C>
  __device__ __forceinline__ void add(const T* t) {
    T cm = t[0];
#pragma unroll
    for (int k = 1; k < C; ++k) cm = Num<T>::fmax(cm, t[k]);
    const T mn = Num<T>::fmax(m, cm);
    const T sh = (mn == Num<T>::ninf()) ? T(0) : mn;   // all -inf so far: keep s = 0
    T acc = s * Num<T>::exp2(m - sh);
#pragma unroll
    for (int k = 0; k < C; ++k) acc += Num<T>::exp2(t[k] - sh);
    m = mn;
    s = acc;
  }

  __device__ __forceinline__ void merge(T m2, T s2) {
    const T mn = Num<T>::fmax(m, m2);
    if (mn == Num<T>::ninf()) return;
    s = s * Num<T>::exp2(m - mn) + s2 * Num<T>::exp2(m2 - mn);
    m = mn;
  }

  // log2 of the sum; -inf for an empty / all -inf sum
  __device__ __forceinline__ T result() const { return m + Num<T>::log2(s); }
};

// ---------------------------------------------------------------------------
// control block: one per solve, lives in the workspace.  Every kernel reads
// eps and its skip flag here, so a captured chunk of iterations is the same
// graph for every eps stage and stops by itself once converged.
// ---------------------------------------------------------------------------
struct Ctrl {
  // Per-iteration state lives in two slots indexed by the parity of the
  // iteration, so the control step of iteration l (which fills the slot of
  // l + 1) may run inside a kernel whose other blocks still read the slot of l.
  int32_t stop;      // set once the solve has stopped (read by the host)
  int32_t status;    // 0 ok, 1 not converged, -3 non-finite residual
  int32_t skip[2];   // the half-steps of an iteration of parity p skip when skip[p] is set
  int32_t stage[2];  // eps stage of the iteration of parity p
  int32_t n_stages;  // annealing stages before the final eps
  int32_t iters_per_stage;
  int64_t iter;      // completed iterations (= index of the next one)
  int64_t max_iter;
  double tol;
  double res;        // residual of the last iteration
  double du;         // max |u_new - u_old| of the last iteration (potential units)
  double eps[2];     // eps of the iteration of parity p
  double eps_tab[kMaxStages + 1];
  double zeta;       // log z of a total-mass penalty (Algorithm 4); 0 otherwise
  // ragged batches only
  int32_t active[2];  // problems still active after the last iteration (slot = iteration parity)
  int32_t nstop;      // problems stopped so far
  int32_t built[2];   // nstop when the item lists were last rebuilt (slot = iteration parity)
  uint64_t t0_clock;  // device wall clock at the start of the solve
  // timed solves: pair evaluations of the matrix-core products
  unsigned long long pairs;
};

// A kernel's `side` argument: bit 0 the half-step (0: X, 1: Y), bit 1 the
// parity of the iteration it belongs to.
__device__ __forceinline__ int half_of(int side) { return side & 1; }
__device__ __forceinline__ int par_of(int side) { return (side >> 1) & 1; }
__device__ __forceinline__ bool skip_side(const Ctrl* c, int side) { return c->skip[par_of(side)] != 0; }
__device__ __forceinline__ double eps_of(const Ctrl* c, int side) { return c->eps[par_of(side)]; }
__device__ __forceinline__ int stage_of(const Ctrl* c, int side) { return c->stage[par_of(side)]; }
// eps of the half-step that reads this epilogue's w: the Y half-step of the
// same iteration (X side) or the X half-step of the next one (Y side)
__device__ __forceinline__ double eps_next_of(const Ctrl* c, int side) {
  return c->eps[par_of(side) ^ half_of(side)];
}

// per-problem state of a ragged batch (arrays of length B in the workspace)
struct BCtrl {
  int32_t* stop;     // set by the control step of the iteration the problem stopped in
  int32_t* yskip;    // stop as it was before the last control step: the Y half-step after that
                     // step still runs for a problem that stopped in it
  int32_t* status;
  int64_t* iters;
  double* res;
  uint64_t* clock;   // device wall clock when the problem stopped
};

// one work item of a ragged batch: rows [row0, row0 + nrows) of problem prob;
// its residual partial goes to slot part
struct BItem {
  int32_t prob, row0, nrows, part;
};

// Item lists of a ragged batch (k_batch_compact): each side's problems in a
// fixed order (largest column count first, so the list runs from the
// costliest row tiles down), every listed problem contributing its row
// tiles.  The lists are rebuilt from the problems still running once enough
// of the listed ones have stopped; until then the products skip the items of
// stopped problems.
struct BatchLists {
  const int32_t* ord[2];   // problem order of the X-row and Y-row lists
  const int64_t* off[2];   // row offsets of each side (offN, offM)
  const int32_t* pstart;   // residual slot of the first X item of each problem
  const int32_t* pstartY;  // mass-partial slot of the first Y item of each problem
  BItem* items[2];         // the lists (written)
  int* count[2];           // their lengths (written)
  int* cursor[2];          // the products' work cursors (reset every iteration)
  int rows;                // rows per item
};

// residual partial (per block): value = 2^m * {den, num} (m in log2 units);
// du: the block's largest |u_new - u_old| (potential units)
struct ResPart {
  float m, den, num, du;
};

// ---------------------------------------------------------------------------
// proxdiv rows of Table proximalexplicit in the log domain, returning the new
// potential eps*log(a) from S = log K(b dy) (natural log), zero absorbed offset.
// ---------------------------------------------------------------------------
struct DivDev {
  int kind;          // 0 =, 1 KL, 2 TV, 3 RG, 4 growth
  int has_lo, has_hi;
  int pad;
  double lam, log_alpha, log_beta;   // growth: log_alpha = log(1 - lam)
};

template <typename T>
__device__ __forceinline__ T proxdiv_pot(const DivDev& F, T logp, T S, T eps) {
  // log(p/s): -inf where p = 0 (also where s = 0: 0/0 = 0), +inf where only s = 0
  const T d = (logp == Num<T>::ninf()) ? Num<T>::ninf() : logp - S;
  switch (F.kind) {
    case 0:
      return eps * d;
    case 1: {
      const T lam = T(F.lam);
      return (eps * lam / (lam + eps)) * d;
    }
    case 2: {
      const T lam = T(F.lam);
      return Num<T>::fmin(Num<T>::fmax(eps * d, -lam), lam);
    }
    case 3: {
      const T lo = F.has_lo ? eps * (T(F.log_alpha) + d) : Num<T>::ninf();
      const T hi = F.has_hi ? eps * (T(F.log_beta) + d) : Num<T>::pinf();
      return Num<T>::fmin(hi, Num<T>::fmax(lo, T(0)));
    }
    default: {
      // growth functional (tumour example of the WF gradient flows): the
      // constant branch -log kappa below the switch, the KL(1)-like branch
      // eps (log p - log s) / (1 + eps) above it; p is the density cap
      return Num<T>::fmin(-T(F.log_alpha), (eps / (T(1) + eps)) * d);
    }
  }
}

// relative residual num / den with 0/0 = 0 (a marginal that vanishes before
// and after the update) and +inf for mass that vanished
__device__ __forceinline__ double res_ratio(double num, double den) {
  return den > 0.0 ? num / den : (num > 0.0 ? __builtin_inf() : 0.0);
}

// ---------------------------------------------------------------------------
// wave64 / block reductions
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void res_merge(T& m, T& den, T& num, T m2, T den2, T num2) {
  const T mn = Num<T>::fmax(m, m2);
  if (mn == Num<T>::ninf()) return;
  const T f1 = Num<T>::exp2(m - mn), f2 = Num<T>::exp2(m2 - mn);
  den = den * f1 + den2 * f2;
  num = num * f1 + num2 * f2;
  m = mn;
}

// Cross-lane exchanges that stay in the VALU (no LDS crossbar).
//   lane_xor16 / lane_xor32 (gfx950 v_permlane16_swap / v_permlane32_swap):
//     with both operands x, the swap leaves x and its partner at distance
//     16 (32) in the two results, in some order; callers combine the pair
//     with a symmetric operation, so the order does not matter.
//   dpp_* : row-local DPP moves (quad_perm [1,0,3,2], [2,3,0,1], row half
//     mirror, row mirror) that complete a reduction over a row of 16 lanes.
struct LanePair {
  float a, b;
};
__device__ __forceinline__ LanePair lane_xor16(float x) {
  const unsigned u = __float_as_uint(x);
  const auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return {__uint_as_float(p[0]), __uint_as_float(p[1])};
}
__device__ __forceinline__ LanePair lane_xor32(float x) {
  const unsigned u = __float_as_uint(x);
  const auto p = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  return {__uint_as_float(p[0]), __uint_as_float(p[1])};
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i of 8 <- lane 7 - i
constexpr int kDppMirror = 0x140;      // lane i of 16 <- lane 15 - i

// max over the four lanes l % 16 + {0, 16, 32, 48}
__device__ __forceinline__ float max_over_rows(float x) {
  const LanePair p = lane_xor16(x);
  const float y = fmaxf(p.a, p.b);
  const LanePair r = lane_xor32(y);
  return fmaxf(r.a, r.b);
}

// Reduce (m, den, num) over a wave with res_merge; every lane ends with the
// wave total (up to rounding order).
__device__ __forceinline__ void wave_res_reduce(float& m, float& den, float& num, float& du) {
#define UOT_RES_STEP(MOVE)                                               \
  {                                                                      \
    const float m2 = MOVE(m), d2 = MOVE(den), n2 = MOVE(num), u2 = MOVE(du); \
    res_merge<float>(m, den, num, m2, d2, n2);                           \
    du = fmaxf(du, u2);                                                  \
  }
  UOT_RES_STEP(dpp_mov<kDppXor1>)
  UOT_RES_STEP(dpp_mov<kDppXor2>)
  UOT_RES_STEP(dpp_mov<kDppHalfMirror>)
  UOT_RES_STEP(dpp_mov<kDppMirror>)
#undef UOT_RES_STEP
  {
    const LanePair pm = lane_xor16(m), pd = lane_xor16(den), pn = lane_xor16(num), pu = lane_xor16(du);
    m = pm.a;
    den = pd.a;
    num = pn.a;
    res_merge<float>(m, den, num, pm.b, pd.b, pn.b);
    du = fmaxf(pu.a, pu.b);
  }
  {
    const LanePair pm = lane_xor32(m), pd = lane_xor32(den), pn = lane_xor32(num), pu = lane_xor32(du);
    m = pm.a;
    den = pd.a;
    num = pn.a;
    res_merge<float>(m, den, num, pm.b, pd.b, pn.b);
    du = fmaxf(pu.a, pu.b);
  }
}

// Reduce (m, den, num) and the largest |du| over a block of 256 threads (m in
// log2 units); thread 0 writes the result.  Every thread of the block must
// call this.  The partials only feed the stopping test and the reported
// sup-norm, so FP32 with the hardware exp2 is enough (relative error ~1e-7
// on r; du is rounded once to FP32).
template <typename T>
__device__ __forceinline__ void block_res_reduce(T m_in, T den_in, T num_in, T du_in, ResPart* out) {
  __shared__ float sm[4][4];
  float m = float(m_in), den = float(den_in), num = float(num_in), du = float(du_in);
  wave_res_reduce(m, den, num, du);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm[w][0] = m;
    sm[w][1] = den;
    sm[w][2] = num;
    sm[w][3] = du;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float M = sm[0][0], D = sm[0][1], U = sm[0][2], X = sm[0][3];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
      res_merge<float>(M, D, U, sm[k][0], sm[k][1], sm[k][2]);
      X = fmaxf(X, sm[k][3]);
    }
    out->m = M;
    out->den = D;
    out->num = U;
    out->du = X;
  }
}

}  // namespace uot
