// C ABI of libuot (declared in include/uot.h): validation, workspace layout,
// the iteration driver (direct launches or replayed hipGraph chunks) and the
// objective / barycentre / single half-step entry points.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <type_traits>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/uot.h"
#include "uot_device.h"
#include "uot_launch.h"

using namespace uot;

#include "uot_ctx.h"

namespace uot {
thread_local std::string g_err;
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
}  // namespace uot

// Scratch memory of uot_half_step_noalloc: one zero-initialised array in the
// code object, so each GPU the library runs on holds its own copy from module
// load until the process ends, and that entry point allocates nothing.  On the
// host `scratch` is only a stand-in for the symbol: kernels receive the device
// address that hipGetSymbolAddress returns for the current device, looked up
// once per device by uot_create.
static __device__ __align__(256) char scratch[UOT_SCRATCH_BYTES];

namespace {

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on `dev` (the current device), looked up on the
// first call for that device and kept
hipError_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Per-launch HIP-event timing of the kernels of a solve (when requested): every
// launch enqueued through timed() is bracketed by two events on the library
// stream; after each chunk the host adds the elapsed times per kernel class.
struct KTimer {
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> pool;
  std::vector<int> cls;
  size_t used = 0;
  double ms[4] = {0, 0, 0, 0};
  int64_t count[4] = {0, 0, 0, 0};
  ~KTimer() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  void collect() {
    for (size_t k = 0; k < used; ++k) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, pool[2 * k], pool[2 * k + 1]) == hipSuccess) {
        ms[cls[k]] += t;
        count[cls[k]] += 1;
      }
    }
    used = 0;
    cls.clear();
  }
};
thread_local KTimer* g_timer = nullptr;

template <typename F>
void timed(int c, F&& launch) {
  KTimer* t = g_timer;
  if (!t) {
    launch();
    return;
  }
  if (2 * (t->used + 1) > t->pool.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        launch();
        return;
      }
      t->pool.push_back(e);
    }
  }
  (void)hipEventRecord(t->pool[2 * t->used], t->s);
  launch();
  (void)hipEventRecord(t->pool[2 * t->used + 1], t->s);
  t->cls.push_back(c);
  t->used += 1;
}

DivDev to_dev(const uot_div& d) {
  DivDev r{};
  r.kind = d.kind;
  r.lam = d.lambda;
  r.has_lo = (d.kind == UOT_DIV_RG && d.alpha > 0) ? 1 : 0;
  r.has_hi = (d.kind == UOT_DIV_RG && std::isfinite(d.beta)) ? 1 : 0;
  r.log_alpha = r.has_lo ? std::log(d.alpha) : 0.0;
  r.log_beta = r.has_hi ? std::log(d.beta) : 0.0;
  if (d.kind == UOT_DIV_GROWTH) r.log_alpha = std::log1p(-d.lambda);
  return r;
}

int check_div(const uot_div& d, const char* name) {
  if (d.kind < 0 || d.kind > 4) return fail(UOT_E_INVALID, std::string(name) + ": unknown divergence kind");
  if (d.kind == UOT_DIV_GROWTH && !(d.lambda >= 0 && d.lambda < 1))
    return fail(UOT_E_INVALID, std::string(name) + ": growth needs 0 <= lambda (= 2 tau alpha) < 1");
  if ((d.kind == UOT_DIV_KL || d.kind == UOT_DIV_TV) && !(d.lambda > 0 && std::isfinite(d.lambda)))
    return fail(UOT_E_INVALID, std::string(name) + ": lambda must be finite and > 0");
  if (d.kind == UOT_DIV_RG && !(d.alpha >= 0 && d.beta >= d.alpha && d.beta > 0))
    return fail(UOT_E_INVALID, std::string(name) + ": RG needs 0 <= alpha <= beta, beta > 0");
  return UOT_OK;
}

// ---------------------------------------------------------------------------
// problem plan + workspace layout
// ---------------------------------------------------------------------------
struct Plan {
  int dtype = 0;
  size_t esz = 0;
  int geom = 0;
  int dim = 0;
  int64_t N = 0, M = 0;
  int64_t n[3] = {1, 1, 1};
  double h[3] = {0, 0, 0};
  int nb = 1;            // fields (barycentre marginals)
  int nst = 1;           // eps stages incl. the final one (tables per axis)
  // dense split configuration per side (0: rows X, 1: rows Y)
  int R[2] = {1, 1};
  int splits[2] = {1, 1};
  int64_t cps[2] = {0, 0};
  int nparts_x = 0;      // residual partials written by the X epilogue
  int nparts_y = 0;      // blocks of the Y epilogue (mass partials of Algorithm 4)
  int gk = 1;            // grid passes: 1 direct log-sum-exp, 2 tile-factored MFMA where allowed
  bool tf_axis[3] = {false, false, false};   // tile-factored pass used on this axis
  bool tf16_axis[3] = {false, false, false}; // ... with FP16 operands
  CostArgs cost{0, 0, 0.0};                  // squared Euclidean or WF with a cut locus
  int band[3] = {0, 0, 0};                   // grid axes: taps |i - j| < band can be non-zero
  int split1d = 1;                           // 1-D grids: tap slices of the (direct) pass
  mutable void* split_pm = nullptr;          // ... their partial LSEs (set by carve)
  mutable void* split_ps = nullptr;
  bool dense_tf = false;                     // points: tile-factored product
  bool dense_mf = false;                     // points: product on the matrix cores
  bool mf_split = false;                     // ... with BF16 x 3 operands (else FP32)
  int mf_groups = 4;                         // its row groups of 16 per wave (4 or 8)
  int mf_target[2] = {0, 0};                 // its block target per side (0: 1024)
  // the factored products run on Morton-ordered copies of the clouds (rows
  // of a wave or block lie close together, so the factored exponents keep
  // small magnitudes), and so do the WF products (the boxes of row waves and
  // column groups stay small, so few pairs of them lie within the cut);
  // results are scattered back to the caller's order
  bool sorted() const { return dense_tf || dense_mf || (geom == UOT_GEOM_POINTS && cost.kind == UOT_COST_WF); }
  // workspace offsets
  size_t o_ctrl, o_logp, o_logq, o_logdx, o_logdy, o_wu, o_wv, o_t1, o_t2, o_t3, o_pm, o_ps, o_parts, o_gtab[3],
      o_gcost, o_obj, o_scal, o_mass, o_xs, o_ys, o_permx, o_permy, o_code, o_box, o_us, o_vs, o_pw, o_wfl[2],
      o_wfpart, total;
  int64_t obj_doubles = 0;
  int64_t np_pw = 0;                         // points: row maxima per side (matrix-core product)
  int64_t wf_slots = 0;                      // WF points: unit slots of the larger side
  bool wfl = false;                          // WF points: work lists built for this call
  int wf_umax[2] = {0, 0};                   // ... and the largest unit count of a row wave per side
};

// WF points, one side (rows against columns): row waves of 64 rows, column
// groups of 16, mask words of 32 groups per row wave, and unit slots (a unit
// holds up to 16 groups within the cut)
struct WfShape {
  int64_t nrw, ngr, nwd;
  explicit WfShape(int64_t Nr, int64_t Mc) : nrw((Nr + 63) / 64), ngr((Mc + 15) / 16), nwd((ngr + 31) / 32) {}
  int64_t words() const { return nrw * nwd; }
  int64_t slots() const { return nrw * ((ngr + 15) / 16); }
};

bool use_tf(const Plan& P, int axis) { return P.tf_axis[axis]; }

// The tile-factored pass multiplies by Khat = 2^{2 c e f} with |e|, |f| <= 7.5
// and c = h^2 log2(e) / eps; it is used on an axis only while 2 c 7.5^2 stays
// far inside the FP32 range (c <= 0.5, i.e. |log2 Khat| <= 56.25) at the
// smallest eps of the schedule, and only for FP32 axes of a multiple of 16 cells.
constexpr double kTfMaxC = 0.5;
// FP16 operands (grid_kernel 3): Khat must stay below the FP16 maximum, 2 c
// 7.5^2 <= 15 (c <= 0.133); axes beyond that use the FP32 MFMA pass.
constexpr double kTf16MaxC = 0.125;
// Mixed precision (grid_kernel 4): FP16 operands until the residual reaches
// this value (the FP16 passes level off near 2e-5), FP32 operands after.
constexpr double kMixedSwitchTol = 1e-4;

bool has_tf16(const Plan& P) { return P.tf16_axis[0] || P.tf16_axis[1] || P.tf16_axis[2]; }

int grid_final_parts_for(const Plan& P, bool tf0) {
  const int64_t nb = P.nb;
  if (P.dim == 1 && !tf0 && P.split1d > 1) return (int)((nb * P.n[0] + 255) / 256);   // merge blocks
  if (P.dim == 1) return tf0 ? grid_tf_parts((int)P.n[0], nb, 1, false) : grid_contig_parts<float>((int)P.n[0], nb);
  const int64_t B = P.dim == 2 ? P.n[1] : P.n[1] * P.n[2];
  return tf0 ? grid_tf_parts((int)P.n[0], nb, B, true) : grid_strided_parts<float>((int)P.n[0], nb, B);
}

int grid_final_parts(const Plan& P) { return grid_final_parts_for(P, use_tf(P, 0)); }

int dense_blocks_env() {
  static const int v = [] {
    const char* e = getenv("UOT_DENSE_BLOCKS");
    return e ? atoi(e) : 0;
  }();
  return v;
}

// block targets the matrix-core product's tuner times (the first is the
// untuned default): 4 blocks of 256 rows are resident per compute unit, so
// 1024 fill the chip once; where the last column chunk of a split or the last
// round of blocks falls depends on the sizes
constexpr int kMfTargets[] = {1024, 1280, 1536, 2048};
constexpr int kMfNTargets = 4;

void dense_config(Plan& P, int side) {
  const int64_t Nr = side == 0 ? P.N : P.M;
  const int64_t Mc = side == 0 ? P.M : P.N;
  // rows per thread (the matrix-core kernel: mf_groups / 4, with mf_groups
  // row groups of 16 per wave)
  // (the WF cost: one row per thread, so a wave's box is that of 64 rows)
  const int R = P.dense_mf ? P.mf_groups / 4 : (P.dtype == UOT_F32 && P.cost.kind != UOT_COST_WF) ? 2 : 1;
  const int64_t rt = (Nr + 256 * R - 1) / (256 * R);
  // blocks to aim for: 2048 (8 resident per compute unit), 1024 for the
  // matrix-core product (its column chunks after the first cost one pass,
  // so longer column ranges per block pay; the tuner may pick up to 2048);
  // UOT_DENSE_BLOCKS overrides the target of the factored kernels
  const int fac_blocks = dense_blocks_env();
  // the matrix-core product: fewer splits to merge; the WF cost: more, as
  // the pairs within the cut concentrate in few (row block, split) pairs and
  // smaller splits spread them over more compute units (blocks and merges
  // skip the pairs whose boxes are beyond the cut)
  int64_t target = P.dense_mf ? (P.mf_target[side] > 0 ? P.mf_target[side] : kMfTargets[0])
                              : (P.cost.kind == UOT_COST_WF ? 16384 : 2048);
  if ((P.dense_tf || P.dense_mf || P.cost.kind == UOT_COST_WF) && fac_blocks > 0) target = fac_blocks;
  int64_t sp = (target + rt - 1) / rt;
  const int64_t maxsp = (Mc + 31) / 32;
  if (sp > maxsp) sp = maxsp;
  if (sp < 1) sp = 1;
  int64_t cps = (Mc + sp - 1) / sp;
  cps = (cps + 31) / 32 * 32;
  sp = (Mc + cps - 1) / cps;
  P.R[side] = R;
  P.splits[side] = (int)sp;
  P.cps[side] = cps;
}

int make_plan(Plan& P, int dtype, const uot_geom& g, int nb, int nst, int grid_kernel = 0, double eps_min = 0.0,
              int dense_kernel = 1) {
  if (dtype != UOT_F32 && dtype != UOT_F64) return fail(UOT_E_INVALID, "dtype must be UOT_F32 or UOT_F64");
  if (dense_kernel < 0 || dense_kernel > 4) return fail(UOT_E_INVALID, "dense_kernel must be 0 .. 4");
  if (grid_kernel < 0 || grid_kernel > 4) return fail(UOT_E_INVALID, "grid_kernel must be 0 .. 4");
  P.gk = grid_kernel == 0 ? (dtype == UOT_F32 ? 2 : 1) : grid_kernel;
  P.dtype = dtype;
  P.esz = dtype == UOT_F32 ? 4 : 8;
  P.geom = g.kind;
  P.dim = g.dim;
  P.nb = nb;
  P.nst = nst;
  if (g.dim < 1 || g.dim > 3) return fail(UOT_E_UNSUPPORTED, "dim must be 1, 2 or 3");
  if (g.cost != UOT_COST_SQEUCLID && g.cost != UOT_COST_WF) return fail(UOT_E_INVALID, "unknown cost kind");
  if (g.cost == UOT_COST_WF) {
    if (!(g.cut > 0 && std::isfinite(g.cut))) return fail(UOT_E_INVALID, "the WF cost needs a finite cut > 0");
    if (g.kind == UOT_GEOM_GRID && g.dim != 1)
      return fail(UOT_E_UNSUPPORTED, "the WF cost is not separable: grids need dim = 1");
  }
  P.cost.kind = g.cost;
  P.cost.cut = g.cost == UOT_COST_WF ? g.cut : 0.0;
  if (g.kind == UOT_GEOM_POINTS) {
    if (g.N < 1 || g.M < 1) return fail(UOT_E_INVALID, "N and M must be >= 1");
    if (!g.x || !g.y) return fail(UOT_E_INVALID, "point coordinates x and y are required");
    if (nb != 1) return fail(UOT_E_UNSUPPORTED, "several fields need a grid geometry");
    P.N = g.N;
    P.M = g.M;
    // default: the BF16 x 3 matrix-core product where it applies (FP32, squared
    // Euclidean cost) and both clouds have 2048 points or more (below that
    // its per-block set-up outweighs the pairs), the direct product otherwise
    if (dense_kernel == 0)
      dense_kernel = dtype == UOT_F32 && g.cost == UOT_COST_SQEUCLID && std::min(g.N, g.M) >= 2048 ? 4 : 1;
    P.dense_tf = dense_kernel == 2;
    P.dense_mf = dense_kernel == 3 || dense_kernel == 4;
    P.mf_split = dense_kernel == 4;
    static const int mf_groups = [] {
      const char* e = getenv("UOT_DENSE_MF_GROUPS");
      return e && atoi(e) == 8 ? 8 : 4;
    }();
    P.mf_groups = mf_groups;
    if ((P.dense_tf || P.dense_mf) && (dtype != UOT_F32 || g.cost != UOT_COST_SQEUCLID))
      return fail(UOT_E_UNSUPPORTED, "the factored dense products take FP32 and the squared Euclidean cost");
  } else if (g.kind == UOT_GEOM_GRID) {
    int64_t sz = 1;
    for (int k = 0; k < g.dim; ++k) {
      if (g.n[k] < 1 || g.n[k] > 4096) return fail(UOT_E_UNSUPPORTED, "grid axes must have 1..4096 cells");
      if (!(g.h[k] > 0)) return fail(UOT_E_INVALID, "grid spacing must be > 0");
      P.n[k] = g.n[k];
      P.h[k] = g.h[k];
      sz *= g.n[k];
    }
    if (g.dim == 3 && (int64_t)nb * g.n[0] > 65535) return fail(UOT_E_UNSUPPORTED, "fields x n[0] must be <= 65535");
    P.N = P.M = sz;
    for (int k = 0; k < g.dim; ++k) {
      const double c = eps_min > 0 ? g.h[k] * g.h[k] * kLog2e / eps_min : INFINITY;
      // the tile factorization is that of the Gaussian kernel
      P.tf_axis[k] = P.gk >= 2 && dtype == UOT_F32 && g.n[k] % 16 == 0 && c <= kTfMaxC && g.cost == UOT_COST_SQEUCLID;
      P.tf16_axis[k] = P.tf_axis[k] && (P.gk == 3 || P.gk == 4) && c <= kTf16MaxC;
      P.band[k] = (int)g.n[k];
      if (g.cost == UOT_COST_WF) P.band[k] = (int)std::min<double>((double)g.n[k], std::ceil(g.cut / g.h[k]));
    }
    if (g.dim == 1) P.split1d = grid_contig_splits((int)g.n[0], nb, P.band[0]);
  } else {
    return fail(UOT_E_INVALID, "unknown geometry kind");
  }
  const size_t e = P.esz;
  const int64_t F = (int64_t)nb * std::max(P.N, P.M);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  P.o_ctrl = take(sizeof(Ctrl));
  P.o_logp = take(e * nb * P.N);
  P.o_logq = take(e * nb * P.M);
  P.o_logdx = take(e * P.N);
  P.o_logdy = take(e * P.M);
  P.o_wu = take(e * nb * P.N);
  P.o_wv = take(e * nb * P.M);
  P.o_t1 = take(e * F);
  P.o_t2 = take(e * F);
  P.o_t3 = take(e * F);
  if (P.geom == UOT_GEOM_POINTS) {
    // partials sized for every product kernel, so one workspace size query
    // covers every dense_kernel choice; the plan's own kernel is set last
    int64_t np = 0;
    const Plan keep = P;
    for (int pass = 0; pass < 5; ++pass) {
      P.dense_tf = pass == 1;
      P.dense_mf = pass >= 2;
      P.mf_groups = pass == 2 ? 8 : 4;
      if (pass == 4) P = keep;
      // every block target the matrix-core tuner may pick
      for (int k = 0; k < (P.dense_mf ? kMfNTargets : 1); ++k) {
        P.mf_target[0] = P.mf_target[1] = P.dense_mf ? kMfTargets[k] : 0;
        dense_config(P, 0);
        dense_config(P, 1);
        np = std::max(np, std::max((int64_t)P.splits[0] * P.N, (int64_t)P.splits[1] * P.M));
      }
    }
    P.mf_target[0] = P.mf_target[1] = 0;
    dense_config(P, 0);
    dense_config(P, 1);
    P.o_pm = take(e * np);
    P.o_ps = take(e * np);
    P.np_pw = np;
    P.nparts_x = (int)((P.N + 255) / 256);
  } else {
    const size_t np = P.dim == 1 && P.split1d > 1 ? (size_t)P.split1d * nb * P.N : 0;
    P.o_pm = take(e * np);
    P.o_ps = take(e * np);
    P.nparts_x = grid_final_parts(P);
  }
  // room for either pass kind, so a size query without eps fits every solve
  const int parts_room = P.geom == UOT_GEOM_GRID
                             ? std::max(grid_final_parts_for(P, false), P.n[0] % 16 == 0 ? grid_final_parts_for(P, true) : 0)
                             : P.nparts_x;
  P.o_parts = take(sizeof(ResPart) * std::max(parts_room, 1));
  P.nparts_y = P.geom == UOT_GEOM_GRID ? P.nparts_x : (int)((P.M + 255) / 256);
  P.o_mass = take(2 * e * std::max(std::max(parts_room, P.nparts_y), 1));
  for (int k = 0; k < 3; ++k) P.o_gtab[k] = take(P.geom == UOT_GEOM_GRID && k < P.dim ? e * (2 * P.n[k] - 1) * nst : 0);
  int64_t gmax = 1;
  for (int k = 0; k < P.dim; ++k) gmax = std::max(gmax, 2 * P.n[k] - 1);
  P.o_gcost = take(P.geom == UOT_GEOM_GRID ? e * gmax : 0);
  P.obj_doubles = 4 * ((std::max(P.N, P.M) + 255) / 256) * 2 + 8 * ((std::max(P.N, P.M) + 255) / 256);
  P.o_obj = take(sizeof(double) * P.obj_doubles);
  P.o_scal = take(sizeof(double) * 8);
  // Morton-ordered copies of point clouds (tile-factored product)
  const bool pts = P.geom == UOT_GEOM_POINTS;
  P.o_xs = take(pts ? e * P.dim * P.N : 0);
  P.o_ys = take(pts ? e * P.dim * P.M : 0);
  P.o_permx = take(pts ? sizeof(int32_t) * P.N : 0);
  P.o_permy = take(pts ? sizeof(int32_t) * P.M : 0);
  P.o_code = take(pts ? sizeof(uint32_t) * std::max(P.N, P.M) : 0);
  P.o_box = take(pts ? e * 6 : 0);
  P.o_us = take(pts ? e * P.N : 0);
  P.o_vs = take(pts ? e * P.M : 0);
  // row maxima the matrix-core product leaves for the next product of the
  // same side (two sides)
  P.o_pw = take(pts ? sizeof(float) * 2 * P.np_pw : 0);
  // WF points: the work lists of both sides (boxes, masks, units, counts)
  // and the unit partials (shared by the sides, which run one after the other)
  const bool wf = pts && P.cost.kind == UOT_COST_WF;
  for (int h = 0; h < 2; ++h) {
    const WfShape sh(h == 0 ? P.N : P.M, h == 0 ? P.M : P.N);
    P.o_wfl[h] = take(wf ? e * 6 * (sh.nrw + sh.ngr) + 8 * sh.slots() + 4 * sh.words() + 4 * sh.nrw + 512 : 0);
    P.wf_slots = std::max(P.wf_slots, wf ? sh.slots() : 0);
  }
  P.o_wfpart = take(wf ? 2 * e * 64 * P.wf_slots : 0);
  P.total = o;
  return UOT_OK;
}

template <typename T> T* at(char* ws, size_t off) { return reinterpret_cast<T*>(ws + off); }

int check_ws(const Plan& P, void* ws, size_t bytes) {
  if (!ws) return fail(UOT_E_WORKSPACE, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(UOT_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < P.total) return fail(UOT_E_WORKSPACE, "workspace too small: need " + std::to_string(P.total));
  return UOT_OK;
}

Ctrl make_ctrl(double eps, double eps0, int stages, int ips, double tol, int64_t max_iter) {
  Ctrl c{};
  const bool anneal = eps0 > eps && stages > 0 && ips > 0;
  c.n_stages = anneal ? stages : 0;
  c.iters_per_stage = anneal ? ips : 0;
  if (anneal) {
    const double f = std::pow(eps / eps0, 1.0 / stages);
    for (int k = 0; k < stages; ++k) c.eps_tab[k] = eps0 * std::pow(f, k);
  }
  c.eps_tab[c.n_stages] = eps;
  c.stage[0] = c.stage[1] = 0;
  c.eps[0] = c.eps[1] = c.eps_tab[0];
  c.tol = tol;
  c.max_iter = max_iter;
  c.iter = 0;
  c.stop = 0;
  c.skip[0] = c.skip[1] = 0;
  c.status = 1;
  c.res = INFINITY;
  return c;
}


// ---------------------------------------------------------------------------
// Gibbs-product chains
// ---------------------------------------------------------------------------
template <typename T> struct Bufs {
  Ctrl* ctrl;
  T *logp, *logq, *logdx, *logdy, *wu, *wv, *t1, *t2, *t3, *pm, *ps;
  ResPart* parts;
  T* gtab[3];
  T* gcost;
  double* obj;
  double* scal;
  T *mass_m, *mass_s;     // mass partials of Algorithm 4 (Y epilogue)
  float* pw;              // points: row maxima of the two sides' products
  WfLists<T> wfl[2];      // WF points: work lists per side
  T *wfpm, *wfps;         // WF points: unit partials
};

template <typename T> Bufs<T> carve(const Plan& P, char* ws) {
  Bufs<T> b;
  b.ctrl = at<Ctrl>(ws, P.o_ctrl);
  b.logp = at<T>(ws, P.o_logp);
  b.logq = at<T>(ws, P.o_logq);
  b.logdx = at<T>(ws, P.o_logdx);
  b.logdy = at<T>(ws, P.o_logdy);
  b.wu = at<T>(ws, P.o_wu);
  b.wv = at<T>(ws, P.o_wv);
  b.t1 = at<T>(ws, P.o_t1);
  b.t2 = at<T>(ws, P.o_t2);
  b.t3 = at<T>(ws, P.o_t3);
  b.pm = at<T>(ws, P.o_pm);
  b.ps = at<T>(ws, P.o_ps);
  b.pw = at<float>(ws, P.o_pw);
  for (int h = 0; h < 2; ++h) {
    const WfShape sh(h == 0 ? P.N : P.M, h == 0 ? P.M : P.N);
    char* base = ws + P.o_wfl[h];
    b.wfl[h].rbox = reinterpret_cast<T*>(base);
    b.wfl[h].gbox = b.wfl[h].rbox + 6 * sh.nrw;
    char* q = reinterpret_cast<char*>(b.wfl[h].gbox + 6 * sh.ngr);
    q = ws + align_up((size_t)(q - ws));
    b.wfl[h].units = reinterpret_cast<int2*>(q);
    b.wfl[h].mask = reinterpret_cast<uint32_t*>(b.wfl[h].units + sh.slots());
    b.wfl[h].ucnt = reinterpret_cast<int*>(b.wfl[h].mask + sh.words());
    b.wfl[h].umax = b.wfl[h].ucnt + sh.nrw;
  }
  b.wfpm = at<T>(ws, P.o_wfpart);
  b.wfps = b.wfpm + 64 * P.wf_slots;
  b.parts = at<ResPart>(ws, P.o_parts);
  for (int k = 0; k < 3; ++k) b.gtab[k] = at<T>(ws, P.o_gtab[k]);
  b.gcost = at<T>(ws, P.o_gcost);
  b.obj = at<double>(ws, P.o_obj);
  b.scal = at<double>(ws, P.o_scal);
  b.mass_m = at<T>(ws, P.o_mass);
  b.mass_s = b.mass_m + std::max(std::max(P.nparts_x, P.nparts_y), 1);
  P.split_pm = b.pm;
  P.split_ps = b.ps;
  return b;
}

// separable grid product on nb fields: input w (log2 units), per-axis tables
// (direct passes) or the tile-factored MFMA pass where the plan selects it
template <typename T>
void contig_pass(const Plan& P, int axis, const T* w, int64_t A, T* const* tabs, int side, Ctrl* c,
                 const EpiArgs<T>& ep, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (use_tf(P, axis)) {
      timed(0, [&] { launch_grid_tf(w, A, (int)P.n[axis], 1, false, P.tf16_axis[axis], P.h[axis], side, c, ep, s); });
      return;
    }
  }
  if (P.dim == 1 && P.split1d > 1) {
    // few long lines: tap slices, then the merge with the epilogue
    T* pm = static_cast<T*>(P.split_pm);
    T* ps = static_cast<T*>(P.split_ps);
    timed(0, [&] {
      launch_grid_contig_split<T>(w, A, (int)P.n[axis], tabs[axis], side, c, P.band[axis], P.split1d, pm, ps, s);
    });
    timed(1, [&] { launch_dense_epi<T>(pm, ps, P.split1d, A * P.n[axis], side, c, ep, s); });
    return;
  }
  timed(0, [&] { launch_grid_contig<T>(w, A, (int)P.n[axis], tabs[axis], side, c, ep, P.band[axis], s); });
}

template <typename T>
void strided_pass(const Plan& P, int axis, const T* w, int64_t A, int64_t B, T* const* tabs, int side, Ctrl* c,
                  const EpiArgs<T>& ep, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (use_tf(P, axis)) {
      timed(1, [&] { launch_grid_tf(w, A, (int)P.n[axis], B, true, P.tf16_axis[axis], P.h[axis], side, c, ep, s); });
      return;
    }
  }
  timed(1, [&] { launch_grid_strided<T>(w, A, (int)P.n[axis], B, tabs[axis], side, c, ep, s); });
}

// control step hosted by the first pass of a chain (see k_control)
struct CtlHost {
  Ctrl* c = nullptr;
  const ResPart* parts = nullptr;
  int nparts = 0;
  double* hist = nullptr;
};

template <typename T>
void grid_chain(const Plan& P, const T* w, T* const* tabs, int side, Ctrl* c, const EpiArgs<T>& ep, T* tmp1,
                T* tmp2, hipStream_t s, const CtlHost* host = nullptr) {
  const int64_t nb = P.nb;
  // first pass (no epilogue on 2 or 3 axes): writes tmp1 and may host the
  // control step; only such a pass may, as an epilogue reads the slot the
  // control step writes
  EpiArgs<T> first{};
  first.mode = EPI_RAW;
  first.out = tmp1;
  if (host) {
    first.host_ctl = host->c;
    first.host_parts = host->parts;
    first.host_nparts = host->nparts;
    first.host_hist = host->hist;
  }
  if (P.dim == 1) {
    contig_pass<T>(P, 0, w, nb, tabs, side, c, ep, s);
  } else if (P.dim == 2) {
    contig_pass<T>(P, 1, w, nb * P.n[0], tabs, side, c, first, s);
    strided_pass<T>(P, 0, tmp1, nb, P.n[1], tabs, side, c, ep, s);
  } else {
    contig_pass<T>(P, 2, w, nb * P.n[0] * P.n[1], tabs, side, c, first, s);
    EpiArgs<T> mid{};
    mid.mode = EPI_RAW;
    mid.out = tmp2;
    strided_pass<T>(P, 1, tmp1, nb * P.n[0], P.n[2], tabs, side, c, mid, s);
    strided_pass<T>(P, 0, tmp2, nb, P.n[1] * P.n[2], tabs, side, c, ep, s);
  }
}

// WF point clouds: the work lists of both sides (the (row wave, column
// group) pairs within the cut and their units), once per call (the geometry
// is fixed); P.wfl tells the products of this call to run on them
template <typename T>
int wf_lists(Plan& P, const uot_geom& g, Bufs<T>& B, hipStream_t s) {
  if (P.geom != UOT_GEOM_POINTS || P.cost.kind != UOT_COST_WF) return UOT_OK;
  const T* x = static_cast<const T*>(g.x);
  const T* y = static_cast<const T*>(g.y);
  launch_wf_lists<T>(x, P.N, y, P.M, P.dim, P.cost.cut, B.wfl[0], s);
  launch_wf_lists<T>(y, P.M, x, P.N, P.dim, P.cost.cut, B.wfl[1], s);
  // the launch size of the products: the largest unit count of a row wave
  for (int h = 0; h < 2; ++h) HIP_TRY(hipMemcpyAsync(&P.wf_umax[h], B.wfl[h].umax, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  P.wfl = true;
  return UOT_OK;
}

// the matrix-core products' tile skipping, and their pair count in timed
// solves (into the control block)
MfSkip mf_skip(Ctrl* c, bool count) {
  MfSkip k;
  k.on = tile_skip_enabled() ? 1 : 0;
  k.pairs = count && g_timer ? &c->pairs : nullptr;
  return k;
}

// dense point-cloud product for one side; returns the residual partial count
template <typename T>
void dense_half(const Plan& P, const uot_geom& g, int side, const T* w_cols, Bufs<T>& B, Ctrl* c,
                const EpiArgs<T>& ep, hipStream_t s) {
  const int half = side & 1;
  const T* rows = static_cast<const T*>(half == 0 ? g.x : g.y);
  const T* cols = static_cast<const T*>(half == 0 ? g.y : g.x);
  const int64_t Nr = half == 0 ? P.N : P.M;
  const int64_t Mc = half == 0 ? P.M : P.N;
  timed(0, [&] {
    if constexpr (std::is_same<T, float>::value) {
      if (P.dense_tf) {
        launch_dense_tf(P.dim, rows, Nr, cols, w_cols, Mc, P.splits[half], P.cps[half], B.pm, B.ps, side, c, s);
        return;
      }
      if (P.dense_mf) {
        launch_dense_mf(P.dim, P.mf_groups, P.mf_split, rows, Nr, cols, w_cols, Mc, P.splits[half], P.cps[half], B.pm, B.ps,
                        B.pw + half * P.np_pw, side, c, mf_skip(c, true), s);
        return;
      }
    }
    if (P.wfl) {
      launch_wf_lse<T>(P.dim, rows, Nr, cols, w_cols, Mc, P.cost.cut, B.wfl[half], P.wf_umax[half], B.wfpm, B.wfps,
                       side, c, s);
      return;
    }
    launch_dense_lse<T>(P.dim, P.R[half], rows, Nr, cols, w_cols, Mc, P.splits[half], P.cps[half], B.pm, B.ps, side,
                        c, P.cost, s);
  });
  timed(1, [&] {
    if (P.wfl) launch_wf_epi<T>(B.wfpm, B.wfps, B.wfl[half], Nr, Mc, side, c, ep, s);
    else launch_dense_epi<T>(B.pm, B.ps, P.splits[half], Nr, side, c, ep, s);
  });
}

template <typename T>
EpiArgs<T> prox_epi(T* pot, T* wnext, const T* logp, const T* logd, T* lse_out, ResPart* part, int64_t size,
                    const uot_div& F) {
  EpiArgs<T> ep{};
  ep.mode = EPI_PROX;
  ep.pot = pot;
  ep.wnext = wnext;
  ep.logp = logp;
  ep.logd = logd;
  ep.lse_out = lse_out;
  ep.part = part;
  ep.size = size;
  ep.F = to_dev(F);
  return ep;
}

// one half-step (X: side 0 reads wv, writes u / wu; Y: side 1 reads wu, writes
// v / wv); bit 1 of side is the parity of the iteration
template <typename T>
void half_step(const Plan& P, const uot_problem& pb, int side, Bufs<T>& B, T* pot, T* lse_out, bool with_res,
               hipStream_t s, const CtlHost* host = nullptr, bool mass = false) {
  if ((side & 1) == 0) {
    EpiArgs<T> ep = prox_epi<T>(pot, B.wu, B.logp, B.logdx, lse_out, with_res ? B.parts : nullptr, P.N, pb.F1);
    if (P.geom == UOT_GEOM_GRID) grid_chain<T>(P, B.wv, B.gtab, side, B.ctrl, ep, B.t1, B.t2, s);
    else dense_half<T>(P, pb.geom, side, B.wv, B, B.ctrl, ep, s);
  } else {
    EpiArgs<T> ep = prox_epi<T>(pot, B.wv, B.logq, B.logdy, lse_out, nullptr, P.M, pb.F2);
    if (mass) {
      ep.mass_m = B.mass_m;
      ep.mass_s = B.mass_s;
    }
    if (P.geom == UOT_GEOM_GRID) grid_chain<T>(P, B.wu, B.gtab, side, B.ctrl, ep, B.t1, B.t2, s, host);
    else dense_half<T>(P, pb.geom, side, B.wu, B, B.ctrl, ep, s);
  }
}

int validate_problem(const uot_problem* pb) {
  if (!pb) return fail(UOT_E_INVALID, "problem is NULL");
  if (!pb->p || !pb->q || !pb->dx || !pb->dy) return fail(UOT_E_INVALID, "p, q, dx, dy are required");
  int r = check_div(pb->F1, "F1");
  if (r) return r;
  return check_div(pb->F2, "F2");
}

int validate_params(const uot_params* pr, bool batch = false) {
  if (!pr) return fail(UOT_E_INVALID, "params is NULL");
  if (pr->rebalance_at < 0 || pr->rebalance_at == 1)
    return fail(UOT_E_INVALID, "rebalance_at must be 0 (off) or >= 2 (the start takes uot_batch_balance)");
  if (pr->rebalance_at != 0 && !batch)
    return fail(UOT_E_UNSUPPORTED, "rebalance_at applies to ragged batches only");
  if (!(pr->eps > 0 && std::isfinite(pr->eps))) return fail(UOT_E_INVALID, "eps must be finite and > 0");
  if (pr->max_iter < 1) return fail(UOT_E_INVALID, "max_iter must be >= 1");
  if (!(pr->tol >= 0)) return fail(UOT_E_INVALID, "tol must be >= 0");
  if (pr->eps_stages < 0 || pr->eps_stages > kMaxStages) return fail(UOT_E_INVALID, "eps_stages must be in [0, 32]");
  if (pr->check_every < 0) return fail(UOT_E_INVALID, "check_every must be >= 0");
  return UOT_OK;
}

// polling interval in iterations, rounded up to even: the iterations of a
// captured chunk alternate in parity, so every replay starts at an even one
inline int even_chunk(int check_every) {
  const int c = check_every > 0 ? check_every : 50;
  return c + (c & 1);
}

// a captured chunk kept across solves whose launches are the same (the steps
// of a gradient flow): captured by the first solve, replayed by the others
struct GraphCache {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~GraphCache() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// drive iterations until the device sets stop; `iteration(par)` enqueues one
// iteration of parity par.  With a second phase (`iteration2`, non-null
// `final_tol`), a stop with status 0 ends phase one (whose control block
// tolerance was looser): the solve resumes at `final_tol` with iteration2.
template <typename F, typename F2 = std::remove_reference_t<F>>
int run_loop(uot_ctx* ctx, Ctrl* dctrl, const uot_params* pr, F&& iteration, uot_result* res,
             F2* iteration2 = nullptr, const double* final_tol = nullptr, GraphCache* cache = nullptr) {
  hipStream_t s = ctx->work;
  const int chunk = even_chunk(pr->check_every);
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  KTimer timer;
  timer.s = s;
  const bool timing = pr->kernel_ms != nullptr;
  if (timing) g_timer = &timer;
  struct Reset {
    ~Reset() { g_timer = nullptr; }
  } reset_timer;
  auto capture = [&](auto& it) -> int {
    if (!pr->use_graph || timing) return UOT_OK;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < chunk; ++k) it(k & 1);
    HIP_TRY(hipStreamEndCapture(s, &graph));
    HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    return UOT_OK;
  };
  auto release = [&] {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  };
  int rc = UOT_OK;
  if (cache && cache->exec && pr->use_graph && !timing) {
    exec = cache->exec;
    graph = cache->graph;
  } else {
    rc = capture(iteration);
    if (rc) return rc;
  }
  bool second = false;
  auto t0 = std::chrono::steady_clock::now();
  int64_t launched = 0;
  while (true) {
    if (exec) {
      if (hipGraphLaunch(exec, s) != hipSuccess) { rc = fail(UOT_E_HIP, "hipGraphLaunch failed"); break; }
    } else {
      for (int k = 0; k < chunk; ++k) {
        if (second) (*iteration2)(k & 1);
        else iteration(k & 1);
      }
    }
    launched += chunk;
    if (hipMemcpyAsync(ctx->pinned, dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(UOT_E_HIP, std::string("iteration chunk failed: ") + hipGetErrorString(hipGetLastError()));
      break;
    }
    if (timing) timer.collect();
    if (ctx->pinned->stop) {
      if (iteration2 && !second && ctx->pinned->status == 0) {
        second = true;
        // a phase-one graph taken from the cache is destroyed here: the cache
        // must not keep its handles
        if (cache && cache->exec == exec) {
          cache->exec = nullptr;
          cache->graph = nullptr;
        }
        release();
        launch_ctrl_resume(dctrl, *final_tol, s);
        if ((rc = capture(*iteration2))) break;
        continue;
      }
      break;
    }
    if (launched > pr->max_iter + 2 * chunk) { rc = fail(UOT_E_HIP, "control block did not stop"); break; }
  }
  if (timing) {
    for (int k = 0; k < 4; ++k) {
      pr->kernel_ms[k] = timer.ms[k];
      if (pr->kernel_launches) pr->kernel_launches[k] = timer.count[k];
    }
    // class [3]: the matrix-core products' pair evaluations (the control
    // block as copied back after the last chunk)
    if (pr->kernel_launches) pr->kernel_launches[3] = (int64_t)ctx->pinned->pairs;
  }
  auto t1 = std::chrono::steady_clock::now();
  if (cache && !second) {
    // keep the phase-one graph for the next solve
    cache->exec = exec;
    cache->graph = graph;
  } else {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
  if (rc) return rc;
  res->iters = ctx->pinned->iter;
  res->residual = ctx->pinned->res;
  res->du_inf = ctx->pinned->du;
  res->status = ctx->pinned->status;
  res->elapsed_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  return UOT_OK;
}

// The asynchronous form of run_loop: enqueue ceil(max_iter / chunk) chunks
// without polling (the iterations after the device stops are no-ops: each
// kernel of a skipped iteration returns at once), then a stream-ordered copy
// of the control block to the pinned mirror.  The context keeps the chunk
// graph until uot_sync_result.
template <typename F>
int run_async(uot_ctx* ctx, Ctrl* dctrl, const uot_params* pr, F&& iteration) {
  hipStream_t s = ctx->work;
  const int chunk = even_chunk(pr->check_every);
  const int64_t n = (pr->max_iter + chunk - 1) / chunk;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (pr->use_graph) {
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < chunk; ++k) iteration(k & 1);
    HIP_TRY(hipStreamEndCapture(s, &graph));
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(UOT_E_HIP, "hipGraphInstantiate failed");
    }
  }
  ctx->pending = true;   // from here the context owns the graph
  ctx->pending_graph = graph;
  ctx->pending_exec = exec;
  HIP_TRY(hipEventRecord(ctx->ev_t0, s));
  for (int64_t k = 0; k < n; ++k) {
    if (exec) {
      HIP_TRY(hipGraphLaunch(exec, s));
    } else {
      for (int j = 0; j < chunk; ++j) iteration(j & 1);
    }
  }
  HIP_TRY(hipEventRecord(ctx->ev_t1, s));
  HIP_TRY(hipMemcpyAsync(ctx->pinned, dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
  return UOT_OK;
}

// Morton-ordered copies of both clouds for the tile-factored dense product:
// coordinates gathered into the workspace (permutations kept there), the
// problem returned points at the copies
template <typename T>
uot_problem sorted_points(const Plan& P, const uot_problem& pb, char* ws, hipStream_t s) {
  T* xs = at<T>(ws, P.o_xs);
  T* ys = at<T>(ws, P.o_ys);
  int32_t* px = at<int32_t>(ws, P.o_permx);
  int32_t* py = at<int32_t>(ws, P.o_permy);
  uint32_t* code = at<uint32_t>(ws, P.o_code);
  T* box = at<T>(ws, P.o_box);
  const T* x = static_cast<const T*>(pb.geom.x);
  const T* y = static_cast<const T*>(pb.geom.y);
  launch_spatial_order<T>(x, P.N, P.dim, box, code, px, s);
  launch_spatial_order<T>(y, P.M, P.dim, box, code, py, s);
  launch_gather<T>(x, px, P.N, P.dim, xs, s);
  launch_gather<T>(y, py, P.M, P.dim, ys, s);
  uot_problem q = pb;
  q.geom.x = xs;
  q.geom.y = ys;
  return q;
}

// log of a caller array, in the caller's order or gathered by perm
template <typename T>
void log_into(const void* src, T* dst, int64_t n, int zero_is_ninf, const int32_t* perm, T* tmp, hipStream_t s) {
  if (!perm) {
    launch_log<T>(static_cast<const T*>(src), dst, n, zero_is_ninf, s);
    return;
  }
  launch_log<T>(static_cast<const T*>(src), tmp, n, zero_is_ninf, s);
  launch_gather<T>(tmp, perm, n, 1, dst, s);
}

// total-mass penalty of Algorithm 4: F3 on the one-point space, log m0
struct MassOpt {
  DivDev F3;
  double log_m0;
};

// The matrix-core product's column splits, per side: each block target of
// kMfTargets is timed once per context and product shape (a cold launch, then
// the mean of 3 warm ones; rows, columns and column weights log dy / log dx of
// the solve, whose values do not change the work), and the fastest is kept.
// Leaves the row maxima of the side's workspace to be reset by the caller.
template <typename T>
int tune_dense_mf(uot_ctx* ctx, Plan& P, const uot_geom& g, Bufs<T>& B, hipStream_t s) {
  if constexpr (!std::is_same<T, float>::value) {
    return UOT_OK;
  } else {
    if (!P.dense_mf || dense_blocks_env() > 0) return UOT_OK;
    for (int half = 0; half < 2; ++half) {
      const int64_t Nr = half == 0 ? P.N : P.M;
      const int64_t Mc = half == 0 ? P.M : P.N;
      const std::string key = std::to_string(P.dim) + ":" + std::to_string(Nr) + ":" + std::to_string(Mc) + ":" +
                              std::to_string(P.mf_groups) + ":" + std::to_string((int)P.mf_split);
      const auto found = ctx->dense_tuned.find(key);
      if (found != ctx->dense_tuned.end()) {
        P.mf_target[half] = found->second;
        dense_config(P, half);
        continue;
      }
      const float* rows = static_cast<const float*>(half == 0 ? g.x : g.y);
      const float* cols = static_cast<const float*>(half == 0 ? g.y : g.x);
      const float* wc = half == 0 ? B.logdy : B.logdx;
      float* pw = B.pw + half * P.np_pw;
      // the two timing events, released on every return
      struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
          for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
        }
      } ev;
      HIP_TRY(hipEventCreate(&ev.e[0]));
      HIP_TRY(hipEventCreate(&ev.e[1]));
      hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
      int best = kMfTargets[0], last_sp = -1;
      float best_t = 0.f;
      for (int k = 0; k < kMfNTargets; ++k) {
        P.mf_target[half] = kMfTargets[k];
        dense_config(P, half);
        if (P.splits[half] == last_sp) continue;
        last_sp = P.splits[half];
        auto launch = [&] {
          launch_dense_mf(P.dim, P.mf_groups, P.mf_split, rows, Nr, cols, wc, Mc, P.splits[half], P.cps[half], B.pm,
                          B.ps, pw, half, B.ctrl, mf_skip(B.ctrl, false), s);
        };
        HIP_TRY(hipMemsetAsync(pw, 0xFF, sizeof(float) * P.np_pw, s));
        launch();
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) launch();
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        if (k == 0 || t < best_t) {
          best_t = t;
          best = kMfTargets[k];
        }
      }
      HIP_TRY(hipGetLastError());
      P.mf_target[half] = best;
      dense_config(P, half);
      ctx->dense_tuned[key] = best;
    }
    return UOT_OK;
  }
}

template <typename T>
int solve_t(uot_ctx* ctx, const uot_problem* pb, const uot_params* pr, T* u, T* v, char* ws, size_t wsb,
            uot_result* res, int nb = 1, const MassOpt* mass = nullptr, double* log_z = nullptr,
            bool async = false) {
  Plan P;
  const bool anneal = pr->eps0 > pr->eps && pr->eps_stages > 0 && pr->iters_per_stage > 0;
  int rc = make_plan(P, pb->dtype, pb->geom, nb, anneal ? pr->eps_stages + 1 : 1, pr->grid_kernel, pr->eps,
                     pr->dense_kernel);
  if (rc) return rc;
  if ((rc = check_ws(P, ws, wsb))) return rc;
  if (!u || !v) return fail(UOT_E_INVALID, "u and v output buffers are required");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  Bufs<T> B = carve<T>(P, ws);
  // the iteration runs on pbs into uo / vo: the caller's problem and outputs,
  // or Morton-ordered copies whose potentials are scattered back at the end
  uot_problem pbs = *pb;
  T* uo = u;
  T* vo = v;
  const int32_t* px = nullptr;
  const int32_t* py = nullptr;
  if (P.sorted()) {
    pbs = sorted_points<T>(P, *pb, ws, s);
    px = at<int32_t>(ws, P.o_permx);
    py = at<int32_t>(ws, P.o_permy);
    uo = at<T>(ws, P.o_us);
    vo = at<T>(ws, P.o_vs);
  }
  // mixed precision: FP16 passes down to kMixedSwitchTol, then FP32 passes
  const bool mixed = P.gk == 4 && has_tf16(P) && pr->tol < kMixedSwitchTol;
  if (async && mixed)
    return fail(UOT_E_UNSUPPORTED, "the mixed-precision grid passes switch under host control: solve synchronously");
  if (async && pr->kernel_ms) return fail(UOT_E_INVALID, "timed solves run synchronously");
  const double tol1 = mixed ? kMixedSwitchTol : pr->tol;
  Ctrl init = make_ctrl(pr->eps, pr->eps0, pr->eps_stages, pr->iters_per_stage, tol1, pr->max_iter);
  launch_ctrl_init(B.ctrl, init, s);
  log_into<T>(pb->p, B.logp, nb * P.N, 1, px, B.t1, s);
  log_into<T>(pb->q, B.logq, nb * P.M, 1, py, B.t1, s);
  log_into<T>(pb->dx, B.logdx, P.N, 0, px, B.t1, s);
  log_into<T>(pb->dy, B.logdy, P.M, 0, py, B.t1, s);
  if (P.geom == UOT_GEOM_GRID)
    for (int k = 0; k < P.dim; ++k) launch_gtab<T>(B.gtab[k], (int)P.n[k], P.h[k], B.ctrl, P.nst, P.cost, s);
  launch_init_pot<T>(nullptr, B.logdx, uo, nullptr, nb * P.N, P.N, B.ctrl, 0, s);
  const T* v0 = static_cast<const T*>(pr->v0);
  if (v0 && py) {
    launch_gather<T>(v0, py, P.M, 1, vo, s);
    v0 = vo;
  }
  launch_init_pot<T>(v0, B.logdy, vo, B.wv, nb * P.M, P.M, B.ctrl, 0, s);
  HIP_TRY(hipGetLastError());
  if (P.dense_mf) {
    if ((rc = tune_dense_mf<T>(ctx, P, pbs.geom, B, s))) return rc;
    // the matrix-core product starts this solve with no row maxima (all bits
    // set: not finite), so a solve does not depend on what the workspace held
    HIP_TRY(hipMemsetAsync(B.pw, 0xFF, sizeof(float) * 2 * P.np_pw, s));
  }
  if ((rc = wf_lists<T>(P, pbs.geom, B, s))) return rc;
  Plan P2 = P;
  for (int k = 0; k < 3; ++k) P2.tf16_axis[k] = false;
  const int nfields = nb > 1 ? nb : 0;
  // a single problem on a grid of 2 or 3 axes: the first Y pass (no
  // epilogue) hosts the control step; otherwise it is its own launch
  CtlHost host;
  const bool hosted = nfields == 0 && P.geom == UOT_GEOM_GRID && P.dim >= 2;
  if (hosted) {
    host.c = B.ctrl;
    host.parts = B.parts;
    host.nparts = P.nparts_x;
    host.hist = pr->res_hist;
  }
  auto iteration_with = [&](const Plan& PP) {
    return [&, pp = &PP](int par) {
      half_step<T>(*pp, pbs, 0 | par << 1, B, uo, nullptr, true, s);
      if (!hosted) timed(2, [&] { launch_control(B.ctrl, B.parts, pp->nparts_x, pr->res_hist, s, nfields, par); });
      half_step<T>(*pp, pbs, 1 | par << 1, B, vo, nullptr, false, s, hosted ? &host : nullptr, mass != nullptr);
      if (mass)
        timed(2, [&] { launch_mass_update<T>(B.ctrl, B.mass_m, B.mass_s, pp->nparts_y, mass->F3, mass->log_m0, par, s); });
    };
  };
  auto iteration = iteration_with(P);
  auto iteration2 = iteration_with(P2);
  const double final_tol = pr->tol;
  if (async) {
    if ((rc = run_async(ctx, B.ctrl, pr, iteration))) return rc;
  } else {
    rc = run_loop(ctx, B.ctrl, pr, iteration, res, mixed ? &iteration2 : nullptr, &final_tol);
    if (rc) return rc;
  }
  if (P.sorted()) {
    launch_scatter<T>(uo, px, P.N, u, s);
    launch_scatter<T>(vo, py, P.M, v, s);
    HIP_TRY(hipGetLastError());
  }
  if (async) return finish(ctx);   // the result waits for uot_sync_result
  if (log_z) *log_z = ctx->pinned->zeta;
  if ((rc = finish(ctx))) return rc;
  if (res->status == -3) return fail(UOT_E_NONFINITE, "non-finite residual");
  return res->status == 0 ? UOT_OK : UOT_NOT_CONVERGED;
}

template <typename T>
int half_step_t(uot_ctx* ctx, const uot_problem* pb, double eps, int side, const T* pot_in, T* pot_io, T* lse_out,
                double* residual, char* ws, size_t wsb) {
  Plan P;
  int rc = make_plan(P, pb->dtype, pb->geom, 1, 1, 0, eps);
  if (rc) return rc;
  if ((rc = check_ws(P, ws, wsb))) return rc;
  if (!pot_in || !pot_io) return fail(UOT_E_INVALID, "pot_in and pot_io are required");
  if (!(eps > 0)) return fail(UOT_E_INVALID, "eps must be > 0");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  Bufs<T> B = carve<T>(P, ws);
  Ctrl init = make_ctrl(eps, 0, 0, 0, 0, 1);
  launch_ctrl_init(B.ctrl, init, s);
  launch_log<T>(static_cast<const T*>(pb->p), B.logp, P.N, 1, s);
  launch_log<T>(static_cast<const T*>(pb->q), B.logq, P.M, 1, s);
  launch_log<T>(static_cast<const T*>(pb->dx), B.logdx, P.N, 0, s);
  launch_log<T>(static_cast<const T*>(pb->dy), B.logdy, P.M, 0, s);
  if (P.geom == UOT_GEOM_GRID)
    for (int k = 0; k < P.dim; ++k) launch_gtab<T>(B.gtab[k], (int)P.n[k], P.h[k], B.ctrl, 1, P.cost, s);
  if (side == 0) {
    launch_init_pot<T>(pot_in, B.logdy, nullptr, B.wv, P.M, P.M, B.ctrl, 0, s);
    half_step<T>(P, *pb, 0, B, pot_io, lse_out, true, s);
    launch_res_reduce(B.parts, P.nparts_x, B.scal, s);
  } else {
    launch_init_pot<T>(pot_in, B.logdx, nullptr, B.wu, P.N, P.N, B.ctrl, 0, s);
    half_step<T>(P, *pb, 1, B, pot_io, lse_out, false, s);
  }
  HIP_TRY(hipGetLastError());
  double r = 0.0;
  if (side == 0) {
    HIP_TRY(hipMemcpyAsync(ctx->pinned, B.scal, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (side == 0) std::memcpy(&r, ctx->pinned, sizeof(double));
  if (residual) *residual = r;
  return finish(ctx);
}

template <typename T>
int objective_t(uot_ctx* ctx, const uot_problem* pb, double eps, const T* u, const T* v, T* pi1, T* pi2,
                uot_objective_values* out, char* ws, size_t wsb) {
  Plan P;
  int rc = make_plan(P, pb->dtype, pb->geom, 1, 1);
  if (rc) return rc;
  if ((rc = check_ws(P, ws, wsb))) return rc;
  if (!u || !v || !out) return fail(UOT_E_INVALID, "u, v and out are required");
  if (!(eps > 0)) return fail(UOT_E_INVALID, "eps must be > 0");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  Bufs<T> B = carve<T>(P, ws);
  Ctrl init = make_ctrl(eps, 0, 0, 0, 0, 1);
  launch_ctrl_init(B.ctrl, init, s);
  launch_log<T>(static_cast<const T*>(pb->dx), B.logdx, P.N, 0, s);
  launch_log<T>(static_cast<const T*>(pb->dy), B.logdy, P.M, 0, s);
  if (P.geom == UOT_GEOM_GRID)
    for (int k = 0; k < P.dim; ++k) launch_gtab<T>(B.gtab[k], (int)P.n[k], P.h[k], B.ctrl, 1, P.cost, s);
  // w fields of u and v, and of the zero potential (for m(K))
  launch_init_pot<T>(v, B.logdy, nullptr, B.wv, P.M, P.M, B.ctrl, 0, s);
  launch_init_pot<T>(u, B.logdx, nullptr, B.wu, P.N, P.N, B.ctrl, 0, s);
  EpiArgs<T> raw{};
  raw.mode = EPI_RAW;
  auto product = [&](int side, const T* w, T* outp, T* const* tabs) {
    raw.out = outp;
    if (P.geom == UOT_GEOM_GRID) {
      grid_chain<T>(P, w, tabs, side, B.ctrl, raw, B.t2, B.t3, s);
    } else {
      dense_half<T>(P, pb->geom, side, w, B, B.ctrl, raw, s);
    }
  };
  // S(v) -> t1, T(u) -> pm region is busy in dense mode, so T goes to t2 after S is consumed
  double* part = B.obj;
  const int64_t nbx = (P.N + 255) / 256, nby = (P.M + 255) / 256;
  product(0, B.wv, B.t1, B.gtab);
  launch_obj_side<T>(u, B.t1, static_cast<const T*>(pb->p), static_cast<const T*>(pb->dx), P.N, eps,
                     to_dev(pb->F1), pi1, part, s);
  product(1, B.wu, B.t1, B.gtab);
  launch_obj_side<T>(v, B.t1, static_cast<const T*>(pb->q), static_cast<const T*>(pb->dy), P.M, eps,
                     to_dev(pb->F2), pi2, part + 4 * nbx, s);
  double* part2 = part + 4 * (nbx + nby);
  // m(K) = sum_i dx_i e^{S0_i}, S0 = log K(dy):  w = log2 dy  (zero potential)
  launch_init_pot<T>(nullptr, B.logdy, nullptr, B.t3, P.M, P.M, B.ctrl, 0, s);
  launch_init_pot<T>(nullptr, B.logdx, nullptr, B.t2, P.N, P.N, B.ctrl, 0, s);
  if (P.geom == UOT_GEOM_GRID) {
    // product() uses t2/t3 as temporaries on grids: keep the two w fields in logp/logq
    launch_init_pot<T>(nullptr, B.logdy, nullptr, B.logq, P.M, P.M, B.ctrl, 0, s);
    launch_init_pot<T>(nullptr, B.logdx, nullptr, B.logp, P.N, P.N, B.ctrl, 0, s);
    product(0, B.logq, B.t1, B.gtab);
    launch_sum_exp2<T>(B.logp, B.t1, P.N, part2, s);
  } else {
    product(0, B.t3, B.t1, B.gtab);
    launch_sum_exp2<T>(B.t2, B.t1, P.N, part2, s);
  }
  double* part3 = part2 + nbx;
  // <C, R>: one product per axis with that axis' kernel times C (grid), or a direct pass (points)
  int ncost = 0;
  if (P.geom == UOT_GEOM_GRID) {
    for (int a = 0; a < P.dim; ++a) {
      launch_gtab_cost<T>(B.gcost, (int)P.n[a], P.h[a], eps, P.cost, s);
      T* tabs[3] = {B.gtab[0], B.gtab[1], B.gtab[2]};
      tabs[a] = B.gcost;
      product(0, B.wv, B.t1, tabs);
      launch_sum_exp2<T>(B.wu, B.t1, P.N, part3 + ncost * nbx, s);
      ++ncost;
    }
  } else {
    launch_dense_cost<T>(P.dim, static_cast<const T*>(pb->geom.x), P.N, static_cast<const T*>(pb->geom.y), B.wv, P.M,
                         eps, B.t1, P.cost, s);
    launch_sum_exp2<T>(B.wu, B.t1, P.N, part3, s);
    ncost = 1;
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t tot = 4 * (nbx + nby) + nbx * (1 + ncost);
  std::vector<double> h(tot);
  HIP_TRY(hipMemcpy(h.data(), part, sizeof(double) * tot, hipMemcpyDeviceToHost));
  double sx[4] = {0, 0, 0, 0}, sy[4] = {0, 0, 0, 0}, mK = 0, cost = 0;
  for (int64_t b = 0; b < nbx; ++b)
    for (int q = 0; q < 4; ++q) sx[q] += h[b * 4 + q];
  for (int64_t b = 0; b < nby; ++b)
    for (int q = 0; q < 4; ++q) sy[q] += h[4 * nbx + b * 4 + q];
  for (int64_t b = 0; b < nbx; ++b) mK += h[4 * (nbx + nby) + b];
  for (int k = 0; k < ncost; ++k)
    for (int64_t b = 0; b < nbx; ++b) cost += h[4 * (nbx + nby) + nbx * (1 + k) + b];
  out->mass1 = sx[0];
  out->mass2 = sy[0];
  out->massK = mK;
  out->transport_cost = cost;
  out->primal = sx[2] + sy[2] + sx[1] + sy[1] - eps * sx[0] + eps * mK;
  out->dual = -sx[3] - sy[3] - eps * sx[0] + eps * mK;
  auto finite_valued = [](int k) { return k == UOT_DIV_KL || k == UOT_DIV_TV || k == UOT_DIV_GROWTH; };
  const bool finite_gap = finite_valued(pb->F1.kind) && finite_valued(pb->F2.kind);
  out->gap = finite_gap ? (sx[2] + sx[3] + sx[1]) + (sy[2] + sy[3] + sy[1]) : NAN;
  if (!finite_gap) out->primal = NAN;
  return finish(ctx);
}

template <typename T>
int bary_t(uot_ctx* ctx, const uot_bary_problem* pb, const uot_params* pr, T* u, T* v, T* logh, char* ws, size_t wsb,
           uot_result* res) {
  Plan P;
  const bool anneal = pr->eps0 > pr->eps && pr->eps_stages > 0 && pr->iters_per_stage > 0;
  int rc = make_plan(P, pb->dtype, pb->geom, pb->n, anneal ? pr->eps_stages + 1 : 1, pr->grid_kernel, pr->eps);
  if (rc) return rc;
  if ((rc = check_ws(P, ws, wsb))) return rc;
  if (!u || !v) return fail(UOT_E_INVALID, "u and v output buffers are required");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  Bufs<T> B = carve<T>(P, ws);
  const int64_t size = P.N, nb = pb->n;
  const bool mixed = P.gk == 4 && has_tf16(P) && pr->tol < kMixedSwitchTol;
  Plan P2 = P;
  for (int k = 0; k < 3; ++k) P2.tf16_axis[k] = false;
  Ctrl init = make_ctrl(pr->eps, pr->eps0, pr->eps_stages, pr->iters_per_stage, mixed ? kMixedSwitchTol : pr->tol,
                        pr->max_iter);
  launch_ctrl_init(B.ctrl, init, s);
  launch_log<T>(static_cast<const T*>(pb->p), B.logp, nb * size, 1, s);
  launch_log<T>(static_cast<const T*>(pb->dx), B.logdx, size, 0, s);
  launch_log<T>(static_cast<const T*>(pb->dy), B.logdy, size, 0, s);
  for (int k = 0; k < P.dim; ++k) launch_gtab<T>(B.gtab[k], (int)P.n[k], P.h[k], B.ctrl, P.nst, P.cost, s);
  launch_init_pot<T>(nullptr, B.logdx, u, nullptr, nb * size, size, B.ctrl, 0, s);
  launch_init_pot<T>(static_cast<const T*>(pr->v0), B.logdy, v, B.wv, nb * size, size, B.ctrl, 0, s);
  HIP_TRY(hipGetLastError());
  BaryW la{};
  double asum = 0;
  for (int k = 0; k < pb->n; ++k) {
    la.v[k] = std::log(pb->alpha[k]);
    la.a[k] = pb->alpha[k];
    asum += pb->alpha[k];
  }
  const DivDev F2 = to_dev(pb->F2);
  auto iteration_with = [&](const Plan& PP) {
    return [&, pp = &PP](int par) {
      EpiArgs<T> ep = prox_epi<T>(u, B.wu, B.logp, B.logdx, nullptr, B.parts, size, pb->F1);
      grid_chain<T>(*pp, B.wv, B.gtab, 0 | par << 1, B.ctrl, ep, B.t1, B.t2, s);
      launch_control(B.ctrl, B.parts, pp->nparts_x, pr->res_hist, s, 0, par);
      EpiArgs<T> raw{};
      raw.mode = EPI_RAW;
      raw.out = B.t3;
      grid_chain<T>(*pp, B.wu, B.gtab, 1 | par << 1, B.ctrl, raw, B.t1, B.t2, s);
      launch_bary_combine<T>(B.t3, pb->n, size, la, std::log(asum), F2, B.logdy, v, B.wv, logh, B.ctrl,
                             1 | par << 1, s);
    };
  };
  auto iteration = iteration_with(P);
  auto iteration2 = iteration_with(P2);
  const double final_tol = pr->tol;
  rc = run_loop(ctx, B.ctrl, pr, iteration, res, mixed ? &iteration2 : nullptr, &final_tol);
  if (rc) return rc;
  if ((rc = finish(ctx))) return rc;
  if (res->status == -3) return fail(UOT_E_NONFINITE, "non-finite residual");
  return res->status == 0 ? UOT_OK : UOT_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// barycentric projection (colour transfer, Sec. 5.1): T = R (y dy) / R dy
// from v alone (u cancels), as dim + 1 Gibbs products of the X side (2 dim + 1
// for points: positive and negative parts of each coordinate)
// ---------------------------------------------------------------------------
template <typename T>
int map_t(uot_ctx* ctx, const uot_problem* pb, double eps, const T* v, T* Tout, char* ws, size_t wsb) {
  Plan P;
  int rc = make_plan(P, pb->dtype, pb->geom, 1, 1, 0, eps);
  if (rc) return rc;
  if ((rc = check_ws(P, ws, wsb))) return rc;
  if (!v || !Tout) return fail(UOT_E_INVALID, "v and T are required");
  if (!(eps > 0 && std::isfinite(eps))) return fail(UOT_E_INVALID, "eps must be finite and > 0");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  Bufs<T> B = carve<T>(P, ws);
  const Ctrl init = make_ctrl(eps, 0, 0, 0, 0, 1);
  launch_ctrl_init(B.ctrl, init, s);
  launch_log<T>(static_cast<const T*>(pb->dy), B.logdy, P.M, 0, s);
  if (P.geom == UOT_GEOM_GRID)
    for (int k = 0; k < P.dim; ++k) launch_gtab<T>(B.gtab[k], (int)P.n[k], P.h[k], B.ctrl, 1, P.cost, s);
  launch_init_pot<T>(v, B.logdy, nullptr, B.wv, P.M, P.M, B.ctrl, 0, s);
  EpiArgs<T> raw{};
  raw.mode = EPI_RAW;
  auto product = [&](const T* w, T* out) {
    raw.out = out;
    if (P.geom == UOT_GEOM_GRID) grid_chain<T>(P, w, B.gtab, 0, B.ctrl, raw, B.t1, B.t2, s);
    else dense_half<T>(P, pb->geom, 0, w, B, B.ctrl, raw, s);
  };
  product(B.wv, B.t3);   // log2 of sum_j R_ij dy_j (up to the factor a_i)
  int64_t stride = 1;
  for (int k = P.dim - 1; k >= 0; --k) {
    T* num = Tout + (int64_t)k * P.N;
    if (P.geom == UOT_GEOM_GRID) {
      launch_coord_weight<T>(B.wv, B.logq, P.M, stride, P.n[k], P.h[k], nullptr, 1, s);
      product(B.logq, num);
      launch_map_finish<T>(num, B.t3, nullptr, P.N, s);
      stride *= P.n[k];
    } else {
      const T* yk = static_cast<const T*>(pb->geom.y) + (int64_t)k * P.M;
      launch_coord_weight<T>(B.wv, B.logq, P.M, 1, 1, 0.0, yk, 1, s);
      product(B.logq, num);
      launch_coord_weight<T>(B.wv, B.logq, P.M, 1, 1, 0.0, yk, -1, s);
      product(B.logq, B.wu);
      launch_map_finish<T>(num, B.t3, B.wu, P.N, s);
    }
  }
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

// ---------------------------------------------------------------------------
// gradient flows (Sec. 5.3): a sequence of steps, each one problem of the
// generic form solved by the scaling iteration, warm-started with the previous
// step's v; the next density is read off the optimal coupling on the device
// ---------------------------------------------------------------------------
struct FlowDivs {
  uot_div F1, F2;
};

int validate_flow(const uot_flow_problem* fp, FlowDivs& d) {
  if (!fp) return fail(UOT_E_INVALID, "flow problem is NULL");
  if (!fp->p0 || !fp->q || !fp->dx) return fail(UOT_E_INVALID, "p0, q and dx are required");
  if (fp->kind < UOT_FLOW_HEAT || fp->kind > UOT_FLOW_GROWTH) return fail(UOT_E_INVALID, "unknown flow kind");
  if (!(fp->tau > 0 && std::isfinite(fp->tau))) return fail(UOT_E_INVALID, "tau must be finite and > 0");
  if (fp->species < 1 || fp->species > kMaxBary) return fail(UOT_E_UNSUPPORTED, "1 <= species <= 64");
  if (fp->species > 1 && fp->kind != UOT_FLOW_GROWTH)
    return fail(UOT_E_UNSUPPORTED, "several species only for the growth flow");
  if (fp->species > 1 && fp->geom.kind != UOT_GEOM_GRID)
    return fail(UOT_E_UNSUPPORTED, "several species need a grid geometry");
  if (fp->geom.kind == UOT_GEOM_POINTS && (fp->geom.x != fp->geom.y || fp->geom.N != fp->geom.M))
    return fail(UOT_E_INVALID, "a flow moves densities on one space: x and y must be the same points");
  const double lam = 2.0 * fp->tau * fp->alpha;
  if (fp->kind == UOT_FLOW_GROWTH && !(fp->alpha >= 0 && lam < 1))
    return fail(UOT_E_INVALID, "growth flow: alpha >= 0 and 2 tau alpha < 1");
  d.F1 = uot_div{fp->kind == UOT_FLOW_GROWTH ? UOT_DIV_KL : UOT_DIV_EQ, 0, 1.0, 0.0, INFINITY};
  if (fp->kind == UOT_FLOW_HEAT) d.F2 = uot_div{UOT_DIV_KL, 0, 2.0 * fp->tau, 0.0, INFINITY};
  else if (fp->kind == UOT_FLOW_CROWD) d.F2 = uot_div{UOT_DIV_RG, 0, 1.0, 0.0, 1.0};
  else d.F2 = uot_div{UOT_DIV_GROWTH, 0, lam, 0.0, INFINITY};
  return UOT_OK;
}

int flow_plan(Plan& P, const uot_flow_problem* fp, int nst, int grid_kernel, double eps_min, size_t& o_u) {
  int rc = make_plan(P, fp->dtype, fp->geom, fp->species, nst, grid_kernel, eps_min);
  if (rc) return rc;
  o_u = align_up(P.total);
  P.total = align_up(o_u + P.esz * (size_t)fp->species * P.N);
  return UOT_OK;
}

template <typename T>
int flow_t(uot_ctx* ctx, const uot_flow_problem* fp, const FlowDivs& fd, const uot_params* pr, int n_steps, T* dens,
           T* v, char* ws, size_t wsb, uot_result* steps) {
  Plan P;
  size_t o_u = 0;
  const bool anneal = pr->eps0 > pr->eps && pr->eps_stages > 0 && pr->iters_per_stage > 0;
  int rc = flow_plan(P, fp, anneal ? pr->eps_stages + 1 : 1, pr->grid_kernel, pr->eps, o_u);
  if (rc) return rc;
  if ((rc = check_ws(P, ws, wsb))) return rc;
  if (!dens || !v) return fail(UOT_E_INVALID, "dens and v output buffers are required");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  Bufs<T> B = carve<T>(P, ws);
  T* u = at<T>(ws, o_u);
  const int S = fp->species;
  const int64_t N = P.N, SN = (int64_t)S * N;
  const Ctrl init = make_ctrl(pr->eps, pr->eps0, pr->eps_stages, pr->iters_per_stage, pr->tol, pr->max_iter);
  launch_ctrl_init(B.ctrl, init, s);
  launch_log<T>(static_cast<const T*>(fp->dx), B.logdx, N, 0, s);
  launch_log<T>(static_cast<const T*>(fp->dx), B.logdy, N, 0, s);
  launch_log<T>(static_cast<const T*>(fp->q), B.logq, N, 1, s);
  if (P.geom == UOT_GEOM_GRID)
    for (int k = 0; k < P.dim; ++k) launch_gtab<T>(B.gtab[k], (int)P.n[k], P.h[k], B.ctrl, P.nst, P.cost, s);
  HIP_TRY(hipMemcpyAsync(dens, fp->p0, sizeof(T) * SN, hipMemcpyDeviceToDevice, s));
  if (pr->v0) HIP_TRY(hipMemcpyAsync(v, pr->v0, sizeof(T) * SN, hipMemcpyDeviceToDevice, s));
  else launch_init_pot<T>(nullptr, B.logdy, v, nullptr, SN, N, B.ctrl, 0, s);
  uot_problem pb{};
  pb.dtype = fp->dtype;
  pb.geom = fp->geom;
  pb.F1 = fd.F1;
  pb.F2 = fd.F2;
  const DivDev Fg = to_dev(fd.F2);
  const bool growth = fp->kind == UOT_FLOW_GROWTH;
  auto iteration = [&](int par) {
    if (S == 1) {
      half_step<T>(P, pb, 0 | par << 1, B, u, nullptr, true, s);
      timed(2, [&] { launch_control(B.ctrl, B.parts, P.nparts_x, pr->res_hist, s, 0, par); });
      half_step<T>(P, pb, 1 | par << 1, B, v, nullptr, false, s);
    } else {
      // several species: KL(. | p_k) on each first marginal, the joint growth
      // proxdiv on the sum of the second marginals
      EpiArgs<T> ep = prox_epi<T>(u, B.wu, B.logp, B.logdx, nullptr, B.parts, N, fd.F1);
      grid_chain<T>(P, B.wv, B.gtab, 0 | par << 1, B.ctrl, ep, B.t1, B.t2, s);
      timed(2, [&] { launch_control(B.ctrl, B.parts, P.nparts_x, pr->res_hist, s, 0, par); });
      EpiArgs<T> raw{};
      raw.mode = EPI_RAW;
      raw.out = B.t3;
      grid_chain<T>(P, B.wu, B.gtab, 1 | par << 1, B.ctrl, raw, B.t1, B.t2, s);
      launch_growth_combine<T>(B.t3, S, N, Fg, B.logq, B.logdy, v, B.wv, B.ctrl, 1 | par << 1, s);
    }
  };
  GraphCache cache;
  int worst = UOT_OK;
  for (int k = 0; k < n_steps; ++k) {
    T* pk = dens + (int64_t)k * SN;
    T* pn = pk + SN;
    launch_ctrl_init(B.ctrl, init, s);
    launch_log<T>(pk, B.logp, SN, 1, s);
    launch_init_pot<T>(nullptr, B.logdx, u, nullptr, SN, N, B.ctrl, 0, s);
    launch_init_pot<T>(v, B.logdy, v, B.wv, SN, N, B.ctrl, 0, s);   // warm start: last step's v
    HIP_TRY(hipGetLastError());
    uot_result r{};
    rc = run_loop(ctx, B.ctrl, pr, iteration, &r, static_cast<decltype(iteration)*>(nullptr), nullptr, &cache);
    if (rc) return rc;
    if (steps) steps[k] = r;
    if (r.status == -3) return fail(UOT_E_NONFINITE, "non-finite residual in flow step " + std::to_string(k));
    if (r.status != 0) worst = UOT_NOT_CONVERGED;
    // the second marginals of the final plans: one more Y product at the last eps
    launch_ctrl_post(B.ctrl, s);
    launch_init_pot<T>(u, B.logdx, nullptr, B.wu, SN, N, B.ctrl, 0, s);
    EpiArgs<T> raw{};
    raw.mode = EPI_RAW;
    raw.out = B.t3;
    if (P.geom == UOT_GEOM_GRID) grid_chain<T>(P, B.wu, B.gtab, 1, B.ctrl, raw, B.t1, B.t2, s);
    else dense_half<T>(P, fp->geom, 1, B.wu, B, B.ctrl, raw, s);
    launch_flow_next<T>(B.t3, v, B.logq, S, N, growth ? 1 : 0, std::log1p(-2.0 * fp->tau * fp->alpha), B.ctrl, pn,
                        s);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(s));
  if ((rc = finish(ctx))) return rc;
  return worst;
}

// average device time of each Gibbs-product kernel of one X half-step over nb
// fields (grids; points: nb = 1), with HIP events around `reps` back-to-back
// launches of that kernel alone
template <typename T>
int time_half_step_t(uot_ctx* ctx, const uot_problem* pb, int nb, double eps, const T* v, int reps, double* ms,
                     int* nk, char* ws, size_t wsb, int grid_kernel) {
  Plan P;
  if (nb < 1) return fail(UOT_E_INVALID, "nb must be >= 1");
  // point clouds: kernel 2 times the tile-factored product on Morton-ordered
  // copies, kernels 3 and 4 the matrix-core products
  const int dk = (pb->geom.kind == UOT_GEOM_POINTS && grid_kernel >= 2 && grid_kernel <= 4) ? grid_kernel : 1;
  int rc = make_plan(P, pb->dtype, pb->geom, nb, 1, pb->geom.kind == UOT_GEOM_GRID ? grid_kernel : 0, eps, dk);
  if (rc) return rc;
  if ((rc = check_ws(P, ws, wsb))) return rc;
  if (!v || !ms || !nk || reps < 1) return fail(UOT_E_INVALID, "v, ms, n_kernels and reps >= 1 are required");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  Bufs<T> B = carve<T>(P, ws);
  Ctrl init = make_ctrl(eps, 0, 0, 0, 0, 1);
  launch_ctrl_init(B.ctrl, init, s);
  uot_problem pbs = *pb;
  const int32_t* px = nullptr;
  const int32_t* py = nullptr;
  if (P.sorted()) {
    pbs = sorted_points<T>(P, *pb, ws, s);
    px = at<int32_t>(ws, P.o_permx);
    py = at<int32_t>(ws, P.o_permy);
  }
  log_into<T>(pb->p, B.logp, nb * P.N, 1, px, B.t1, s);
  log_into<T>(pb->dx, B.logdx, P.N, 0, px, B.t1, s);
  log_into<T>(pb->dy, B.logdy, P.M, 0, py, B.t1, s);
  if (P.geom == UOT_GEOM_GRID)
    for (int k = 0; k < P.dim; ++k) launch_gtab<T>(B.gtab[k], (int)P.n[k], P.h[k], B.ctrl, 1, P.cost, s);
  const T* vin = v;
  if (py) {
    launch_gather<T>(v, py, P.M, 1, B.t2, s);
    vin = B.t2;
  }
  launch_init_pot<T>(vin, B.logdy, nullptr, B.wv, nb * P.M, P.M, B.ctrl, 0, s);
  launch_init_pot<T>(nullptr, B.logdx, B.t3, nullptr, nb * P.N, P.N, B.ctrl, 0, s);   // u = 0 in t3
  if (P.dense_mf) {
    int rc2 = tune_dense_mf<T>(ctx, P, pbs.geom, B, s);
    if (rc2) return rc2;
    HIP_TRY(hipMemsetAsync(B.pw, 0xFF, sizeof(float) * 2 * P.np_pw, s));
  }
  if (int rc3 = wf_lists<T>(P, pbs.geom, B, s)) return rc3;
  EpiArgs<T> ep = prox_epi<T>(B.t3, B.wu, B.logp, B.logdx, nullptr, B.parts, P.N, pb->F1);
  EpiArgs<T> raw{};
  raw.mode = EPI_RAW;
  bool count_pairs = false;   // the matrix-core product's pair counter, off while timed
  std::vector<std::function<void()>> ks;
  if (P.geom == UOT_GEOM_GRID) {
    const int64_t nbf = nb;
    if (P.dim == 1) {
      ks.push_back([&] { contig_pass<T>(P, 0, B.wv, nbf, B.gtab, 0, B.ctrl, ep, s); });
    } else if (P.dim == 2) {
      raw.out = B.t1;
      ks.push_back([&] { contig_pass<T>(P, 1, B.wv, nbf * P.n[0], B.gtab, 0, B.ctrl, raw, s); });
      ks.push_back([&] { strided_pass<T>(P, 0, B.t1, nbf, P.n[1], B.gtab, 0, B.ctrl, ep, s); });
    } else {
      EpiArgs<T> raw2 = raw;
      raw.out = B.t1;
      raw2.out = B.t2;
      ks.push_back([&, raw] { contig_pass<T>(P, 2, B.wv, nbf * P.n[0] * P.n[1], B.gtab, 0, B.ctrl, raw, s); });
      ks.push_back([&, raw2] { strided_pass<T>(P, 1, B.t1, nbf * P.n[0], P.n[2], B.gtab, 0, B.ctrl, raw2, s); });
      ks.push_back([&] { strided_pass<T>(P, 0, B.t2, nbf, P.n[1] * P.n[2], B.gtab, 0, B.ctrl, ep, s); });
    }
  } else {
    const T* rows = static_cast<const T*>(pbs.geom.x);
    const T* cols = static_cast<const T*>(pbs.geom.y);
    ks.push_back([&] {
      if constexpr (std::is_same<T, float>::value) {
        if (P.dense_tf) {
          launch_dense_tf(P.dim, rows, P.N, cols, B.wv, P.M, P.splits[0], P.cps[0], B.pm, B.ps, 0, B.ctrl, s);
          return;
        }
        if (P.dense_mf) {
          MfSkip sk;   // counted only in the extra launch after the timed ones
          sk.on = tile_skip_enabled() ? 1 : 0;
          sk.pairs = count_pairs ? &B.ctrl->pairs : nullptr;
          launch_dense_mf(P.dim, P.mf_groups, P.mf_split, rows, P.N, cols, B.wv, P.M, P.splits[0], P.cps[0], B.pm, B.ps,
                          B.pw, 0, B.ctrl, sk, s);
          return;
        }
      }
      if (P.wfl) {
        launch_wf_lse<T>(P.dim, rows, P.N, cols, B.wv, P.M, P.cost.cut, B.wfl[0], P.wf_umax[0], B.wfpm, B.wfps, 0,
                         B.ctrl, s);
        return;
      }
      launch_dense_lse<T>(P.dim, P.R[0], rows, P.N, cols, B.wv, P.M, P.splits[0], P.cps[0], B.pm, B.ps, 0, B.ctrl,
                          P.cost, s);
    });
    ks.push_back([&] {
      if (P.wfl) launch_wf_epi<T>(B.wfpm, B.wfps, B.wfl[0], P.N, P.M, 0, B.ctrl, ep, s);
      else launch_dense_epi<T>(B.pm, B.ps, P.splits[0], P.N, 0, B.ctrl, ep, s);
    });
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  for (auto& k : ks) k();   // warm: every intermediate exists before timing
  for (size_t q = 0; q < ks.size(); ++q) {
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) ks[q]();
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    ms[q] = double(t) / reps;
  }
  *nk = (int)ks.size();
  if (P.geom == UOT_GEOM_POINTS && P.dense_mf) {
    // one more launch of the product, counted and not timed (the same state
    // as the timed ones: v fixed, the row maxima they left)
    count_pairs = true;
    ks[0]();
    unsigned long long pairs = 0;
    HIP_TRY(hipMemcpyAsync(&pairs, &B.ctrl->pairs, sizeof(pairs), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    ms[2] = double(pairs);
    *nk = 3;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}


// ---------------------------------------------------------------------------
// ragged batches
// ---------------------------------------------------------------------------
struct BatchPlan {
  int dtype = 0, dim = 0;
  size_t esz = 0;
  int64_t B = 0, totN = 0, totM = 0;
  int64_t max_items = 0;       // items per side at R = 1 (upper bound for any R)
  int64_t nmaxN = 0, nmaxM = 0;   // largest problem per side
  bool mf = false;                // FP32: the matrix-core product is among the tuner's choices
  size_t o_ctrl, o_logp, o_logq, o_logdx, o_logdy, o_wu, o_wv, o_stop, o_yskip, o_status, o_iters, o_res, o_clock, o_itx,
      o_ity, o_pstart, o_parts, o_curs, o_offN, o_offM, o_ordx, o_ordy, o_xs, o_ys, o_permx, o_permy, o_code, o_box,
      o_us, o_vs, o_pw, o_pstartY, o_bal, total;
};

int make_batch_plan(BatchPlan& P, const uot_batch_problem* pb) {
  if (pb->dtype != UOT_F32 && pb->dtype != UOT_F64) return fail(UOT_E_INVALID, "dtype must be UOT_F32 or UOT_F64");
  if (pb->dim < 1 || pb->dim > 3) return fail(UOT_E_UNSUPPORTED, "dim must be 1, 2 or 3");
  if (pb->B < 1 || pb->B > (1 << 24)) return fail(UOT_E_INVALID, "B must be in [1, 2^24]");
  if (!pb->offN || !pb->offM) return fail(UOT_E_INVALID, "offN and offM are required");
  P.dtype = pb->dtype;
  P.dim = pb->dim;
  P.esz = pb->dtype == UOT_F32 ? 4 : 8;
  P.B = pb->B;
  if (pb->offN[0] != 0 || pb->offM[0] != 0) return fail(UOT_E_INVALID, "offsets must start at 0");
  int64_t items = 0, itemsy = 0;
  for (int64_t b = 0; b < pb->B; ++b) {
    const int64_t n = pb->offN[b + 1] - pb->offN[b], m = pb->offM[b + 1] - pb->offM[b];
    if (n < 1 || m < 1) return fail(UOT_E_INVALID, "every problem needs N, M >= 1");
    if (n > (1 << 30) || m > (1 << 30)) return fail(UOT_E_UNSUPPORTED, "problem too large for a batch");
    items += (n + 255) / 256;
    itemsy += (m + 255) / 256;
    P.nmaxN = std::max(P.nmaxN, n);
    P.nmaxM = std::max(P.nmaxM, m);
  }
  P.totN = pb->offN[pb->B];
  P.totM = pb->offM[pb->B];
  P.max_items = std::max(items, itemsy);
  const size_t e = P.esz;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  P.o_ctrl = take(align_up(sizeof(Ctrl), 64) + sizeof(BCtrl));
  P.o_logp = take(e * P.totN);
  P.o_logq = take(e * P.totM);
  P.o_logdx = take(e * P.totN);
  P.o_logdy = take(e * P.totM);
  P.o_wu = take(e * P.totN);
  P.o_wv = take(e * P.totM);
  P.o_stop = take(4 * P.B);
  P.o_yskip = take(4 * P.B);
  P.o_status = take(4 * P.B);
  P.o_iters = take(8 * P.B);
  P.o_res = take(8 * P.B);
  P.o_clock = take(8 * P.B);
  P.o_itx = take(sizeof(BItem) * P.max_items);
  P.o_ity = take(sizeof(BItem) * P.max_items);
  P.o_pstart = take(4 * (P.B + 1));
  P.o_parts = take(sizeof(ResPart) * P.max_items);
  P.o_curs = take(4 * 4);   // lengths of the two item lists, then their work cursors
  P.o_offN = take(8 * (P.B + 1));
  P.o_offM = take(8 * (P.B + 1));
  P.o_ordx = take(4 * P.B);
  P.o_ordy = take(4 * P.B);
  // FP32: Morton-ordered copies per problem for the matrix-core product
  // (coordinates, permutations, codes, boxes, potentials) and its row maxima
  P.mf = P.dtype == UOT_F32;
  const bool mf = P.mf;
  P.o_xs = take(mf ? 4 * P.dim * P.totN : 0);
  P.o_ys = take(mf ? 4 * P.dim * P.totM : 0);
  P.o_permx = take(mf ? 4 * P.totN : 0);
  P.o_permy = take(mf ? 4 * P.totM : 0);
  P.o_code = take(mf ? 4 * std::max(P.totN, P.totM) : 0);
  P.o_box = take(mf ? 4 * 6 * P.B : 0);
  P.o_us = take(mf ? 4 * P.totN : 0);
  P.o_vs = take(mf ? 4 * P.totM : 0);
  P.o_pw = take(mf ? 4 * (P.totN + P.totM) : 0);
  // the in-solve mass balance: first Y slot of each problem, and the mass
  // partials of the X items, then of the Y items
  P.o_pstartY = take(4 * (P.B + 1));
  P.o_bal = take(4 * e * P.max_items);
  P.total = o;
  return UOT_OK;
}

// every work item of one side for rows per item 256*R, sorted by cost
// (largest first): the fixed lists of the plain batch Gibbs products
void build_items(const int64_t* offR, const int64_t* offC, int64_t B, int R, std::vector<BItem>& items) {
  items.clear();
  const int rows = 256 * R;
  int32_t slot = 0;
  for (int64_t b = 0; b < B; ++b) {
    const int64_t n = offR[b + 1] - offR[b];
    for (int64_t r0 = 0; r0 < n; r0 += rows) {
      BItem it;
      it.prob = (int32_t)b;
      it.row0 = (int32_t)r0;
      it.nrows = (int32_t)std::min<int64_t>(rows, n - r0);
      it.part = slot++;
      items.push_back(it);
    }
  }
  std::stable_sort(items.begin(), items.end(), [&](const BItem& a, const BItem& c) {
    const int64_t ca = (int64_t)a.nrows * (offC[a.prob + 1] - offC[a.prob]);
    const int64_t cc = (int64_t)c.nrows * (offC[c.prob + 1] - offC[c.prob]);
    return ca > cc;
  });
}

// Problem order of the item lists of one side (rows from offR, columns from
// offC): largest column count first, then largest row count, so the rebuilt
// lists run from the costliest row tiles down
void build_order(const int64_t* offR, const int64_t* offC, int64_t B, std::vector<int32_t>& ord) {
  ord.resize(B);
  for (int64_t b = 0; b < B; ++b) ord[b] = (int32_t)b;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t c) {
    const int64_t ma = offC[a + 1] - offC[a], mc = offC[c + 1] - offC[c];
    if (ma != mc) return ma > mc;
    return offR[a + 1] - offR[a] > offR[c + 1] - offR[c];
  });
}

// residual slots of the X items: problem-major, 256 R rows per item
void build_pstart(const int64_t* offN, int64_t B, int R, std::vector<int32_t>& pstart) {
  pstart.assign(B + 1, 0);
  const int64_t rows = 256 * R;
  int64_t slot = 0;
  for (int64_t b = 0; b < B; ++b) {
    pstart[b] = (int32_t)slot;
    slot += (offN[b + 1] - offN[b] + rows - 1) / rows;
  }
  pstart[B] = (int32_t)slot;
}

// Workspace views and one-time set-up shared by the plain Gibbs products of a
// batch (uot_batch_gibbs, the cloud warm-start features): offsets and the
// per-problem flags on the device, every problem active.
struct BatchGibbs {
  Ctrl* ctrl;
  BCtrl* bc_dev;
  int64_t *offN_d, *offM_d;
  BItem *items[2];     // rows X, rows Y (columns of the other side or the same side, see gibbs_items)
  int n_items[2];
  int* curs;           // list lengths, then work cursors, on the device
  int ncu;
};

template <typename T>
int batch_gibbs_setup(uot_ctx* ctx, const BatchPlan& P, const uot_batch_problem* pb, char* ws, BatchGibbs& G) {
  hipStream_t s = ctx->work;
  G.ctrl = at<Ctrl>(ws, P.o_ctrl);
  BCtrl bc;
  bc.stop = at<int32_t>(ws, P.o_stop);
  bc.yskip = at<int32_t>(ws, P.o_yskip);
  bc.status = at<int32_t>(ws, P.o_status);
  bc.iters = at<int64_t>(ws, P.o_iters);
  bc.res = at<double>(ws, P.o_res);
  bc.clock = at<uint64_t>(ws, P.o_clock);
  G.bc_dev = reinterpret_cast<BCtrl*>(reinterpret_cast<char*>(G.ctrl) + align_up(sizeof(Ctrl), 64));
  G.offN_d = at<int64_t>(ws, P.o_offN);
  G.offM_d = at<int64_t>(ws, P.o_offM);
  G.items[0] = at<BItem>(ws, P.o_itx);
  G.items[1] = at<BItem>(ws, P.o_ity);
  G.curs = at<int>(ws, P.o_curs);
  HIP_TRY(hipDeviceGetAttribute(&G.ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  // the synchronous copies below overwrite workspace earlier work on the stream may still read
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(G.offN_d, pb->offN, 8 * (P.B + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(G.offM_d, pb->offM, 8 * (P.B + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(G.bc_dev, &bc, sizeof(BCtrl), hipMemcpyHostToDevice));
  return UOT_OK;
}

// items of rows of side `rows` (0: X, 1: Y) against the columns of side
// `cols`, uploaded into the items slot of the rows side
int gibbs_items(const BatchPlan& P, const uot_batch_problem* pb, int rows, int cols, BatchGibbs& G) {
  std::vector<BItem> it;
  build_items(rows ? pb->offM : pb->offN, cols ? pb->offM : pb->offN, P.B, 1, it);
  HIP_TRY(hipMemcpy(G.items[rows], it.data(), sizeof(BItem) * it.size(), hipMemcpyHostToDevice));
  G.n_items[rows] = (int)it.size();
  return UOT_OK;
}

// out_r = log sum_c exp(w_c - |row_r - col_c|^2 / eps) for every problem
// (natural log), direct product; w2 is workspace for the log2 input
template <typename T>
void gibbs_launch(const BatchPlan& P, const uot_batch_problem* pb, const BatchGibbs& G, double eps, int rows, int cols,
                  const T* w, T* w2, T* out, char* ws, hipStream_t s) {
  launch_ctrl_init(G.ctrl, make_ctrl(eps, 0, 0, 0, 0, 1), s);
  launch_batch_init(G.bc_dev, (int)P.B, G.ctrl, s);
  launch_set_int(G.curs + rows, 1, G.n_items[rows], s);
  launch_set_int(G.curs + 2 + rows, 1, 0, s);
  const int64_t totR = rows ? P.totM : P.totN, totC = cols ? P.totM : P.totN;
  launch_init_pot<T>(nullptr, w, nullptr, w2, totC, totC, G.ctrl, 0, s);   // w2 = w log2(e)
  EpiArgs<T> ep{};
  ep.mode = EPI_RAW;
  ep.out = out;
  const int64_t* offR = rows ? G.offM_d : G.offN_d;
  const int64_t* offC = cols ? G.offM_d : G.offN_d;
  const T* xr = static_cast<const T*>(rows ? pb->y : pb->x);
  const T* yc = static_cast<const T*>(cols ? pb->y : pb->x);
  if constexpr (std::is_same<T, float>::value) {
    if (P.mf) {
      // FP32: the matrix-core product (items of 256 rows, 4 blocks per CU),
      // from no starting maxima; with none, no tile could be left out, so
      // the tile records are not staged
      float* pw = at<float>(ws, P.o_pw) + (rows ? P.totN : 0);
      (void)hipMemsetAsync(pw, 0xFF, sizeof(float) * totR, s);
      MfSkip sk;
      sk.on = 0;
      launch_batch_mf(P.dim, 4, G.ncu * 4, G.items[rows], G.curs + rows, G.curs + 2 + rows, offR, offC, xr, totR, yc,
                      totC, w2, pw, G.bc_dev, G.ctrl, 0, ep, sk, s);
      launch_scale<T>(out, totR, kLn2, s);
      return;
    }
  }
  launch_batch_lse<T>(P.dim, 1, G.ncu * 8, G.items[rows], G.curs + rows, G.curs + 2 + rows, offR, offC, xr, totR, yc,
                      totC, w2, G.bc_dev, G.ctrl, 0, ep, s);
  launch_scale<T>(out, totR, kLn2, s);
}

int check_batch_ws(const BatchPlan& P, const void* ws, size_t wsb, size_t need) {
  if (!ws) return fail(UOT_E_WORKSPACE, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(UOT_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (wsb < need) return fail(UOT_E_WORKSPACE, "workspace too small: need " + std::to_string(need));
  (void)P;
  return UOT_OK;
}

template <typename T>
int batch_gibbs_t(uot_ctx* ctx, const uot_batch_problem* pb, double eps, int rows, int cols, const T* w, T* out,
                  char* ws, size_t wsb) {
  BatchPlan P;
  int rc = make_batch_plan(P, pb);
  if (rc) return rc;
  if ((rc = check_batch_ws(P, ws, wsb, P.total))) return rc;
  if (!pb->x || !pb->y || !w || !out) return fail(UOT_E_INVALID, "x, y, w and out are required");
  if (!(eps > 0) || !std::isfinite(eps)) return fail(UOT_E_INVALID, "eps must be > 0");
  if ((rows != 0 && rows != 1) || (cols != 0 && cols != 1)) return fail(UOT_E_INVALID, "rows and cols are 0 or 1");
  if ((rc = begin(ctx))) return rc;
  BatchGibbs G;
  if ((rc = batch_gibbs_setup<T>(ctx, P, pb, ws, G))) return rc;
  if ((rc = gibbs_items(P, pb, rows, cols, G))) return rc;
  gibbs_launch<T>(P, pb, G, eps, rows, cols, w, at<T>(ws, cols ? P.o_wv : P.o_wu), out, ws, ctx->work);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

int batch_balance_t(uot_ctx* ctx, const uot_batch_problem* pb, double eps, float* v0, float* shift, char* ws,
                    size_t wsb) {
  BatchPlan P;
  int rc = make_batch_plan(P, pb);
  if (rc) return rc;
  if (P.dtype != UOT_F32) return fail(UOT_E_UNSUPPORTED, "the mass balance takes FP32 batches");
  if (pb->F1.kind != UOT_DIV_KL || pb->F2.kind != UOT_DIV_KL)
    return fail(UOT_E_UNSUPPORTED, "the mass balance takes KL penalties on both marginals");
  if (!(pb->F1.lambda > 0) || !(pb->F2.lambda > 0) || !std::isfinite(pb->F1.lambda) || !std::isfinite(pb->F2.lambda))
    return fail(UOT_E_INVALID, "KL lambda must be finite and > 0");
  if ((rc = check_batch_ws(P, ws, wsb, P.total))) return rc;
  if (!pb->x || !pb->y || !pb->p || !pb->q || !pb->dx || !pb->dy || !v0)
    return fail(UOT_E_INVALID, "x, y, p, q, dx, dy and v0 are required");
  if (!(eps > 0) || !std::isfinite(eps)) return fail(UOT_E_INVALID, "eps must be > 0");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  BatchGibbs G;
  if ((rc = batch_gibbs_setup<float>(ctx, P, pb, ws, G))) return rc;
  if ((rc = gibbs_items(P, pb, 0, 1, G))) return rc;
  // workspace slots of the solve reused here: w (totM), its log2 copy (totM), S (totN)
  float* w = at<float>(ws, P.o_logq);
  float* w2 = at<float>(ws, P.o_wv);
  float* S = at<float>(ws, P.o_wu);
  const float* dy = static_cast<const float*>(pb->dy);
  launch_balance_w(v0, dy, P.totM, eps, w, s);
  gibbs_launch<float>(P, pb, G, eps, 0, 1, w, w2, S, ws, s);
  launch_batch_balance(S, static_cast<const float*>(pb->p), static_cast<const float*>(pb->dx), G.offN_d,
                       static_cast<const float*>(pb->q), dy, G.offM_d, P.B, eps, pb->F1.lambda, pb->F2.lambda, v0,
                       shift, s);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

static_assert(kCloudFeatures == UOT_CLOUD_FEATURES, "feature count of the C header");

// the Gibbs products behind the cloud features (rows Y): columns, input and
// scale factor of eps per product, in feature order after eps log q
struct CloudProd {
  int cols;      // 0: X, 1: Y
  int input;     // 0: log p + log dx, 1: log q + log dy, 2: log dx, 3: log dy
  double a;      // product at eps a (kCloudWhole: the total over the problem)
};
constexpr double kCloudWhole = -1.0;   // a kernel equal to 1: the log of the total mass, per problem
constexpr CloudProd kCloudProds[kCloudFeatures - 2] = {
    {0, 0, 0.5}, {0, 0, 1.0}, {0, 0, 2.0}, {0, 0, 4.0},   // mass of the first measure near y_j
    {1, 1, 0.5}, {1, 1, 1.0}, {1, 1, 2.0}, {1, 1, 4.0},   // mass of the second measure near y_j
    {0, 2, 0.5}, {0, 2, 1.0}, {0, 2, 2.0},                // reference mass of the first cloud near y_j
    {1, 3, 1.0},                                          // reference mass of the second cloud near y_j
    {0, 0, kCloudWhole}, {1, 1, kCloudWhole}};            // total masses of the two measures

size_t cloud_extra_bytes(const BatchPlan& P) {
  return align_up(4 * (size_t)(kCloudFeatures - 2) * P.totM) + 2 * align_up(4 * (size_t)P.totN) +
         3 * align_up(4 * (size_t)P.totM);
}

int cloud_features_t(uot_ctx* ctx, const uot_batch_problem* pb, double eps, const float* shift, const float* scale,
                     float* x, char* ws, size_t wsb) {
  BatchPlan P;
  int rc = make_batch_plan(P, pb);
  if (rc) return rc;
  if (P.dtype != UOT_F32) return fail(UOT_E_UNSUPPORTED, "the cloud warm start takes FP32 batches");
  if ((rc = check_batch_ws(P, ws, wsb, P.total + cloud_extra_bytes(P)))) return rc;
  if (!pb->x || !pb->y || !pb->p || !pb->q || !pb->dx || !pb->dy || !shift || !scale || !x)
    return fail(UOT_E_INVALID, "x, y, p, q, dx, dy, shift, scale and x_out are required");
  if (!(eps > 0) || !std::isfinite(eps)) return fail(UOT_E_INVALID, "eps must be > 0");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  BatchGibbs G;
  if ((rc = batch_gibbs_setup<float>(ctx, P, pb, ws, G))) return rc;
  // rows Y against columns X go to the X items slot, rows Y against columns Y to the Y slot
  std::vector<BItem> it;
  build_items(pb->offM, pb->offN, P.B, 1, it);
  HIP_TRY(hipMemcpy(G.items[0], it.data(), sizeof(BItem) * it.size(), hipMemcpyHostToDevice));
  G.n_items[0] = (int)it.size();
  if ((rc = gibbs_items(P, pb, 1, 1, G))) return rc;
  char* ex = ws + P.total;
  float* prod = reinterpret_cast<float*>(ex);
  ex += align_up(4 * (size_t)(kCloudFeatures - 2) * P.totM);
  float* in_x[2];
  float* in_y[3];
  for (auto& p : in_x) { p = reinterpret_cast<float*>(ex); ex += align_up(4 * (size_t)P.totN); }
  for (auto& p : in_y) { p = reinterpret_cast<float*>(ex); ex += align_up(4 * (size_t)P.totM); }
  const float* px = static_cast<const float*>(pb->p);
  const float* qy = static_cast<const float*>(pb->q);
  const float* dxp = static_cast<const float*>(pb->dx);
  const float* dyp = static_cast<const float*>(pb->dy);
  launch_log_sum(px, dxp, in_x[0], P.totN, s);                 // log p + log dx
  launch_log<float>(dxp, in_x[1], P.totN, 0, s);               // log dx
  launch_log_sum(qy, dyp, in_y[0], P.totM, s);                 // log q + log dy
  launch_log<float>(dyp, in_y[1], P.totM, 0, s);               // log dy
  launch_log<float>(qy, in_y[2], P.totM, 1, s);                // log q
  const float* inputs[4] = {in_x[0], in_y[0], in_x[1], in_y[1]};
  for (int k = 0; k < kCloudFeatures - 2; ++k) {
    const CloudProd& c = kCloudProds[k];
    if (c.a == kCloudWhole) {
      launch_problem_lse(inputs[c.input], c.cols ? G.offM_d : G.offN_d, G.offM_d, P.B, prod + (int64_t)k * P.totM, s);
      continue;
    }
    // rows Y; the items slot of the columns' side holds the matching list
    BatchGibbs Gk = G;
    Gk.items[1] = G.items[c.cols];
    Gk.n_items[1] = G.n_items[c.cols];
    gibbs_launch<float>(P, pb, Gk, c.a * eps, 1, c.cols, inputs[c.input],
                        at<float>(ws, c.cols ? P.o_wv : P.o_wu),
                        prod + (int64_t)k * P.totM, ws, s);
  }
  launch_cloud_assemble(prod, kCloudFeatures - 2, in_y[2], G.offN_d, G.offM_d, P.B, P.totM, (float)eps, shift, scale,
                        x, s);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

template <typename T>
int batch_t(uot_ctx* ctx, const uot_batch_problem* pb, const uot_params* pr, T* u, T* v, char* ws, size_t wsb,
            uot_batch_result* res) {
  BatchPlan P;
  int rc = make_batch_plan(P, pb);
  if (rc) return rc;
  if (!ws) return fail(UOT_E_WORKSPACE, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(UOT_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (wsb < P.total) return fail(UOT_E_WORKSPACE, "workspace too small: need " + std::to_string(P.total));
  if (!u || !v || !pb->x || !pb->y || !pb->p || !pb->q || !pb->dx || !pb->dy)
    return fail(UOT_E_INVALID, "x, y, p, q, dx, dy, u, v are required");
  hipStream_t s = ctx->work;
  if ((rc = begin(ctx))) return rc;
  Ctrl* ctrl = at<Ctrl>(ws, P.o_ctrl);
  T *logp = at<T>(ws, P.o_logp), *logq = at<T>(ws, P.o_logq), *logdx = at<T>(ws, P.o_logdx),
    *logdy = at<T>(ws, P.o_logdy), *wu = at<T>(ws, P.o_wu), *wv = at<T>(ws, P.o_wv);
  BCtrl bc;
  bc.stop = at<int32_t>(ws, P.o_stop);
  bc.yskip = at<int32_t>(ws, P.o_yskip);
  bc.status = at<int32_t>(ws, P.o_status);
  bc.iters = at<int64_t>(ws, P.o_iters);
  bc.res = at<double>(ws, P.o_res);
  bc.clock = at<uint64_t>(ws, P.o_clock);
  BItem* itx = at<BItem>(ws, P.o_itx);
  BItem* ity = at<BItem>(ws, P.o_ity);
  int32_t* pstart_d = at<int32_t>(ws, P.o_pstart);
  int32_t* pstartY_d = at<int32_t>(ws, P.o_pstartY);
  ResPart* parts = at<ResPart>(ws, P.o_parts);
  T* bal_xm = at<T>(ws, P.o_bal);   // mass partials: X (m, s), then Y (m, s)
  T* bal_xs = bal_xm + P.max_items;
  T* bal_ym = bal_xs + P.max_items;
  T* bal_ys = bal_ym + P.max_items;
  int* curs = at<int>(ws, P.o_curs);
  int64_t* offN_d = at<int64_t>(ws, P.o_offN);
  int64_t* offM_d = at<int64_t>(ws, P.o_offM);
  int32_t* ordx_d = at<int32_t>(ws, P.o_ordx);
  int32_t* ordy_d = at<int32_t>(ws, P.o_ordy);
  BCtrl* bc_dev = nullptr;   // BCtrl itself travels by value inside a small device copy
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(offN_d, pb->offN, 8 * (P.B + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(offM_d, pb->offM, 8 * (P.B + 1), hipMemcpyHostToDevice));
  {
    std::vector<int32_t> ord;
    build_order(pb->offN, pb->offM, P.B, ord);
    HIP_TRY(hipMemcpy(ordx_d, ord.data(), 4 * P.B, hipMemcpyHostToDevice));
    build_order(pb->offM, pb->offN, P.B, ord);
    HIP_TRY(hipMemcpy(ordy_d, ord.data(), 4 * P.B, hipMemcpyHostToDevice));
  }
  BatchLists lists;
  lists.ord[0] = ordx_d;
  lists.ord[1] = ordy_d;
  lists.off[0] = offN_d;
  lists.off[1] = offM_d;
  lists.pstart = pstart_d;
  lists.pstartY = pstartY_d;
  lists.items[0] = itx;
  lists.items[1] = ity;
  lists.count[0] = curs;
  lists.count[1] = curs + 1;
  lists.cursor[0] = curs + 2;
  lists.cursor[1] = curs + 3;
  lists.rows = 256;
  // the BCtrl pointer block lives right after the Ctrl struct in the control slot
  bc_dev = reinterpret_cast<BCtrl*>(reinterpret_cast<char*>(ctrl) + align_up(sizeof(Ctrl), 64));
  HIP_TRY(hipMemcpy(bc_dev, &bc, sizeof(BCtrl), hipMemcpyHostToDevice));

  int ncu = 0;
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  int clock_khz = 0;
  HIP_TRY(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, ctx->device));
  const uot_geom dummy{};
  (void)dummy;
  // FP32: both sides in Morton order per problem; the iteration runs on the
  // ordered copies and the potentials are scattered back at the end
  const T* xo = static_cast<const T*>(pb->x);
  const T* yo = static_cast<const T*>(pb->y);
  T* uo = u;
  T* vo = v;
  const int32_t* px = nullptr;
  const int32_t* py = nullptr;
  float* pw = nullptr;
  if constexpr (std::is_same<T, float>::value) {
    if (P.mf) {
      float* xs = at<float>(ws, P.o_xs);
      float* ys = at<float>(ws, P.o_ys);
      int32_t* pxw = at<int32_t>(ws, P.o_permx);
      int32_t* pyw = at<int32_t>(ws, P.o_permy);
      uint32_t* code = at<uint32_t>(ws, P.o_code);
      float* box = at<float>(ws, P.o_box);
      launch_spatial_order_batch<float>(xo, P.totN, offN_d, P.B, P.nmaxN, P.dim, box, code, pxw, s);
      launch_spatial_order_batch<float>(yo, P.totM, offM_d, P.B, P.nmaxM, P.dim, box, code, pyw, s);
      launch_gather<float>(xo, pxw, P.totN, P.dim, xs, s);
      launch_gather<float>(yo, pyw, P.totM, P.dim, ys, s);
      HIP_TRY(hipGetLastError());
      xo = xs;
      yo = ys;
      px = pxw;
      py = pyw;
      uo = at<float>(ws, P.o_us);
      vo = at<float>(ws, P.o_vs);
      pw = at<float>(ws, P.o_pw);
    }
  }

  std::vector<int32_t> pst;
  // rows per item 256 R: the residual slots of the X items (the lists are
  // rebuilt on the device)
  auto upload_items = [&](int R) -> int {
    build_pstart(pb->offN, P.B, R, pst);
    HIP_TRY(hipMemcpy(pstart_d, pst.data(), 4 * (P.B + 1), hipMemcpyHostToDevice));
    build_pstart(pb->offM, P.B, R, pst);
    HIP_TRY(hipMemcpy(pstartY_d, pst.data(), 4 * (P.B + 1), hipMemcpyHostToDevice));
    lists.rows = 256 * R;
    return UOT_OK;
  };
  // the in-solve mass balance at iteration rebalance_at (0-based index
  // rebalance_at - 1: the X epilogue of that iteration and the Y epilogue of
  // the one before run while the counter holds it)
  const bool rebal = pr->rebalance_at >= 2;
  if (rebal && (pb->F1.kind != UOT_DIV_KL || pb->F2.kind != UOT_DIV_KL))
    return fail(UOT_E_UNSUPPORTED, "rebalance_at takes KL penalties on both marginals");
  BatchBalance<T> bbal{};
  if (rebal) {
    bbal.pxm = bal_xm;
    bbal.pxs = bal_xs;
    bbal.pym = bal_ym;
    bbal.pys = bal_ys;
    bbal.pstartY = pstartY_d;
    bbal.offN = offN_d;
    bbal.pot = uo;
    bbal.w = wu;
    bbal.iter = pr->rebalance_at - 1;
    bbal.lam1 = pb->F1.lambda;
    bbal.lam2 = pb->F2.lambda;
  }
  auto init_state = [&]() {
    Ctrl init = make_ctrl(pr->eps, pr->eps0, pr->eps_stages, pr->iters_per_stage, pr->tol, pr->max_iter);
    launch_ctrl_init(ctrl, init, s);
    launch_batch_init(bc_dev, (int)P.B, ctrl, s);
    launch_batch_compact(ctrl, bc_dev, (int)P.B, lists, s);   // every problem's items
    log_into<T>(pb->p, logp, P.totN, 1, px, uo, s);
    log_into<T>(pb->q, logq, P.totM, 1, py, vo, s);
    log_into<T>(pb->dx, logdx, P.totN, 0, px, uo, s);
    log_into<T>(pb->dy, logdy, P.totM, 0, py, vo, s);
    launch_init_pot<T>(nullptr, logdx, uo, nullptr, P.totN, P.totN, ctrl, 0, s);
    const T* v0 = static_cast<const T*>(pr->v0);
    if (v0 && py) {
      launch_gather<T>(v0, py, P.totM, 1, vo, s);
      v0 = vo;
    }
    launch_init_pot<T>(v0, logdy, vo, wv, P.totM, P.totM, ctrl, 0, s);
    // the matrix-core product starts with no row maxima (all bits set: not
    // finite), so the run does not depend on what the workspace held
    if (pw) (void)hipMemsetAsync(pw, 0xFF, sizeof(float) * (P.totN + P.totM), s);
  };
  int R = 1, bpc = 8;
  bool mfk = false;   // the matrix-core product (rows per item 256 R, R = 1 or 2)
  auto iteration = [&](int par) {
    EpiArgs<T> epx = prox_epi<T>(uo, wu, logp, logdx, nullptr, parts, P.totN, pb->F1);
    EpiArgs<T> epy = prox_epi<T>(vo, wv, logq, logdy, nullptr, nullptr, P.totM, pb->F2);
    if (rebal) {
      epx.bal_m = bal_xm;
      epx.bal_s = bal_xs;
      epy.bal_m = bal_ym;
      epy.bal_s = bal_ys;
      epx.bal_iter = epy.bal_iter = pr->rebalance_at - 1;
    }
    auto product = [&](int half, const BItem* items, int* count, const int64_t* offR, const int64_t* offC,
                       const T* xr, int64_t totR, const T* yc, int64_t totC, const T* w, float* pwr,
                       const EpiArgs<T>& ep) {
      if constexpr (std::is_same<T, float>::value) {
        if (mfk) {
          launch_batch_mf(P.dim, 4 * R, ncu * bpc, items, count, count + 2, offR, offC, xr, totR, yc, totC, w, pwr,
                          bc_dev, ctrl, half | par << 1, ep, mf_skip(ctrl, true), s);
          return;
        }
      }
      launch_batch_lse<T>(P.dim, R, ncu * bpc, items, count, count + 2, offR, offC, xr, totR, yc, totC, w, bc_dev,
                          ctrl, half | par << 1, ep, s);
    };
    // (count + 2: the list's work cursor)
    timed(0, [&] { product(0, itx, curs + 0, offN_d, offM_d, xo, P.totN, yo, P.totM, wv, pw, epx); });
    timed(2, [&] { launch_batch_control<T>(ctrl, bc_dev, (int)P.B, parts, pstart_d, lists, par, bbal, s); });
    timed(1, [&] {
      product(1, ity, curs + 1, offM_d, offN_d, yo, P.totM, xo, P.totN, wu, pw ? pw + P.totN : nullptr, epy);
    });
  };

  // autotuner: rows per item (256 R) and persistent blocks per CU, measured on
  // two iterations from the initial state; cached per batch signature
  if (pr->dense_kernel != 0 && pr->dense_kernel != 1 && pr->dense_kernel != 4)
    return fail(UOT_E_INVALID, "batches take dense_kernel 0 (tuned), 1 (direct) or 4 (matrix core)");
  if (pr->dense_kernel == 4 && !P.mf) return fail(UOT_E_UNSUPPORTED, "the matrix-core product takes FP32 data");
  std::string key = std::to_string(P.dtype) + ":" + std::to_string(P.dim) + ":" + std::to_string(P.B) + ":" +
                    std::to_string(P.totN) + ":" + std::to_string(P.totM) + ":" + std::to_string(pr->dense_kernel);
  {
    uint64_t hsh = 1469598103934665603ull;
    for (int64_t b = 0; b <= P.B; ++b) hsh = (hsh ^ (uint64_t)(pb->offN[b] * 31 + pb->offM[b])) * 1099511628211ull;
    key += ":" + std::to_string(hsh);
  }
  double tune_ms = 0.0;
  auto found = ctx->batch_tuned.find(key);
  if (found != ctx->batch_tuned.end()) {
    R = found->second.first & 15;
    mfk = (found->second.first & 16) != 0;
    bpc = found->second.second;
  } else {
    auto t0 = std::chrono::steady_clock::now();
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    int bestR = 1, bestB = 8;
    bool bestMf = false;
    // products: direct with 256 R rows per item (R = 1, 2, 4), and on FP32
    // data the matrix-core one (R = 1, 2: 4 or 8 row groups per wave)
    const int Rs[5] = {1, 2, 4, 1, 2};
    const int Bs[3] = {4, 8, 16};
    const int r_lo = pr->dense_kernel == 4 ? 3 : 0;
    const int r_hi = pr->dense_kernel == 1 || !P.mf ? 3 : 5;
    for (int ri = r_lo; ri < r_hi; ++ri) {
      if ((rc = upload_items(Rs[ri]))) return rc;
      // persistent blocks of the matrix-core product: none beyond what a
      // compute unit holds at once (4 of 4 row groups per wave, 2 of 8: its
      // launch bounds and LDS), or 4 when it holds fewer; blocks past that
      // only queue until the list is empty (measured at 8 per CU: about 5 %
      // slower per warm launch than at 4, a choice two timed iterations did
      // not reliably see)
      int nb = 3;
      if (ri >= 3) {
        const int res = batch_mf_resident_blocks(P.dim, 4 * Rs[ri]);
        nb = 0;
        while (nb < 3 && Bs[nb] <= std::max(res, 4)) ++nb;
      }
      for (int bi = 0; bi < nb; ++bi) {
        R = Rs[ri];
        mfk = ri >= 3;
        bpc = Bs[bi];
        init_state();
        iteration(0);   // first iteration: caches and code warm
        HIP_TRY(hipEventRecord(e0, s));
        iteration(1);
        iteration(0);
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        if (t < best) {
          best = t;
          bestR = R;
          bestB = bpc;
          bestMf = mfk;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    R = bestR;
    bpc = bestB;
    mfk = bestMf;
    ctx->batch_tuned[key] = {R | (mfk ? 16 : 0), bpc};
    tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if ((rc = upload_items(R))) return rc;
  init_state();
  HIP_TRY(hipGetLastError());

  // iteration loop: graph chunks (or timed direct launches) until no problem is active
  const int chunk = even_chunk(pr->check_every);
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  KTimer timer;
  timer.s = s;
  const bool timing = pr->kernel_ms != nullptr;
  if (timing) g_timer = &timer;
  struct Reset {
    ~Reset() { g_timer = nullptr; }
  } reset_timer;
  if (pr->use_graph && !timing) {
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < chunk; ++k) iteration(k & 1);
    HIP_TRY(hipStreamEndCapture(s, &graph));
    HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  auto t0 = std::chrono::steady_clock::now();
  int64_t launched = 0;
  rc = UOT_OK;
  while (true) {
    if (exec) {
      if (hipGraphLaunch(exec, s) != hipSuccess) { rc = fail(UOT_E_HIP, "hipGraphLaunch failed"); break; }
    } else {
      for (int k = 0; k < chunk; ++k) iteration(k & 1);
    }
    launched += chunk;
    if (hipMemcpyAsync(ctx->pinned, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(UOT_E_HIP, std::string("batch chunk failed: ") + hipGetErrorString(hipGetLastError()));
      break;
    }
    if (timing) timer.collect();
    const int64_t L = ctx->pinned->iter;
    if (L > 0 && ctx->pinned->active[(L - 1) & 1] == 0) break;
    if (launched > pr->max_iter + chunk) { rc = fail(UOT_E_HIP, "batch did not stop"); break; }
  }
  auto t1 = std::chrono::steady_clock::now();
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (rc) return rc;
  if (px) {
    launch_scatter<T>(uo, px, P.totN, u, s);
    launch_scatter<T>(vo, py, P.totM, v, s);
    HIP_TRY(hipGetLastError());
  }
  if (timing) {
    for (int k = 0; k < 4; ++k) {
      pr->kernel_ms[k] = timer.ms[k];
      if (pr->kernel_launches) pr->kernel_launches[k] = timer.count[k];
    }
    // class [3]: the matrix-core products' pair evaluations (the control
    // block as copied back after the last chunk)
    if (pr->kernel_launches) pr->kernel_launches[3] = (int64_t)ctx->pinned->pairs;
  }
  std::vector<int64_t> it(P.B);
  std::vector<double> rs(P.B);
  std::vector<int32_t> st(P.B);
  std::vector<uint64_t> ck(P.B);
  HIP_TRY(hipMemcpy(it.data(), bc.iters, 8 * P.B, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(rs.data(), bc.res, 8 * P.B, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(st.data(), bc.status, 4 * P.B, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(ck.data(), bc.clock, 8 * P.B, hipMemcpyDeviceToHost));
  const uint64_t t0c = ctx->pinned->t0_clock;
  int64_t nconv = 0, itmax = 0;
  bool nonfinite = false;
  for (int64_t b = 0; b < P.B; ++b) {
    if (res->iters) res->iters[b] = it[b];
    if (res->residual) res->residual[b] = rs[b];
    if (res->status) res->status[b] = st[b];
    if (res->latency_ms) res->latency_ms[b] = double(ck[b] - t0c) / double(clock_khz);
    nconv += (st[b] == 0);
    nonfinite |= (st[b] == -3);
    itmax = std::max(itmax, it[b]);
  }
  res->iters_max = itmax;
  res->n_converged = nconv;
  res->elapsed_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  res->tile_rows = 256 * R;
  res->blocks_per_cu = bpc;
  res->tune_ms = tune_ms;
  res->product = mfk ? 4 : 1;
  if ((rc = finish(ctx))) return rc;
  if (nonfinite) return fail(UOT_E_NONFINITE, "non-finite residual in a batch problem");
  return nconv == P.B ? UOT_OK : UOT_NOT_CONVERGED;
}

}  // namespace

// ---------------------------------------------------------------------------
// exported C ABI
// ---------------------------------------------------------------------------
extern "C" {

int uot_abi_version(void) { return UOT_ABI_VERSION; }

const char* uot_last_error(void) { return g_err.c_str(); }

const char* uot_status_string(int st) {
  switch (st) {
    case UOT_OK: return "ok";
    case UOT_NOT_CONVERGED: return "not converged (max_iter reached)";
    case UOT_E_INVALID: return "invalid argument";
    case UOT_E_UNSUPPORTED: return "unsupported configuration";
    case UOT_E_NONFINITE: return "non-finite residual";
    case UOT_E_HIP: return "HIP runtime error";
    case UOT_E_WORKSPACE: return "workspace missing, misaligned or too small";
    default: return "unknown status";
  }
}

int uot_create(uot_ctx** out, void* stream) {
  if (!out) return fail(UOT_E_INVALID, "out is NULL");
  uot_ctx* c = new (std::nothrow) uot_ctx();
  if (!c) return fail(UOT_E_INVALID, "out of host memory");
  c->user = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&c->device);
  // the no-allocation entry point's scratch on this device; a failure here
  // only disables that entry point, which reports it
  if (e == hipSuccess) c->scratch_err = scratch_address(c->device, &c->scratch);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&c->ev_t0);
  if (e == hipSuccess) e = hipEventCreate(&c->ev_t1);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&c->pinned), sizeof(Ctrl), hipHostMallocDefault);
  if (e != hipSuccess) {
    uot_destroy(c);
    return fail(UOT_E_HIP, std::string("uot_create: ") + hipGetErrorString(e));
  }
  *out = c;
  return UOT_OK;
}

int uot_destroy(uot_ctx* c) {
  if (!c) return UOT_OK;
  if (c->work) (void)hipStreamSynchronize(c->work);
  if (c->pending_exec) (void)hipGraphExecDestroy(c->pending_exec);
  if (c->pending_graph) (void)hipGraphDestroy(c->pending_graph);
  if (c->ev_t0) (void)hipEventDestroy(c->ev_t0);
  if (c->ev_t1) (void)hipEventDestroy(c->ev_t1);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->work) (void)hipStreamDestroy(c->work);
  delete c;
  return UOT_OK;
}

int uot_workspace_size(const uot_problem* pb, size_t* bytes) {
  if (!pb || !bytes) return fail(UOT_E_INVALID, "NULL argument");
  Plan P;
  int rc = make_plan(P, pb->dtype, pb->geom, 1, kMaxStages + 1);
  if (rc) return rc;
  *bytes = P.total;
  return UOT_OK;
}

int uot_solve(uot_ctx* ctx, const uot_problem* pb, const uot_params* pr, void* u, void* v, void* ws, size_t wsb,
              uot_result* res) {
  if (!ctx || !res) return fail(UOT_E_INVALID, "ctx and res are required");
  int rc = validate_problem(pb);
  if (rc) return rc;
  if ((rc = validate_params(pr))) return rc;
  if (pb->dtype == UOT_F32)
    return solve_t<float>(ctx, pb, pr, static_cast<float*>(u), static_cast<float*>(v), static_cast<char*>(ws), wsb, res);
  return solve_t<double>(ctx, pb, pr, static_cast<double*>(u), static_cast<double*>(v), static_cast<char*>(ws), wsb, res);
}

int uot_solve_async(uot_ctx* ctx, const uot_problem* pb, const uot_params* pr, void* u, void* v, void* ws,
                    size_t wsb) {
  if (!ctx) return fail(UOT_E_INVALID, "ctx is required");
  int rc = validate_problem(pb);
  if (rc) return rc;
  if ((rc = validate_params(pr))) return rc;
  uot_result unused{};
  if (pb->dtype == UOT_F32)
    return solve_t<float>(ctx, pb, pr, static_cast<float*>(u), static_cast<float*>(v), static_cast<char*>(ws), wsb,
                          &unused, 1, nullptr, nullptr, true);
  return solve_t<double>(ctx, pb, pr, static_cast<double*>(u), static_cast<double*>(v), static_cast<char*>(ws), wsb,
                         &unused, 1, nullptr, nullptr, true);
}

int uot_sync_result(uot_ctx* ctx, uot_result* res) {
  if (!ctx || !res) return fail(UOT_E_INVALID, "ctx and res are required");
  if (!ctx->pending) return fail(UOT_E_INVALID, "no asynchronous solve is pending on this context");
  const hipError_t e = hipStreamSynchronize(ctx->work);
  float ms = 0.f;
  const hipError_t et = e == hipSuccess ? hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1) : e;
  if (ctx->pending_exec) (void)hipGraphExecDestroy(ctx->pending_exec);
  if (ctx->pending_graph) (void)hipGraphDestroy(ctx->pending_graph);
  ctx->pending_exec = nullptr;
  ctx->pending_graph = nullptr;
  ctx->pending = false;
  if (e != hipSuccess) return fail(UOT_E_HIP, std::string("asynchronous solve failed: ") + hipGetErrorString(e));
  if (et != hipSuccess) return fail(UOT_E_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(et));
  const Ctrl& c = *ctx->pinned;
  res->iters = c.iter;
  res->residual = c.res;
  res->du_inf = c.du;
  res->status = c.status;
  res->elapsed_ms = ms;
  if (c.status == -3) return fail(UOT_E_NONFINITE, "non-finite residual");
  return c.status == 0 ? UOT_OK : UOT_NOT_CONVERGED;
}

int uot_fields_workspace_size(const uot_problem* pb, int nb, size_t* bytes) {
  if (!pb || !bytes) return fail(UOT_E_INVALID, "NULL argument");
  if (pb->geom.kind != UOT_GEOM_GRID) return fail(UOT_E_UNSUPPORTED, "field batches need a grid geometry");
  if (nb < 1) return fail(UOT_E_INVALID, "nb must be >= 1");
  Plan P;
  int rc = make_plan(P, pb->dtype, pb->geom, nb, kMaxStages + 1);
  if (rc) return rc;
  *bytes = P.total;
  return UOT_OK;
}

int uot_solve_fields(uot_ctx* ctx, const uot_problem* pb, int nb, const uot_params* pr, void* u, void* v, void* ws,
                     size_t wsb, uot_result* res) {
  if (!ctx || !res) return fail(UOT_E_INVALID, "ctx and res are required");
  int rc = validate_problem(pb);
  if (rc) return rc;
  if ((rc = validate_params(pr))) return rc;
  if (pb->geom.kind != UOT_GEOM_GRID) return fail(UOT_E_UNSUPPORTED, "field batches need a grid geometry");
  if (nb < 1) return fail(UOT_E_INVALID, "nb must be >= 1");
  if (pb->dtype == UOT_F32)
    return solve_t<float>(ctx, pb, pr, static_cast<float*>(u), static_cast<float*>(v), static_cast<char*>(ws), wsb,
                          res, nb);
  return solve_t<double>(ctx, pb, pr, static_cast<double*>(u), static_cast<double*>(v), static_cast<char*>(ws), wsb,
                         res, nb);
}

int uot_solve_mass(uot_ctx* ctx, const uot_problem* pb, const uot_div* F3, double mass, const uot_params* pr,
                   void* u, void* v, double* log_z, void* ws, size_t wsb, uot_result* res) {
  if (!ctx || !res || !F3 || !log_z) return fail(UOT_E_INVALID, "ctx, F3, log_z and res are required");
  int rc = validate_problem(pb);
  if (rc) return rc;
  if ((rc = check_div(*F3, "F3"))) return rc;
  if (!(mass > 0 && std::isfinite(mass))) return fail(UOT_E_INVALID, "mass must be finite and > 0");
  if ((rc = validate_params(pr))) return rc;
  if (pr->grid_kernel == 4) return fail(UOT_E_UNSUPPORTED, "the mass penalty runs with grid_kernel 0 .. 3");
  MassOpt m{to_dev(*F3), std::log(mass)};
  if (pb->dtype == UOT_F32)
    return solve_t<float>(ctx, pb, pr, static_cast<float*>(u), static_cast<float*>(v), static_cast<char*>(ws), wsb,
                          res, 1, &m, log_z);
  return solve_t<double>(ctx, pb, pr, static_cast<double*>(u), static_cast<double*>(v), static_cast<char*>(ws), wsb,
                         res, 1, &m, log_z);
}

int uot_barycentric_map(uot_ctx* ctx, const uot_problem* pb, double eps, const void* v, void* T, void* ws,
                        size_t wsb) {
  if (!ctx || !pb) return fail(UOT_E_INVALID, "ctx and problem are required");
  if (!pb->dy) return fail(UOT_E_INVALID, "dy is required");
  if (pb->dtype == UOT_F32)
    return map_t<float>(ctx, pb, eps, static_cast<const float*>(v), static_cast<float*>(T), static_cast<char*>(ws), wsb);
  if (pb->dtype == UOT_F64)
    return map_t<double>(ctx, pb, eps, static_cast<const double*>(v), static_cast<double*>(T), static_cast<char*>(ws),
                         wsb);
  return fail(UOT_E_INVALID, "dtype must be UOT_F32 or UOT_F64");
}

int uot_flow_workspace_size(const uot_flow_problem* fp, size_t* bytes) {
  if (!bytes) return fail(UOT_E_INVALID, "NULL argument");
  FlowDivs d;
  int rc = validate_flow(fp, d);
  if (rc) return rc;
  Plan P;
  size_t o_u = 0;
  if ((rc = flow_plan(P, fp, kMaxStages + 1, 0, 0.0, o_u))) return rc;
  *bytes = P.total;
  return UOT_OK;
}

int uot_flow(uot_ctx* ctx, const uot_flow_problem* fp, const uot_params* pr, int32_t n_steps, void* dens, void* v,
             void* ws, size_t wsb, uot_result* steps) {
  if (!ctx) return fail(UOT_E_INVALID, "ctx is required");
  FlowDivs d;
  int rc = validate_flow(fp, d);
  if (rc) return rc;
  if ((rc = validate_params(pr))) return rc;
  if (n_steps < 0) return fail(UOT_E_INVALID, "n_steps must be >= 0");
  if (pr->grid_kernel == 4) return fail(UOT_E_UNSUPPORTED, "flows run with grid_kernel 0 .. 3");
  if (fp->dtype == UOT_F32)
    return flow_t<float>(ctx, fp, d, pr, n_steps, static_cast<float*>(dens), static_cast<float*>(v),
                         static_cast<char*>(ws), wsb, steps);
  if (fp->dtype == UOT_F64)
    return flow_t<double>(ctx, fp, d, pr, n_steps, static_cast<double*>(dens), static_cast<double*>(v),
                          static_cast<char*>(ws), wsb, steps);
  return fail(UOT_E_INVALID, "dtype must be UOT_F32 or UOT_F64");
}

int uot_half_step(uot_ctx* ctx, const uot_problem* pb, double eps, int side, const void* pot_in, void* pot_io,
                  void* lse_out, double* residual, void* ws, size_t wsb) {
  if (!ctx) return fail(UOT_E_INVALID, "ctx is required");
  int rc = validate_problem(pb);
  if (rc) return rc;
  if (side != 0 && side != 1) return fail(UOT_E_INVALID, "side must be 0 or 1");
  if (pb->dtype == UOT_F32)
    return half_step_t<float>(ctx, pb, eps, side, static_cast<const float*>(pot_in), static_cast<float*>(pot_io),
                              static_cast<float*>(lse_out), residual, static_cast<char*>(ws), wsb);
  return half_step_t<double>(ctx, pb, eps, side, static_cast<const double*>(pot_in), static_cast<double*>(pot_io),
                             static_cast<double*>(lse_out), residual, static_cast<char*>(ws), wsb);
}

int uot_half_step_noalloc(uot_ctx* ctx, const uot_problem* pb, double eps, int side, const void* pot_in,
                          void* pot_io, void* lse_out, double* residual) {
  if (!ctx) return fail(UOT_E_INVALID, "ctx is required");
  int rc = validate_problem(pb);
  if (rc) return rc;
  if (!ctx->scratch)
    return fail(UOT_E_HIP, std::string("no scratch address on this device: ") + hipGetErrorString(ctx->scratch_err));
  // the plan uot_half_step makes for this problem; its workspace must fit
  Plan P;
  if ((rc = make_plan(P, pb->dtype, pb->geom, 1, 1, 0, eps))) return rc;
  if (P.total > (size_t)UOT_SCRATCH_BYTES)
    return fail(UOT_E_WORKSPACE, "this half-step needs " + std::to_string(P.total) +
                                     " bytes of scratch, more than the UOT_SCRATCH_BYTES = " +
                                     std::to_string((size_t)UOT_SCRATCH_BYTES) + " the library holds per GPU");
  return uot_half_step(ctx, pb, eps, side, pot_in, pot_io, lse_out, residual, ctx->scratch, UOT_SCRATCH_BYTES);
}

int uot_objective(uot_ctx* ctx, const uot_problem* pb, double eps, const void* u, const void* v, void* pi1, void* pi2,
                  uot_objective_values* out, void* ws, size_t wsb) {
  if (!ctx) return fail(UOT_E_INVALID, "ctx is required");
  int rc = validate_problem(pb);
  if (rc) return rc;
  if (pb->dtype == UOT_F32)
    return objective_t<float>(ctx, pb, eps, static_cast<const float*>(u), static_cast<const float*>(v),
                              static_cast<float*>(pi1), static_cast<float*>(pi2), out, static_cast<char*>(ws), wsb);
  return objective_t<double>(ctx, pb, eps, static_cast<const double*>(u), static_cast<const double*>(v),
                             static_cast<double*>(pi1), static_cast<double*>(pi2), out, static_cast<char*>(ws), wsb);
}

int uot_time_fields_half_step(uot_ctx* ctx, const uot_problem* pb, int nb, double eps, const void* v, int reps,
                              double* ms, int* n_kernels, void* ws, size_t wsb, int grid_kernel) {
  if (!ctx) return fail(UOT_E_INVALID, "ctx is required");
  int rc = validate_problem(pb);
  if (rc) return rc;
  if (!(eps > 0)) return fail(UOT_E_INVALID, "eps must be > 0");
  if (pb->dtype == UOT_F32)
    return time_half_step_t<float>(ctx, pb, nb, eps, static_cast<const float*>(v), reps, ms, n_kernels,
                                   static_cast<char*>(ws), wsb, grid_kernel);
  return time_half_step_t<double>(ctx, pb, nb, eps, static_cast<const double*>(v), reps, ms, n_kernels,
                                  static_cast<char*>(ws), wsb, grid_kernel);
}

int uot_time_half_step(uot_ctx* ctx, const uot_problem* pb, double eps, const void* v, int reps, double* ms,
                       int* n_kernels, void* ws, size_t wsb, int grid_kernel) {
  return uot_time_fields_half_step(ctx, pb, 1, eps, v, reps, ms, n_kernels, ws, wsb, grid_kernel);
}

int uot_tuning_export(uot_ctx* ctx, char* buf, size_t cap, size_t* len) {
  if (!ctx || !len) return fail(UOT_E_INVALID, "ctx and len are required");
  std::string t;
  for (const auto& e : ctx->batch_tuned) {
    const int R = e.second.first & 15;
    const bool mf = (e.second.first & 16) != 0;
    t += "batch " + e.first + " " + (mf ? "4" : "1") + " " + std::to_string(R) + " " + std::to_string(e.second.second) +
         "\n";
  }
  for (const auto& e : ctx->dense_tuned) t += "dense " + e.first + " " + std::to_string(e.second) + "\n";
  *len = t.size() + 1;
  if (!buf || cap < t.size() + 1) return fail(UOT_E_INVALID, "buffer too small for the tuning table");
  std::memcpy(buf, t.c_str(), t.size() + 1);
  return UOT_OK;
}

int uot_tuning_import(uot_ctx* ctx, const char* text) {
  if (!ctx || !text) return fail(UOT_E_INVALID, "ctx and text are required");
  std::map<std::string, std::pair<int, int>> batch;
  std::map<std::string, int> dense;
  const std::string all(text);
  size_t pos = 0;
  int line_no = 0;
  while (pos <= all.size()) {
    size_t end = all.find('\n', pos);
    if (end == std::string::npos) end = all.size();
    const std::string line = all.substr(pos, end - pos);
    pos = end + 1;
    ++line_no;
    if (line.find_first_not_of(" \t\r") == std::string::npos) {
      if (end == all.size()) break;
      continue;
    }
    std::istringstream in(line);
    std::string kind, sig, extra;
    if (!(in >> kind >> sig)) return fail(UOT_E_INVALID, "tuning table line " + std::to_string(line_no) + ": no signature");
    if (kind == "batch") {
      int product = 0, R = 0, bpc = 0;
      if (!(in >> product >> R >> bpc) || (in >> extra))
        return fail(UOT_E_INVALID, "tuning table line " + std::to_string(line_no) + ": expected three numbers");
      const bool mf = product == 4;
      const bool ok = (product == 1 && (R == 1 || R == 2 || R == 4)) || (mf && (R == 1 || R == 2));
      if (!ok || !(bpc == 4 || bpc == 8 || bpc == 16))
        return fail(UOT_E_INVALID, "tuning table line " + std::to_string(line_no) + ": not a choice of the batch tuner");
      batch[sig] = {R | (mf ? 16 : 0), bpc};
    } else if (kind == "dense") {
      int target = 0;
      if (!(in >> target) || (in >> extra))
        return fail(UOT_E_INVALID, "tuning table line " + std::to_string(line_no) + ": expected one number");
      bool ok = false;
      for (int k = 0; k < kMfNTargets; ++k) ok = ok || target == kMfTargets[k];
      if (!ok) return fail(UOT_E_INVALID, "tuning table line " + std::to_string(line_no) + ": not a block target");
      dense[sig] = target;
    } else {
      return fail(UOT_E_INVALID, "tuning table line " + std::to_string(line_no) + ": unknown kind '" + kind + "'");
    }
    if (end == all.size()) break;
  }
  for (const auto& e : batch) ctx->batch_tuned[e.first] = e.second;
  for (const auto& e : dense) ctx->dense_tuned[e.first] = e.second;
  return UOT_OK;
}

int uot_probe_rates(uot_ctx* ctx, double* exp_per_s, double* add_per_s) {
  if (!ctx || !exp_per_s || !add_per_s) return fail(UOT_E_INVALID, "NULL argument");
  int ncu = 0;
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  const int blocks = ncu * 16;     // 64 waves per CU: the issue ports stay busy
  const int iters = 4096;
  float* buf = nullptr;
  HIP_TRY(hipMalloc(&buf, sizeof(float) * (size_t)blocks * 256));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double rates[2];
  for (int which = 0; which < 2; ++which) {
    launch_probe(which, buf, blocks, iters, ctx->work);   // warm-up
    HIP_TRY(hipEventRecord(e0, ctx->work));
    launch_probe(which, buf, blocks, iters, ctx->work);
    HIP_TRY(hipEventRecord(e1, ctx->work));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    rates[which] = double(blocks) * 256.0 * iters * 8.0 / (double(t) * 1e-3);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(hipFree(buf));
  *exp_per_s = rates[0];
  *add_per_s = rates[1];
  return UOT_OK;
}

int uot_batch_workspace_size(const uot_batch_problem* pb, size_t* bytes) {
  if (!pb || !bytes) return fail(UOT_E_INVALID, "NULL argument");
  BatchPlan P;
  int rc = make_batch_plan(P, pb);
  if (rc) return rc;
  *bytes = P.total;
  return UOT_OK;
}

int uot_batch_gibbs(uot_ctx* ctx, const uot_batch_problem* pb, double eps, int rows, int cols, const void* w,
                    void* out, void* ws, size_t wsb) {
  if (!ctx || !pb) return fail(UOT_E_INVALID, "ctx and problem are required");
  if (pb->dtype == UOT_F32)
    return batch_gibbs_t<float>(ctx, pb, eps, rows, cols, static_cast<const float*>(w), static_cast<float*>(out),
                                static_cast<char*>(ws), wsb);
  return batch_gibbs_t<double>(ctx, pb, eps, rows, cols, static_cast<const double*>(w), static_cast<double*>(out),
                               static_cast<char*>(ws), wsb);
}

int uot_batch_balance(uot_ctx* ctx, const uot_batch_problem* pb, double eps, void* v0, void* shift, void* ws,
                      size_t wsb) {
  if (!ctx || !pb) return fail(UOT_E_INVALID, "ctx and problem are required");
  return batch_balance_t(ctx, pb, eps, static_cast<float*>(v0), static_cast<float*>(shift), static_cast<char*>(ws),
                         wsb);
}

int uot_cloud_features_workspace_size(const uot_batch_problem* pb, size_t* bytes) {
  if (!pb || !bytes) return fail(UOT_E_INVALID, "NULL argument");
  BatchPlan P;
  int rc = make_batch_plan(P, pb);
  if (rc) return rc;
  *bytes = P.total + cloud_extra_bytes(P);
  return UOT_OK;
}

int uot_cloud_features(uot_ctx* ctx, const uot_batch_problem* pb, double eps, const float* shift, const float* scale,
                       float* x, void* ws, size_t wsb) {
  if (!ctx || !pb) return fail(UOT_E_INVALID, "ctx and problem are required");
  return cloud_features_t(ctx, pb, eps, shift, scale, x, static_cast<char*>(ws), wsb);
}

int uot_cloud_v0(uot_ctx* ctx, const float* q, int64_t n, double zeps, const float* y, double out_scale,
                 double out_shift, float* v0) {
  if (!ctx || !q || !y || !v0 || n < 1) return fail(UOT_E_INVALID, "q, y, v0 and n >= 1 are required");
  int rc = begin(ctx);
  if (rc) return rc;
  launch_cloud_v0(y, q, n, (float)zeps, (float)out_scale, (float)out_shift, v0, ctx->work);
  HIP_TRY(hipGetLastError());
  return finish(ctx);
}

int uot_solve_batched(uot_ctx* ctx, const uot_batch_problem* pb, const uot_params* pr, void* u, void* v, void* ws,
                      size_t wsb, uot_batch_result* res) {
  if (!ctx || !pb || !res) return fail(UOT_E_INVALID, "ctx, problem and res are required");
  int rc = check_div(pb->F1, "F1");
  if (rc) return rc;
  if ((rc = check_div(pb->F2, "F2"))) return rc;
  if ((rc = validate_params(pr, true))) return rc;
  if (pb->dtype == UOT_F32)
    return batch_t<float>(ctx, pb, pr, static_cast<float*>(u), static_cast<float*>(v), static_cast<char*>(ws), wsb, res);
  return batch_t<double>(ctx, pb, pr, static_cast<double*>(u), static_cast<double*>(v), static_cast<char*>(ws), wsb,
                         res);
}

int uot_bary_workspace_size(const uot_bary_problem* pb, size_t* bytes) {
  if (!pb || !bytes) return fail(UOT_E_INVALID, "NULL argument");
  if (pb->geom.kind != UOT_GEOM_GRID) return fail(UOT_E_UNSUPPORTED, "barycentres need a grid geometry");
  if (pb->n < 1) return fail(UOT_E_INVALID, "a barycentre needs n >= 1 marginals");
  if (pb->n > kMaxBary) return fail(UOT_E_UNSUPPORTED, "at most 64 marginals");
  Plan P;
  int rc = make_plan(P, pb->dtype, pb->geom, pb->n, kMaxStages + 1);
  if (rc) return rc;
  *bytes = P.total;
  return UOT_OK;
}

int uot_barycenter(uot_ctx* ctx, const uot_bary_problem* pb, const uot_params* pr, void* u, void* v, void* logh,
                   void* ws, size_t wsb, uot_result* res) {
  if (!ctx || !pb || !res) return fail(UOT_E_INVALID, "ctx, problem and res are required");
  if (pb->geom.kind != UOT_GEOM_GRID) return fail(UOT_E_UNSUPPORTED, "barycentres need a grid geometry");
  if (pb->n < 1) return fail(UOT_E_INVALID, "a barycentre needs n >= 1 marginals");
  if (pb->n > kMaxBary) return fail(UOT_E_UNSUPPORTED, "at most 64 marginals");
  if (!pb->p || !pb->dx || !pb->dy || !pb->alpha) return fail(UOT_E_INVALID, "p, dx, dy, alpha are required");
  for (int k = 0; k < pb->n; ++k)
    if (!(pb->alpha[k] > 0)) return fail(UOT_E_INVALID, "alpha_k must be > 0");
  int rc = check_div(pb->F1, "F1");
  if (rc) return rc;
  if ((rc = check_div(pb->F2, "F2"))) return rc;
  if (pb->F2.kind == UOT_DIV_RG && !std::isfinite(pb->F2.beta))
    return fail(UOT_E_UNSUPPORTED, "a range barycentre needs a finite upper bound beta");
  if (pb->F2.kind == UOT_DIV_GROWTH)
    return fail(UOT_E_UNSUPPORTED, "the barycentre side takes =, KL, TV or RG (Table estimatebary)");
  if ((rc = validate_params(pr))) return rc;
  if (pb->dtype == UOT_F32)
    return bary_t<float>(ctx, pb, pr, static_cast<float*>(u), static_cast<float*>(v), static_cast<float*>(logh),
                         static_cast<char*>(ws), wsb, res);
  return bary_t<double>(ctx, pb, pr, static_cast<double*>(u), static_cast<double*>(v), static_cast<double*>(logh),
                        static_cast<char*>(ws), wsb, res);
}

}  // extern "C"
