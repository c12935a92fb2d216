// Host-side launch interface between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "uot_device.h"

namespace uot {

enum EpiMode { EPI_RAW = 0, EPI_PROX = 1 };

// cost of a geometry: kind 0 squared Euclidean, 1 WF with cut locus `cut`
struct CostArgs {
  int kind;
  int pad;
  double cut;
};

// What the last pass of a Gibbs product does with S2 = log2 of the product.
//  EPI_RAW : out[e] = S2
//  EPI_PROX: pot[e] = eps log proxdiv_F(e^S) (old value read first), wnext[e] =
//            (pot/eps_next + logd) log2(e), lse_out[e] = S (optional), and,
//            when part != nullptr, residual partials per block.
template <typename T> struct EpiArgs {
  int mode;
  int pad;
  T* out;
  T* pot;
  T* wnext;
  const T* logp;
  const T* logd;
  T* lse_out;
  ResPart* part;
  int64_t size;   // elements per field: logd is indexed by e % size
  DivDev F;
  // hosted control step (first Y pass of a single-problem grid solve): when
  // host_ctl is set, block 0 of the launch also runs the control step of the
  // iteration on the host_nparts residual partials of the X half-step
  Ctrl* host_ctl;
  const ResPart* host_parts;
  double* host_hist;
  int host_nparts;
  int host_pad;
  // total-mass penalty (Y side): per-block log2-sum-exp partials (m, s) of
  // T + v/eps + log d, the log mass of the plan without the factor z
  T* mass_m;
  T* mass_s;
  // ragged batches: in the half-steps that run while the control block's
  // iteration counter equals bal_iter, each work item also writes the plan's
  // marginal mass over its rows, the log2-sum-exp (bal_m, bal_s)[item part]
  // of S2 + (pot/eps + log d) log2(e); null: off
  T* bal_m;
  T* bal_s;
  int64_t bal_iter;
};

// the in-solve mass balance of a ragged batch (KL on both marginals), taken
// by the control step of iteration `iter`: per running problem the X and Y
// mass partials give s = log(P/Q) / (theta1/lam1 + 1/lam2), and the X side's
// potentials and column weights move by theta1 s; px null: off
template <typename T> struct BatchBalance {
  const T *pxm, *pxs;       // X items' partials (m, s), slots pstart; null: off
  const T *pym, *pys;       // Y items' partials, slots pstartY
  const int32_t* pstartY;   // first Y slot of each problem
  const int64_t* offN;      // X rows of each problem
  T* pot;                   // X potentials (u)
  T* w;                     // X column weights (u/eps + log dx) log2(e)
  int64_t iter;
  double lam1, lam2;
};

template <typename T> void launch_log(const T* src, T* dst, int64_t n, int zero_is_ninf, hipStream_t s);
template <typename T>
void launch_init_pot(const T* v0, const T* logd, T* pot, T* w, int64_t n, int64_t size, const Ctrl* c, int which,
                     hipStream_t s);
template <typename T>
void launch_gtab(T* tab, int n, double h, const Ctrl* c, int nst, const CostArgs& cost, hipStream_t s);
template <typename T> void launch_gtab_cost(T* tab, int n, double h, double eps, const CostArgs& cost, hipStream_t s);
template <typename T> int grid_strided_parts(int n, int64_t A, int64_t B);
template <typename T> int grid_contig_parts(int n, int64_t A);
template <typename T>
void launch_grid_strided(const T* in, int64_t A, int n, int64_t B, const T* gtab, int side, const Ctrl* c,
                         const EpiArgs<T>& ep, hipStream_t s);
template <typename T>
void launch_grid_contig(const T* in, int64_t A, int n, const T* gtab, int side, const Ctrl* c,
                        const EpiArgs<T>& ep, int band, hipStream_t s);
// few long lines: tap slices (grid_contig_splits) with partial LSEs in pm / ps
// (nsplit x A x n each), merged by launch_dense_epi over A n outputs
int grid_contig_splits(int n, int64_t A, int band);
template <typename T>
void launch_grid_contig_split(const T* in, int64_t A, int n, const T* gtab, int side, const Ctrl* c, int band,
                              int nsplit, T* pm, T* ps, hipStream_t s);
template <typename T>
void launch_dense_lse(int dim, int R, const T* xr, int64_t Nr, const T* yc, const T* w, int64_t Mc, int nsplit,
                      int64_t cps, T* pm, T* ps, int side, const Ctrl* c, const CostArgs& cost, hipStream_t s);
// boxes of consecutive chunks of `per` points (SoA, n points, dim <= 3):
// out[6 b + 2 d], out[6 b + 2 d + 1] = min, max of coordinate d over chunk b
template <typename T>
void launch_chunk_boxes(const T* pts, int64_t n, int64_t per, int dim, T* out, hipStream_t s);
// WF point clouds on work lists (one side: rows against columns): boxes of
// the row waves (6 per 64 rows) and of the column groups (6 per 16
// columns), the mask of (row wave, group) pairs within the cut (nwd =
// ceil(groups / 32) words per row wave), the work units (group range
// [g0, g1) holding up to 16 groups within the cut) of each row wave in
// slots k nrw + rw, and their count per row wave
template <typename T> struct WfLists {
  T* rbox;
  T* gbox;
  uint32_t* mask;
  int2* units;
  int* ucnt;
  int* umax;   // the largest unit count of a row wave
};
template <typename T>
void launch_wf_lists(const T* rows, int64_t Nr, const T* cols, int64_t Mc, int dim, double cut, const WfLists<T>& L,
                     hipStream_t s);
// partial log2-sum-exp of every unit (pm, ps: 64 per unit slot)
template <typename T>
void launch_wf_lse(int dim, const T* xr, int64_t Nr, const T* yc, const T* w, int64_t Mc, double cut,
                   const WfLists<T>& L, int umax, T* pm, T* ps, int side, const Ctrl* c, hipStream_t s);
// merge of each row's units in unit order, then the epilogue
template <typename T>
void launch_wf_epi(const T* pm, const T* ps, const WfLists<T>& L, int64_t Nr, int64_t Mc, int side, const Ctrl* c,
                   const EpiArgs<T>& ep, hipStream_t s);
template <typename T>
void launch_dense_epi(const T* pm, const T* ps, int nsplit, int64_t Nr, int side, const Ctrl* c,
                      const EpiArgs<T>& ep, hipStream_t s);
void launch_control(Ctrl* c, const ResPart* part, int nparts, double* hist, hipStream_t s, int nfields, int par);
void launch_res_reduce(const ResPart* part, int nparts, double* out, hipStream_t s);
void launch_ctrl_init(Ctrl* c, const Ctrl& init, hipStream_t s);
void launch_ctrl_resume(Ctrl* c, double tol, hipStream_t s);
// slot 0 valid again after a stopped solve (one more product at the last eps)
// spatial (Morton) order of n points (dim x n, coordinate-major): box (6),
// codes (n) and the permutation perm (n, sorted position -> original index)
template <typename T>
void launch_spatial_order(const T* x, int64_t n, int dim, T* box, uint32_t* code, int32_t* perm, hipStream_t s);
template <typename T> void launch_gather(const T* in, const int32_t* perm, int64_t n, int nrow, T* out, hipStream_t s);
template <typename T> void launch_scatter(const T* in, const int32_t* perm, int64_t n, T* out, hipStream_t s);
// tile-factored dense product (FP32, R = 2), partials as launch_dense_lse
void launch_dense_tf(int dim, const float* xr, int64_t Nr, const float* yc, const float* w, int64_t Mc, int nsplit,
                     int64_t cps, float* pm, float* ps, int side, const Ctrl* c, hipStream_t s);
// Morton order of each problem of a batch (problem b: points off[b] ..
// off[b + 1] - 1, coordinate stride tot; nmax: the largest problem; box: 6
// per problem); perm maps within each problem's range
template <typename T>
void launch_spatial_order_batch(const T* x, int64_t tot, const int64_t* off, int64_t B, int64_t nmax, int dim,
                                T* box, uint32_t* code, int32_t* perm, hipStream_t s);
// the matrix-core products' negligible tiles: on leaves them out (the
// UOT_TILE_SKIP environment switch, on unless it is 0); pairs (device, or
// null) accumulates the pair evaluations the products perform
struct MfSkip {
  int on = 1;
  unsigned long long* pairs = nullptr;
};
bool tile_skip_enabled();
// the ragged batch on the matrix cores (BF16 x 3 operands, FP32 data, squared
// Euclidean): groups = 4 or 8 row groups of 16 per wave (items of 64 groups
// rows); *count items of the list, pulled from *cursor (zero at launch);
// pw: starting row maxima (totR), kept between iterations
// blocks of launch_batch_mf's kernel that one compute unit holds at once
// (its launch bounds, registers and LDS), 0 if the query fails
int batch_mf_resident_blocks(int dim, int groups);
void launch_batch_mf(int dim, int groups, int blocks, const BItem* items, const int* count, int* cursor,
                     const int64_t* offR, const int64_t* offC, const float* xr, int64_t totR, const float* yc,
                     int64_t totC, const float* w, float* pw, const BCtrl* bc, const Ctrl* c, int side,
                     const EpiArgs<float>& ep, const MfSkip& sk, hipStream_t s);
// dense product on the matrix cores (FP32 data, squared Euclidean): groups =
// 4 or 8 row groups of 16 per wave; split: BF16 x 3 operands on
// v_mfma_f32_16x16x32_bf16, else FP32 operands on v_mfma_f32_16x16x4f32;
// pw (nsplit x Nr, kept between the products of one side): the row maxima
// the product starts from and leaves for the next one
void launch_dense_mf(int dim, int groups, bool split, const float* xr, int64_t Nr, const float* yc, const float* w,
                     int64_t Mc, int nsplit, int64_t cps, float* pm, float* ps, float* pw, int side, const Ctrl* c,
                     const MfSkip& sk, hipStream_t s);
template <typename T>
void launch_coord_weight(const T* w, T* out, int64_t M, int64_t stride, int64_t nk, double hk, const T* yk, int sign,
                         hipStream_t s);
template <typename T> void launch_map_finish(T* num, const T* den, const T* neg, int64_t N, hipStream_t s);
void launch_ctrl_post(Ctrl* c, hipStream_t s);
template <typename T>
void launch_growth_combine(const T* T2, int nm, int64_t size, const DivDev& F, const T* logq, const T* logdy, T* v,
                           T* w, const Ctrl* c, int side, hipStream_t s);
template <typename T>
void launch_flow_next(const T* T2, const T* v, const T* logq, int nm, int64_t size, int growth, double log_kappa,
                      const Ctrl* c, T* out, hipStream_t s);
template <typename T>
void launch_mass_update(Ctrl* c, const T* mass_m, const T* mass_s, int nparts, const DivDev& F3, double log_m0, int par,
                        hipStream_t s);
constexpr int kMaxBary = 64;
struct BaryW {
  double v[kMaxBary];   // log alpha_k
  double a[kMaxBary];   // alpha_k
};
template <typename T>
void launch_bary_combine(const T* T2, int nm, int64_t size, const BaryW& log_alpha, double log_sum_alpha,
                         const DivDev& F2, const T* logdy, T* v, T* w, T* logh, const Ctrl* c, int side,
                         hipStream_t s);
template <typename T>
int launch_obj_side(const T* pot, const T* S, const T* p, const T* d, int64_t n, double eps, const DivDev& F,
                    T* pi_out, double* part, hipStream_t s);
template <typename T> int launch_sum_exp2(const T* a, const T* b, int64_t n, double* part, hipStream_t s);
template <typename T>
void launch_dense_cost(int dim, const T* xr, int64_t Nr, const T* yc, const T* w, int64_t Mc, double eps, T* out,
                       const CostArgs& cost, hipStream_t s);

void launch_probe(int which, float* out, int blocks, int iters, hipStream_t s);
int grid_tf_parts(int n, int64_t A, int64_t B, bool strided);
void launch_grid_tf(const float* in, int64_t A, int n, int64_t B, bool strided, bool half, double h, int side,
                    const Ctrl* c, const EpiArgs<float>& ep, hipStream_t s);
// direct batch product over *count items of the list (256 R rows per item),
// pulled from *cursor (zero at launch)
template <typename T>
void launch_batch_lse(int dim, int R, int blocks, const BItem* items, const int* count, int* cursor,
                      const int64_t* offR, const int64_t* offC, const T* xr, int64_t totR, const T* yc, int64_t totC,
                      const T* w, const BCtrl* bc, const Ctrl* c, int side, const EpiArgs<T>& ep, hipStream_t s);
// per-problem control after the X half-step, then the work cursors, the item
// lists (rebuilt when enough problems stopped) and the iteration's eps
// bookkeeping
template <typename T>
void launch_batch_control(Ctrl* c, BCtrl* bc, int B, const ResPart* part, const int32_t* pstart,
                          const BatchLists& L, int par, const BatchBalance<T>& bal, hipStream_t s);
// the item lists of every problem and zero cursors (no bookkeeping): the
// start of a solve
void launch_batch_compact(Ctrl* c, const BCtrl* bc, int B, const BatchLists& L, hipStream_t s);
void launch_balance_w(const float* v0, const float* dy, int64_t n, double eps, float* w, hipStream_t s);
// mass balance of a starting potential v0 of a ragged batch (KL on both
// marginals), in place; S: log K(e^{v0/eps} dy) per X point; shift: [B] or null
void launch_batch_balance(const float* S, const float* p, const float* dx, const int64_t* offN, const float* q,
                          const float* dy, const int64_t* offM, int64_t B, double eps, double lam1, double lam2,
                          float* v0, float* shift, hipStream_t s);
void launch_batch_init(BCtrl* bc, int B, Ctrl* c, hipStream_t s);
void launch_set_int(int* p, int n, int v, hipStream_t s);
template <typename T> void launch_scale(T* a, int64_t n, double f, hipStream_t s);

// warm start of ragged point-cloud batches (uot_net.hip)
constexpr int kCloudFeatures = 16;   // UOT_CLOUD_FEATURES of the C header
void launch_log_sum(const float* a, const float* b, float* out, int64_t n, hipStream_t s);
void launch_cloud_assemble(const float* prod, int n_prod, const float* logq, const int64_t* offN, const int64_t* offM,
                           int64_t B, int64_t totM, float eps, const float* shift, const float* scale, float* x,
                           hipStream_t s);
void launch_problem_lse(const float* w, const int64_t* offC, const int64_t* offR, int64_t B, float* out,
                        hipStream_t s);
void launch_cloud_v0(const float* y, const float* q, int64_t n, float zeps, float out_scale, float out_shift,
                     float* v0, hipStream_t s);

}  // namespace uot
