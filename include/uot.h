/*
 * uot.h -- C ABI of libuot: entropic unbalanced optimal transport by the
 * generalized Sinkhorn scaling iteration, hand-written HIP kernels for
 * MI355X (gfx950).
 *
 * Method: Chizat, Peyre, Schmitzer, Vialard, "Scaling algorithms for
 * unbalanced optimal transport problems".
 *
 *   problem      (P_eps)  min_R F1(R dy) + F2(R^T dx) + eps KL(R | K),
 *                K = exp(-C/eps), dx (x) dy-weighted entropy   (Sec. 3.2, eq. (P_eps))
 *   iteration    (S)      a <- proxdiv_F1(K(b dy)), b <- proxdiv_F2(K^T(a dx))
 *                                                        (Sec. 3.3, Algorithm 1)
 *   proxdiv      Table "proximalexplicit" (Sec. 5.1), stabilized form (Sec. 4.3)
 *
 * Everything runs in the log domain: the library stores the dual potentials
 * u = eps log a and v = eps log b (Prop. "alternating"), i.e. Algorithm 2 with
 * an absorption after every half-step, so that no kernel entry ever over- or
 * underflows for small eps.  The plan w.r.t. dx (x) dy is
 *     R_ij = exp((u_i + v_j - C_ij)/eps)                  (Thm. "duality").
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers (hipMalloc'd or torch CUDA
 *     tensors), caller-owned; the library neither frees nor retains them.
 *   - Float arrays have the problem's dtype (UOT_F64 = double, UOT_F32 = float).
 *   - p, q are DENSITIES w.r.t. the reference weights dx, dy (p = mu/dx,
 *     Sec. 5.1); p_i = 0 is allowed and gives u_i = -inf under KL/=/RG.
 *   - Workspace: the caller allocates ws_bytes >= uot_*_workspace_size(...)
 *     bytes of device memory (256-byte aligned); the library allocates no
 *     device memory inside any solve.
 *   - Work is enqueued on the stream given to uot_create (NULL = the legacy
 *     default stream).  Calls that return scalar results synchronise that
 *     stream before returning.
 *   - Return value: UOT_OK (0), UOT_NOT_CONVERGED (1, informational), or a
 *     negative error; no exception ever crosses the ABI.  uot_last_error()
 *     gives a message for the last error on the calling thread.
 */
#ifndef UOT_H
#define UOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UOT_ABI_VERSION 3

enum uot_status_code {
  UOT_OK = 0,
  UOT_NOT_CONVERGED = 1,   /* max_iter reached before residual <= tol        */
  UOT_E_INVALID = -1,      /* bad shape, pointer, eps <= 0, lambda <= 0 ...  */
  UOT_E_UNSUPPORTED = -2,  /* valid but not implemented (e.g. dim > 3)       */
  UOT_E_NONFINITE = -3,    /* a NaN residual was detected on the device      */
  UOT_E_HIP = -4,          /* a HIP runtime call failed                       */
  UOT_E_WORKSPACE = -5     /* workspace missing, too small or misaligned     */
};

/* Marginal penalties F(s) = sum_i dx_i Dbar_phi(s_i | p_i)  (Sec. 2.1 and
 * eq. "divergencefunctions"); proxdiv rows of Table proximalexplicit:
 *   UOT_DIV_EQ : equality constraint, proxdiv = p/s
 *   UOT_DIV_KL : lambda KL,           proxdiv = (p/s)^(lambda/(lambda+eps))
 *   UOT_DIV_TV : lambda TV,           proxdiv = min(e^(lambda/eps), max(e^(-lambda/eps), p/s))
 *   UOT_DIV_RG : range [alpha, beta], proxdiv = min(beta p/s, max(alpha p/s, 1))
 * beta = +inf (and alpha = 0) are allowed for RG.
 *   UOT_DIV_GROWTH: the growth functional of the WF gradient-flow example
 *                (Sec. 5.3, tumour growth), F(s) = inf_r KL(s|r) - lambda r
 *                over 0 <= r <= p, lambda = 2 tau alpha in [0, 1), p the
 *                density cap (1 in the paper);
 *                proxdiv = min(kappa^{-1/eps}, (p/s)^{1/(1+eps)}),
 *                kappa = 1 - lambda: the example's two branches.  Not
 *                accepted on the barycentre side. */
enum uot_div_kind { UOT_DIV_EQ = 0, UOT_DIV_KL = 1, UOT_DIV_TV = 2, UOT_DIV_RG = 3, UOT_DIV_GROWTH = 4 };

enum uot_dtype { UOT_F64 = 0, UOT_F32 = 1 };

/* Geometry of the cost: C_ij = |x_i - y_j|^2 (squared Euclidean, Sec. 2.3;
 * cost = UOT_COST_SQEUCLID) or the Wasserstein-Fisher-Rao cost of Definition
 * WF, eq. "logcost", C_ij = -log cos^2((pi/2) |x_i - y_j| / cut) for
 * |x_i - y_j| < cut and +inf beyond (cost = UOT_COST_WF; the distance is
 * rescaled so that the cut locus pi/2 sits at `cut`).  K then has exact zeros:
 * a solve puts both clouds in Morton order on the device and, once per call,
 * lists the (64-row wave, 16-column group) pairs whose boxes lie within the
 * cut; its products evaluate only those, in work units of up to 16 groups
 * (results come back in the caller's order, so the storage order of the
 * points does not matter); 1-D grid passes read only the taps within the
 * cut.  The WF cost is
 * not separable over axes: on grids it needs dim = 1.  Ragged batches take
 * the squared Euclidean cost only.
 *   UOT_GEOM_POINTS: point clouds; x is dim x N, y is dim x M, coordinate-major
 *                    (x[k*N + i] = k-th coordinate of x_i); 1 <= dim <= 3.
 *                    The Gibbs product is a dense log-sum-exp that recomputes
 *                    C_ij from the coordinates in registers (Sec. 4.4,
 *                    "Computing the matrix multiplications").
 *   UOT_GEOM_GRID:   X = Y = a regular grid of cell centres (i + 1/2) h[k]
 *                    with n[0] x ... x n[dim-1] cells, row-major (last axis
 *                    fastest); 1 <= dim <= 3.  K is a tensor product of 1-D
 *                    Gaussian kernels applied axis by axis (Sec. 4.4,
 *                    separable kernel), each 1-D pass evaluated as a
 *                    log-sum-exp.  N = M = prod(n). */
enum uot_geom_kind { UOT_GEOM_POINTS = 0, UOT_GEOM_GRID = 1 };
enum uot_cost_kind { UOT_COST_SQEUCLID = 0, UOT_COST_WF = 1 };

typedef struct uot_div {
  int32_t kind;      /* enum uot_div_kind                              */
  int32_t reserved;
  double lambda;     /* KL / TV weight, > 0                            */
  double alpha;      /* RG lower factor, 0 <= alpha <= beta            */
  double beta;       /* RG upper factor, may be +inf                   */
} uot_div;

typedef struct uot_geom {
  int32_t kind;      /* enum uot_geom_kind                             */
  int32_t dim;       /* coordinate dimension (POINTS) / axes (GRID)    */
  int64_t N, M;      /* POINTS: number of points of X and Y            */
  const void *x;     /* POINTS: device, dim x N                        */
  const void *y;     /* POINTS: device, dim x M                        */
  int64_t n[3];      /* GRID: cells per axis                           */
  double h[3];       /* GRID: spacing per axis                         */
  int32_t cost;      /* enum uot_cost_kind (0: squared Euclidean)      */
  int32_t reserved;
  double cut;        /* UOT_COST_WF: cut-locus distance, > 0           */
} uot_geom;

typedef struct uot_problem {
  int32_t dtype;     /* enum uot_dtype of every float array            */
  int32_t reserved;
  uot_geom geom;
  const void *p;     /* device, N: density of mu w.r.t. dx (>= 0)      */
  const void *q;     /* device, M: density of nu w.r.t. dy (>= 0)      */
  const void *dx;    /* device, N: reference weights (> 0)             */
  const void *dy;    /* device, M: reference weights (> 0)             */
  uot_div F1, F2;
} uot_problem;

/* Iteration control.  eps-scaling (Sec. 4.4, "Gradually decreasing eps"):
 * when eps0 > eps and eps_stages > 0 the first eps_stages * iters_per_stage
 * iterations run at eps_k = eps0 * f^k (k = 0..eps_stages-1, f =
 * (eps/eps0)^(1/eps_stages)), then the iteration continues at eps until the
 * residual r <= tol or max_iter iterations in total.  The residual of an
 * iteration is the relative L1 violation of the X marginal against its prox
 * target, measured before the u update:
 *   r = sum_i dx_i |e^{S_i + u_i/eps} - e^{S_i + u'_i/eps}| / sum_i dx_i e^{S_i + u'_i/eps}
 * with S = log K(b dy) and u' the updated potential; it is only tested at the
 * final eps. */
typedef struct uot_params {
  double eps;            /* final regularisation, > 0                        */
  double eps0;           /* annealing start; <= eps or <= 0 disables it      */
  int32_t eps_stages;    /* number of eps divisions (10 in the paper)        */
  int32_t iters_per_stage; /* iterations per annealing stage (100)           */
  double tol;            /* residual tolerance (>= 0)                         */
  int64_t max_iter;      /* iteration cap, >= 1                               */
  int32_t check_every;   /* iterations between host convergence polls (>= 1) */
  int32_t use_graph;     /* 1: replay check_every iterations as a hipGraph   */
  const void *v0;        /* optional device warm start for v (M), or NULL    */
  double *res_hist;      /* optional device array (max_iter) receiving r     */
  double *kernel_ms;     /* optional HOST array [4]: when set, the solve runs
                            without graphs and adds the HIP-event duration of
                            every launch per kernel class: [0] first Gibbs
                            pass / dense LSE, [1] later passes / split merge +
                            epilogue, [2] control, [3] unused              */
  int64_t *kernel_launches; /* optional HOST array [4]: launches per class
                            [0..2]; [3] receives the pair evaluations the
                            matrix-core products performed (they leave out
                            16-column tiles whose terms are all below 2^-50
                            of the row maxima: the on-the-fly form of the
                            kernel truncation of the further tricks of the
                            sparse scaling literature the paper discusses;
                            UOT_TILE_SKIP=0 in the environment turns that
                            off)                                            */
  int32_t grid_kernel;   /* grids: 0 default (2 for FP32, 1 for FP64), 1 direct log-sum-exp
                            passes, 2 tile-factored FP32 MFMA passes (FP32
                            problems, axes with a multiple of 16 cells and
                            h^2 log2(e) / eps <= 0.5 at the final eps; other
                            axes use direct passes), 3 as 2 with FP16 MFMA
                            operands where h^2 log2(e) / eps <= 0.125
                            (results good to ~1e-3 relative; the residual
                            levels off near 2e-5), 4 mixed precision: the
                            passes of 3 until the residual reaches 1e-4, then
                            those of 2 down to tol (FP32 accuracy)         */
  int32_t dense_kernel;  /* point clouds: 0 default (4 for FP32 data with the
                            squared Euclidean cost and N, M >= 2048, else 1),
                            1 direct log-sum-exp
                            product, 2 tile-factored product (FP32, squared
                            Euclidean cost): both clouds are put in Morton
                            order on the device once per solve, tile pairs
                            factor exactly (w_j - c|x_i - y_j|^2 = beta_jI +
                            alpha_iJ + 2c e_i.f_j) and wide tile pairs are
                            summed directly; results come back in the
                            caller's order; 3 and 4 matrix-core products
                            (FP32 data, squared Euclidean cost; Morton-ordered
                            copies as for 2): around a centre per block of
                            rows, w_j - c|x_i - y_j|^2 = R_i + G_j + e_i.B_j,
                            the exponents of 16 x 16 pairs as one MFMA product:
                            3 with FP32 operands (16x16x4 FP32 MFMA), 4 with
                            each operand split into three bf16 parts (24
                            bits; one 16x16x32 BF16 MFMA, FP32 accumulation),
                            which runs beside the exp2 on the vector units.
                            Kernels 2-4 pass the exponent through FP32 terms
                            of size c r^2 (r: half-diagonal of a row block's
                            box), so their potentials err by a few 2^-24 r^2
                            in cost units, the direct product's by a few
                            2^-24 |u|: choose 1 where the potentials are far
                            below r^2 (local transport at tiny eps).
                            Kernels 3 and 4 time their column splits at
                            the first solve of a shape (4 candidates, a few
                            ms; kept in the context; UOT_DENSE_BLOCKS in
                            the environment fixes the block target)       */
  int32_t rebalance_at;  /* ragged batches with KL on both marginals (ABI
                            version 3): at iteration rebalance_at (>= 2,
                            counted from 1; 0 = off) every running problem's
                            v is replaced by v - s with the mass-balance
                            shift of uot_batch_balance (the plan's two
                            marginal masses made equal along the constant
                            direction, the mode the iteration contracts
                            slowest, by theta1 theta2 per iteration).  By
                            Prop. "alternating" only v enters the iterates,
                            so this restarts the iteration from a better v
                            and leaves the fixed point unchanged.  It is
                            taken after that iteration's X half-step as
                            u <- u + theta1 s (u is affine in a constant
                            shift of v under KL); the iteration's residual is
                            that of the unshifted u, and a problem that stops
                            there is not shifted.  Other entry points take 0. */
  int32_t reserved;
} uot_params;

typedef struct uot_result {
  int64_t iters;         /* iterations performed                              */
  double residual;       /* residual of the last iteration                    */
  int32_t status;        /* UOT_OK / UOT_NOT_CONVERGED / UOT_E_NONFINITE      */
  int32_t reserved;
  double elapsed_ms;     /* host wall time of the iteration loop              */
  double du_inf;         /* max_i |u_i - u_i^prev| of the last iteration (the
                            change of the X potentials, ABI version 2): eps
                            times the Thompson distance of the scalings that
                            Thm. "convergenceKL" contracts; +inf when a
                            potential changed to or from -inf              */
} uot_result;

/* Values at the plan R = exp((u + v - C)/eps) (Thm. "duality"):
 *   primal = F1(pi1) + F2(pi2) + <u,pi1>_dx + <v,pi2>_dy - eps m(pi1) + eps m(K)
 *   dual   = -F1*(-u) - F2*(-v) - eps m(pi1) + eps m(K)
 *   gap    = Fenchel-Young form of primal - dual (NaN unless both F are KL/TV)
 *   transport_cost = <C, R>_{dx dy};  mass1 = sum dx pi1, mass2 = sum dy pi2
 * pi1 = R dy, pi2 = R^T dx.  Reductions are accumulated in FP64. */
typedef struct uot_objective_values {
  double primal, dual, gap, transport_cost, mass1, mass2, massK;
} uot_objective_values;

typedef struct uot_ctx uot_ctx;

/* Context bound to one HIP stream (hipStream_t passed as void*, NULL allowed).
 * Holds a small device control block and pinned host mirror, allocated here
 * once.  One context must not be used by two threads at the same time. */
int uot_create(uot_ctx **out, void *stream);
int uot_destroy(uot_ctx *ctx);
const char *uot_status_string(int status);
const char *uot_last_error(void);
int uot_abi_version(void);

/* Workspace bytes needed by uot_solve / uot_half_step / uot_objective for
 * this problem (depends only on sizes, dtype and geometry kind). */
int uot_workspace_size(const uot_problem *pb, size_t *bytes);

/* Scaling iterations (S) from v = v0 (or 0), u = 0, until convergence.
 * u (N) and v (M): device output buffers of the problem dtype, written with
 * the final potentials (u may hold -inf where p = 0).  res: host struct. */
int uot_solve(uot_ctx *ctx, const uot_problem *pb, const uot_params *pr,
              void *u, void *v, void *ws, size_t ws_bytes, uot_result *res);

/* uot_solve without waiting (the asynchronous calls of the boundary): the
 * iteration is enqueued on the context's stream and the call returns.  It
 * enqueues ceil(max_iter / check_every) replays of the check_every-iteration
 * chunk without polling the device: the iterations after the stop cost only
 * their launches (a stopped iteration's kernels return at once), so choose
 * max_iter near the iterations expected (e.g. a fixed count with tol = 0).
 * u and v are written when the stream gets there; uot_sync_result waits for
 * it and fills res (elapsed_ms: device time of the enqueued iterations).
 * One asynchronous solve may be pending per context: every other call on it
 * returns UOT_E_INVALID until uot_sync_result.  The workspace must stay
 * untouched until then.  Not for the mixed-precision grid passes
 * (grid_kernel 4, UOT_E_UNSUPPORTED) or timed solves (kernel_ms). */
int uot_solve_async(uot_ctx *ctx, const uot_problem *pb, const uot_params *pr,
                    void *u, void *v, void *ws, size_t ws_bytes);
/* Wait for the pending asynchronous solve of ctx and fill res; returns what
 * uot_solve would have (UOT_OK, UOT_NOT_CONVERGED, UOT_E_NONFINITE), or
 * UOT_E_INVALID when nothing is pending. */
int uot_sync_result(uot_ctx *ctx, uot_result *res);

/* nb independent problems on one regular grid, solved together: p and q
 * point to nb x size arrays (field k at offset k*size), dx and dy are shared
 * (size), F1/F2/eps/schedule are shared.  u, v: device nb x size outputs.
 * Every launch processes all fields; the residual of an iteration is the
 * largest per-field residual, so the batch stops when every field has
 * r <= tol.  pr->v0, if set, is an nb x size warm start. */
int uot_fields_workspace_size(const uot_problem *pb, int nb, size_t *bytes);
int uot_solve_fields(uot_ctx *ctx, const uot_problem *pb, int nb, const uot_params *pr,
                     void *u, void *v, void *ws, size_t ws_bytes, uot_result *res);

/* Scaling iteration with a function of the total mass (Sec. 4.4, Algorithm
 * 4): min F1(P^X R) + F2(P^Y R) + F3(total mass of R) + eps KL(R|K), with F3
 * = D(. | mass) a divergence on the one-point space (reference measure 1):
 * EQ fixes the mass (with F1 = F2 = RG[0, 1] this is partial transport), KL
 * / TV penalise it, RG bounds it to [alpha mass, beta mass].  In log form,
 * with zeta = log z: both half-steps apply their proxdiv to S + zeta; after
 * the Y half-step, log m = LSE_j(T_j + v_j/eps + log dy_j) (the plan's mass
 * without z) and zeta = log proxdiv_F3(m) (Table proximalexplicit, p = mass).
 * The plan is R_ij = exp(zeta + (u_i + v_j - C_ij)/eps); *log_z (HOST)
 * receives zeta.  Workspace: uot_workspace_size.  grid_kernel 4 is not
 * supported here. */
int uot_solve_mass(uot_ctx *ctx, const uot_problem *pb, const uot_div *F3, double mass,
                   const uot_params *pr, void *u, void *v, double *log_z, void *ws,
                   size_t ws_bytes, uot_result *res);

/* One half-step of (S) from a given state, for checking a single step.
 * side 0 (X half-step): S = log K(e^{v/eps} dy) with v = pot_in (M);
 *   pot_io (N) holds u_old on entry and u' = eps log proxdiv_F1(e^S) on exit;
 *   *residual receives r (definition above).
 * side 1 (Y half-step): T = log K^T(e^{u/eps} dx) with u = pot_in (N);
 *   pot_io (M) receives v' = eps log proxdiv_F2(e^T); *residual is set to 0.
 * lse_out (optional, N or M) receives S or T (natural log). */
int uot_half_step(uot_ctx *ctx, const uot_problem *pb, double eps, int side,
                  const void *pot_in, void *pot_io, void *lse_out,
                  double *residual, void *ws, size_t ws_bytes);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): uot_half_step with
 * the library's own scratch memory in place of the caller's workspace.
 * Arguments, layouts and results are those of uot_half_step; the caller still
 * passes pot_in, pot_io and lse_out.  The call allocates nothing: the scratch
 * is one static array of UOT_SCRATCH_BYTES per GPU, held from the library's
 * load until the process ends, and its address is looked up once per device
 * by uot_create.  A problem whose half-step workspace (at most
 * uot_workspace_size) exceeds UOT_SCRATCH_BYTES returns UOT_E_WORKSPACE before
 * anything is launched.  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents; no call reads a scratch byte it has not
 * written, so nothing needs clearing, but calls that overlap on one GPU
 * (several contexts or streams at once) race: the caller serialises them. */
#define UOT_SCRATCH_BYTES (32u << 20)
int uot_half_step_noalloc(uot_ctx *ctx, const uot_problem *pb, double eps, int side,
                          const void *pot_in, void *pot_io, void *lse_out, double *residual);

/* Objective values, marginals (pi1: N, pi2: M, optional) at (u, v). */
int uot_objective(uot_ctx *ctx, const uot_problem *pb, double eps,
                  const void *u, const void *v, void *pi1, void *pi2,
                  uot_objective_values *out, void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------------
 * Barycentres (Sec. 5.2): n densities p_k on one regular grid (X = Y), with
 * alpha_k-weighted entropy and K_k = exp(-alpha_k c/(alpha_k eps)) = K, F1 =
 * sum_k F1(. | p_k) (any uot_div kind, applied per coupling) and F2(s) =
 * min_h lambda sum_k alpha_k D(s_k | h) with D any uot_div kind (Table
 * estimatebary: (i) equality, (ii) KL, (iii) TV, (iv) RG with finite beta).
 * Per iteration: for every k an X half-step u_k = eps log proxdiv_F1(e^{S_k});
 * then T_k = log K^T(a_k dx) and, per cell, h from the table's row, e.g. (ii)
 *   log h = ((eps+lam)/eps) [LSE_k(log alpha_k + eps/(eps+lam) T_k) - log sum alpha];
 * (iii)/(iv) take the smallest root of their piecewise-linear equation in
 * log h (exact, by its breakpoints); then v_k = eps log proxdiv_{D(.|h)}(e^{T_k}).
 * The residual is the relative L1 X-marginal violation summed over all k.
 * ------------------------------------------------------------------------- */
typedef struct uot_bary_problem {
  int32_t dtype;         /* UOT_F32 or UOT_F64                               */
  int32_t n;             /* number of marginals, >= 1                        */
  uot_geom geom;         /* must be UOT_GEOM_GRID                            */
  const void *p;         /* device, n x size, densities                      */
  const double *alpha;   /* HOST, n weights > 0                              */
  const void *dx;        /* device, size                                     */
  const void *dy;        /* device, size                                     */
  uot_div F1;            /* per-coupling first-marginal penalty              */
  uot_div F2;            /* any kind; RG needs a finite beta                 */
} uot_bary_problem;

int uot_bary_workspace_size(const uot_bary_problem *pb, size_t *bytes);
/* u, v: device n x size outputs; logh: device size output (log h, w.r.t. dy).
 * pr->v0, if set, is an n x size warm start for v. */
int uot_barycenter(uot_ctx *ctx, const uot_bary_problem *pb, const uot_params *pr,
                   void *u, void *v, void *logh, void *ws, size_t ws_bytes,
                   uot_result *res);

/* Barycentric projection (colour transfer, Sec. 5.1): the approximate
 * transport map of a solved problem,
 *   T_i = sum_j R_ij dy_j y_j / sum_j R_ij dy_j,   R_ij = e^{(u_i + v_j - C_ij)/eps},
 * computed from v alone (u cancels) as Gibbs products of the X side: one for
 * the denominator and one per coordinate with y^(k) folded into the input
 * (two per coordinate for point clouds: positive and negative parts).  Grid
 * coordinates are the cell centres (i + 1/2) h[k].  T: device output, dim x N,
 * coordinate-major like x.  Since u cancels, a row with a_i = 0 still gets the
 * projection of its row of K(b dy); T is NaN only where K(b dy) vanishes.  The
 * workspace is that of uot_workspace_size(pb); eps is the eps v belongs to. */
int uot_barycentric_map(uot_ctx *ctx, const uot_problem *pb, double eps, const void *v, void *T,
                        void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------------
 * Gradient flows (Sec. 5.3): n_steps time steps of size tau, each one problem
 * of the generic form on X = Y solved by the scaling iteration (to pr->tol or
 * pr->max_iter iterations per step, pr->eps with optional eps-scaling per
 * step), warm-started with the previous step's v; the next density is read
 * off the optimal coupling on the device.  With p_k the density of step k:
 *   UOT_FLOW_HEAT  : F1 = iota_=(. | p_k), F2 = 2 tau KL(. | q) (Wasserstein
 *                    flow of KL(. | q dx); q = 1 gives the heat flow);
 *                    p_{k+1} = pi2, the density of the coupling's second
 *                    marginal w.r.t. dx.
 *   UOT_FLOW_CROWD : F1 = iota_=(. | p_k), F2 = iota_{<= q} (the projection
 *                    step of the congested crowd model, proxdiv min(q/s, 1);
 *                    its free evolution is another algorithm and is left to
 *                    the caller); p_{k+1} = pi2.
 *   UOT_FLOW_GROWTH: WF flow of -alpha mu(X) + iota_{<= q}: per species
 *                    F1 = KL(. | p_k) and, on the second marginals, the growth
 *                    functional (UOT_DIV_GROWTH, lambda = 2 tau alpha) of
 *                    their sum with cap q; the joint proxdiv gives every
 *                    species the potential -eps log max((Z/q)^{1/(1+eps)},
 *                    kappa^{1/eps}), Z = sum_k s_k, kappa = 1 - 2 tau alpha.
 *                    p_{k+1} = pi2_k / max(kappa, sum_k pi2_k / q), the
 *                    inner minimiser of the growth functional (one species:
 *                    min(pi2 / kappa, q), as the paper states).  The paper
 *                    uses the WF cost (geom.cost = UOT_COST_WF) and q = 1.
 * Several species need a grid; X = Y means a grid, or points with x == y.
 * ------------------------------------------------------------------------- */
enum uot_flow_kind { UOT_FLOW_HEAT = 0, UOT_FLOW_CROWD = 1, UOT_FLOW_GROWTH = 2 };

typedef struct uot_flow_problem {
  int32_t dtype;         /* UOT_F32 or UOT_F64                               */
  int32_t kind;          /* enum uot_flow_kind                               */
  int32_t species;       /* densities moved together, >= 1 (> 1: growth, grid) */
  int32_t reserved;
  uot_geom geom;         /* X = Y (grid, or points with x == y, N == M)      */
  const void *p0;        /* device, species x N: initial densities w.r.t. dx */
  const void *q;         /* device, N: reference (HEAT) / cap (CROWD, GROWTH) */
  const void *dx;        /* device, N: reference weights (dy = dx), > 0      */
  double tau;            /* time step, > 0                                    */
  double alpha;          /* GROWTH: growth rate >= 0, 2 tau alpha < 1         */
} uot_flow_problem;

int uot_flow_workspace_size(const uot_flow_problem *fp, size_t *bytes);
/* dens: device, (n_steps + 1) x species x N output; dens[0] = p0 and
 * dens[k] is the density after step k.  v: device, species x N output, the
 * last step's v (pr->v0, if set, warm-starts the first step).  steps: optional
 * HOST array of n_steps results (iterations, last residual, status, time of
 * each step).  pr->res_hist, if set, holds the last step's residuals.
 * grid_kernel 4 is not available.  Returns UOT_NOT_CONVERGED when a step
 * ended at max_iter (always so with tol = 0, the fixed-iteration steps of the
 * paper's experiments). */
int uot_flow(uot_ctx *ctx, const uot_flow_problem *fp, const uot_params *pr, int32_t n_steps,
             void *dens, void *v, void *ws, size_t ws_bytes, uot_result *steps);

/* ---------------------------------------------------------------------------
 * Ragged batches: B independent point-cloud problems of uneven sizes, solved
 * together (Sec. 4.4 "Multiple couplings": the products run coupling by
 * coupling).  Each half-step is one persistent launch whose blocks pull work
 * items (problem, tile of 256 R rows) from an atomic cursor; every problem has
 * its own residual, stopping test and iteration count, and its items are
 * skipped once it has stopped.  Chunks of check_every iterations are replayed
 * as one hipGraph; the host polls the number of active problems once per
 * chunk.  Tile rows (256 R) and persistent blocks per compute unit are chosen
 * by a built-in autotuner (two timed iterations per candidate from the
 * initial state), cached per batch signature in the context.
 * Layout: the points of problem b are rows offN[b] .. offN[b+1]-1 of the
 * concatenated arrays (x: dim x offN[B], coordinate-major); likewise for Y.
 * eps, the eps schedule, tol and max_iter of uot_params apply to every
 * problem; v0 (optional) is a concatenated warm start (offM[B]).
 * ------------------------------------------------------------------------- */
typedef struct uot_batch_problem {
  int32_t dtype;         /* UOT_F32 or UOT_F64                               */
  int32_t dim;           /* 1..3                                             */
  int64_t B;             /* number of problems                               */
  const int64_t *offN;   /* HOST, B+1 offsets (offN[0] = 0)                  */
  const int64_t *offM;   /* HOST, B+1 offsets (offM[0] = 0)                  */
  const void *x, *y;     /* device, dim x offN[B] / dim x offM[B]            */
  const void *p, *q;     /* device, densities, concatenated                  */
  const void *dx, *dy;   /* device, reference weights, concatenated          */
  uot_div F1, F2;        /* shared by every problem                          */
} uot_batch_problem;

typedef struct uot_batch_result {
  int64_t *iters;        /* HOST [B] or NULL: iterations per problem         */
  double *residual;      /* HOST [B] or NULL: last residual per problem      */
  double *latency_ms;    /* HOST [B] or NULL: device time from the start of
                            the iteration until the problem stopped         */
  int32_t *status;       /* HOST [B] or NULL: 0 converged, 1 max_iter, -3 NaN */
  int64_t iters_max;     /* iterations of the longest problem               */
  int64_t n_converged;
  double elapsed_ms;     /* host wall time of the iteration loop            */
  int32_t tile_rows;     /* autotuned rows per work item                    */
  int32_t blocks_per_cu; /* autotuned persistent blocks per compute unit    */
  double tune_ms;        /* time spent tuning (0 if the cached choice was used) */
  int32_t product;       /* autotuned product: 1 direct log-sum-exp, 4 matrix
                            core (FP32 data; both clouds of every problem in
                            Morton order on the device, potentials returned
                            in the caller's order).  uot_params.dense_kernel
                            restricts the tuner: 0 both, 1 or 4 that one    */
  int32_t reserved;
} uot_batch_result;

int uot_batch_workspace_size(const uot_batch_problem *pb, size_t *bytes);
/* u: device offN[B], v: device offM[B] outputs (problem dtype). */
int uot_solve_batched(uot_ctx *ctx, const uot_batch_problem *pb, const uot_params *pr,
                      void *u, void *v, void *ws, size_t ws_bytes, uot_batch_result *res);

/* Gibbs kernel products of a ragged batch without proxdiv (the product
 * K(b dy) of Sec. 4 written as a log-sum-exp, at one eps): for every problem
 * and every point r of its `rows` cloud (0: X, 1: Y),
 *   out_r = log sum_c exp(w_c - |row_r - col_c|^2 / eps)
 * over the points c of its `cols` cloud (0: X, 1: Y) of the same problem.
 * w: device, concatenated over the problems on the cols side (natural log,
 * -inf allowed); out: device, concatenated on the rows side (natural log;
 * -inf where every term is -inf).  Problem dtype; FP32 batches take the
 * matrix-core product (BF16 x 3 operands, FP32 accumulation), FP64 ones the
 * direct product.  Workspace: uot_batch_workspace_size.  F1, F2, p, q, dx, dy
 * are not read. */
int uot_batch_gibbs(uot_ctx *ctx, const uot_batch_problem *pb, double eps, int rows, int cols,
                    const void *w, void *out, void *ws, size_t ws_bytes);

/* Mass balance of a starting potential v0 of an FP32 batch with KL(lambda1),
 * KL(lambda2) marginal penalties (pb->F1, F2), in place: v0 <- v0 - s_b per
 * problem.  By Prop. "alternating" only v^(0) enters the iterates, so this
 * refines a warm start without touching the iteration or its fixed point.
 * KL row of Table proximalexplicit: the plan's first marginal after an X
 * half-step is p e^{-u/lambda1}, and at the fixed point the second is
 * q e^{-v/lambda2}, both of the plan's mass.  With u1 the X half-step from
 * v0, P = sum p e^{-u1/lambda1} dx and Q = sum q e^{-v0/lambda2} dy;
 * replacing v0 by v0 - s moves u1 by theta1 s (theta1 = lambda1/(lambda1 +
 * eps)), so s = log(P/Q) / (theta1/lambda1 + 1/lambda2) makes the two masses
 * agree.  The constant direction is the one the iteration contracts most
 * slowly (by theta1 theta2 per iteration).  s = 0 for a problem whose P or Q
 * is 0.  v0: device offM[B] FP32; shift: device [B] FP32 or NULL, receives s.
 * x, y, p, q, dx, dy are read.  Workspace: uot_batch_workspace_size.
 * Errors: UOT_E_UNSUPPORTED for other penalties or FP64 data. */
int uot_batch_balance(uot_ctx *ctx, const uot_batch_problem *pb, double eps, void *v0, void *shift,
                      void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------------
 * Warm-start network.  By Prop. "alternating" only v^(0) enters the iterates
 * (the first X half-step overwrites u), so predicting v from the two input
 * measures shortens the iteration while the plain iteration still decides
 * the answer (a wrong prediction costs iterations, never accuracy).
 * Net: 4-layer MLP n_in -> width -> width -> width -> n_out with ReLU hidden
 * layers; every GEMM input (weights, activations) is BF16 (round to nearest
 * even), accumulation FP32 on MFMA; FP32 master weights, Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected).  Loss: mean squared error over the
 * batch x n_out outputs.  Parameter layout of every parameter-sized array:
 * W1 [width x n_in], b1, W2 [width x width], b2, W3, b3, W4 [n_out x width], b4.
 * n_in and width must be multiples of 8, n_out >= 1.  x: batch x n_in FP32 (normalised inside as
 * in_scale * x + in_shift), targets/outputs batch x n_out FP32.
 * ------------------------------------------------------------------------- */
typedef struct uot_net {
  int32_t n_in, width, n_out, reserved;
  float in_scale, in_shift;
  float *master;         /* device, FP32 parameters                         */
  uint16_t *wbf16;       /* device, BF16 copy used by the GEMMs             */
  float *adam_m;         /* device, Adam first moments (training only)      */
  float *adam_v;         /* device, Adam second moments (training only)     */
  int64_t step;          /* Adam step count, advanced by each train step    */
} uot_net;

int uot_net_param_count(const uot_net *net, int64_t *count);
int uot_net_workspace_size(const uot_net *net, int64_t batch, size_t *bytes);
/* refresh wbf16 from master */
int uot_net_sync(uot_ctx *ctx, const uot_net *net);
/* forward pass: y = net(x) */
int uot_warmstart_infer(uot_ctx *ctx, const uot_net *net, const float *x, float *y,
                        int64_t batch, void *ws, size_t ws_bytes);
/* loss and its gradient w.r.t. the parameters (straight through the BF16
 * rounding), without updating anything; grad is device, parameter-sized */
int uot_net_grad(uot_ctx *ctx, const uot_net *net, const float *x, const float *target,
                 int64_t batch, float *grad, double *loss, void *ws, size_t ws_bytes);
/* one Adam step on a batch; *loss (optional) receives the batch loss */
int uot_warmstart_train_step(uot_ctx *ctx, uot_net *net, const float *x, const float *target,
                             int64_t batch, float lr, double *loss, void *ws, size_t ws_bytes);
/* network input of nb grid pairs: average-pool p and q (nb x R x R) to r x r
 * (R a multiple of r) and write x[b] = [log p_r, log q_r] (nb x 2 r^2) */
int uot_warmstart_features(uot_ctx *ctx, const float *p, const float *q, int64_t nb,
                           int R, int r, float *x);
/* Warm start of a ragged FP32 batch of point-cloud problems (the v side):
 * per point y_j of every problem b, UOT_CLOUD_FEATURES = 16 features
 *   c_0 = eps log q_j;
 *   c_1..c_4   = eps G_a(log p + log dx over X),  a = 1/2, 1, 2, 4;
 *   c_5..c_8   = eps G_a(log q + log dy over Y),  a = 1/2, 1, 2, 4;
 *   c_9..c_11  = eps G_a(log dx over X),          a = 1/2, 1, 2;
 *   c_12       = eps G_1(log dy over Y);
 *   c_13, c_14 = eps log sum_i p_i dx_i, eps log sum_j q_j dy_j;
 *   c_15 = eps log(N_b / M_b),
 * with G_a(w) = log sum_c exp(w_c - |y_j - c|^2 / (a eps)) the Gibbs product
 * at eps scaled by a (uot_batch_gibbs): the masses of the two measures and of
 * the two reference measures near y_j at several kernel widths, and the
 * problem's two total masses.  x (device,
 * totM x 16, row per point) receives (c_k - shift_k) * scale_k with shift and
 * scale HOST arrays of 16 (the network's input normalisation).  Workspace:
 * uot_cloud_features_workspace_size. */
#define UOT_CLOUD_FEATURES 16
int uot_cloud_features_workspace_size(const uot_batch_problem *pb, size_t *bytes);
int uot_cloud_features(uot_ctx *ctx, const uot_batch_problem *pb, double eps, const float *shift,
                       const float *scale, float *x, void *ws, size_t ws_bytes);
/* v0_j = zeps log q_j + out_scale y_j + out_shift for n points (device, FP32):
 * y is the network's prediction of the smooth part of v (one output per
 * point); with KL(lambda) on the second marginal zeps = eps lambda /
 * (lambda + eps) makes the first term the exact pointwise part of v at the
 * fixed point (Table proximalexplicit, KL row, in the log domain). */
int uot_cloud_v0(uot_ctx *ctx, const float *q, int64_t n, double zeps, const float *y,
                 double out_scale, double out_shift, float *v0);
/* local (no transport) warm start of a KL(lam) barycentre on a 2-D grid
 * n1 x n2 with cell sides h1, h2: with the Gibbs kernel replaced by its row
 * mass kappa at each cell, every coupling reduces to the one-point problem
 * between p_k and h0 there (the closed form of the KL/KL one-point problem,
 * from the primal of Sec. 3), log r = (lam log p_k + lam log h0 + eps log
 * kappa) / (2 lam + eps), and v0_k = -lam (log r - log h0).  p, v0: device
 * n x n1 n2; h0: device n1 n2 (e.g. uot_bary_estimate); FP32. */
int uot_bary_local_v0(uot_ctx *ctx, const float *p, const float *h0, int n, int n1, int n2,
                      double h1, double h2, double lam, double eps, float *v0);
/* first barycentre estimate for warm starts: Table estimatebary (ii) (KL,
 * lambda = F2->lambda) or (i) (equality) applied pointwise to the input
 * densities p (n x size, FP32) with weights alpha (HOST, n); h: size */
int uot_bary_estimate(uot_ctx *ctx, const float *p, int n, int64_t size, const double *alpha,
                      double eps, const uot_div *F2, float *h);
/* bilinear upsampling of nb cell-centred r x r fields to R x R */
int uot_grid_upsample(uot_ctx *ctx, const float *y, int64_t nb, int r, int R, float *out);
/* the MFMA BF16 GEMM of the network, exposed for checking:
 * C[M x N] = op(A) op(B), op(A)[m][k] = ta ? A[k*lda+m] : A[m*lda+k],
 * op(B)[k][n] = tb ? B[n*ldb+k] : B[k*ldb+n]; A, B BF16 bits, C FP32.
 * A product with few output tiles and a long K splits K over blocks whose
 * partial tiles go to the workspace (uot_gemm_workspace_size bytes, device,
 * 256-byte aligned; 0 when it does not split) and are added in a fixed order;
 * with ws NULL (or too small) it runs unsplit. */
int uot_gemm_workspace_size(int M, int N, int K, size_t *bytes);
int uot_gemm_bf16(uot_ctx *ctx, int ta, int tb, int M, int N, int K, const uint16_t *A,
                  int64_t lda, const uint16_t *B, int64_t ldb, float *C, int64_t ldc,
                  void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------------
 * Tuning table.  The built-in tuners (ragged batches: product, rows per work
 * item and persistent blocks per compute unit, per batch signature; the
 * matrix-core dense products: column-split block target, per shape) time
 * their candidates on the first solve of a signature and keep the choice in
 * the context.  The table moves between contexts and processes as text, one
 * entry per line (signatures are opaque tokens without spaces):
 *   batch <signature> <product: 1 direct, 4 matrix core> <rows per item / 256> <blocks per CU>
 *   dense <shape> <block target>
 * uot_tuning_export writes the table, NUL-terminated, into buf (cap bytes)
 * and the bytes it needs (with the NUL) into *len; a buffer too small (or
 * NULL with cap 0, to ask for the size) gives UOT_E_INVALID with *len set.
 * uot_tuning_import merges a table into the context (an entry replaces one
 * of the same signature; empty lines are skipped).  A line that does not
 * parse, or names a choice the tuner does not make, gives UOT_E_INVALID and
 * nothing is imported.
 * ------------------------------------------------------------------------- */
int uot_tuning_export(uot_ctx *ctx, char *buf, size_t cap, size_t *len);
int uot_tuning_import(uot_ctx *ctx, const char *text);

/* ---------------------------------------------------------------------------
 * Measurement helpers (roofline evidence; not part of the iteration).
 * ------------------------------------------------------------------------- */
/* Average device time in ms of each Gibbs-product kernel of one X half-step
 * (the state v is given), measured with HIP events around `reps` back-to-back
 * launches of that kernel alone on the library stream.
 *   grid   : ms[0] contiguous-axis pass, ms[1..] strided passes (the last
 *            one carries the proxdiv epilogue and residual partials);
 *   points : ms[0] column-split log-sum-exp, ms[1] split merge + epilogue;
 *            with the matrix-core products (grid_kernel 3, 4) ms[2] is no
 *            time but the pair evaluations of one product launch (they
 *            leave out tiles of negligible terms, see kernel_launches).
 * *n_kernels receives the number of entries written (<= 3). */
int uot_time_half_step(uot_ctx *ctx, const uot_problem *pb, double eps, const void *v,
                       int reps, double *ms, int *n_kernels, void *ws, size_t ws_bytes,
                       int grid_kernel);   /* as uot_params.grid_kernel; point
                                              clouds: 2, 3 or 4 time that
                                              dense_kernel, otherwise the
                                              direct one */
/* The same over nb fields on one grid (the layout of uot_solve_fields: pb->p
 * is nb x size, v is nb x size, workspace from uot_fields_workspace_size);
 * every launch processes all nb fields.  nb = 1 is uot_time_half_step. */
int uot_time_fields_half_step(uot_ctx *ctx, const uot_problem *pb, int nb, double eps,
                              const void *v, int reps, double *ms, int *n_kernels, void *ws,
                              size_t ws_bytes, int grid_kernel);

/* Average device time in ms of uot_gemm_bf16 with these arguments over
 * `reps` back-to-back launches on the library stream (HIP events). */
int uot_time_gemm_bf16(uot_ctx *ctx, int ta, int tb, int M, int N, int K, const uint16_t *A,
                       int64_t lda, const uint16_t *B, int64_t ldb, float *C, int64_t ldc,
                       int reps, double *ms, void *ws, size_t ws_bytes);

/* Throughput probe of the current device: v_exp_f32 results per second and
 * v_add_f32 results per second, from 8 independent dependency chains per lane
 * on 64 waves per compute unit.  Allocates a small scratch buffer itself. */
int uot_probe_rates(uot_ctx *ctx, double *exp_per_s, double *add_per_s);

#ifdef __cplusplus
}
#endif
#endif /* UOT_H */
