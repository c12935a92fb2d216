"""Thin Python binding of libuot's C ABI (include/uot.h).

Argument marshalling only: every step of the scaling iteration runs in the
HIP kernels of libuot.so.  PyTorch supplies device memory and the stream.
There is no fallback: if the shared library is missing or fails to load,
every entry point raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libuot.so")

UOT_OK, UOT_NOT_CONVERGED = 0, 1
UOT_E_INVALID, UOT_E_UNSUPPORTED, UOT_E_NONFINITE, UOT_E_HIP, UOT_E_WORKSPACE = -1, -2, -3, -4, -5
UOT_DIV_EQ, UOT_DIV_KL, UOT_DIV_TV, UOT_DIV_RG, UOT_DIV_GROWTH = 0, 1, 2, 3, 4
UOT_F64, UOT_F32 = 0, 1
UOT_GEOM_POINTS, UOT_GEOM_GRID = 0, 1
UOT_COST_SQEUCLID, UOT_COST_WF = 0, 1

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class UotDiv(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("reserved", c_i32), ("lam", c_dbl), ("alpha", c_dbl), ("beta", c_dbl)]


class UotGeom(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("dim", c_i32), ("N", c_i64), ("M", c_i64), ("x", c_vp), ("y", c_vp),
                ("n", c_i64 * 3), ("h", c_dbl * 3), ("cost", c_i32), ("reserved", c_i32), ("cut", c_dbl)]


class UotProblem(ctypes.Structure):
    _fields_ = [("dtype", c_i32), ("reserved", c_i32), ("geom", UotGeom), ("p", c_vp), ("q", c_vp),
                ("dx", c_vp), ("dy", c_vp), ("F1", UotDiv), ("F2", UotDiv)]


class UotParams(ctypes.Structure):
    _fields_ = [("eps", c_dbl), ("eps0", c_dbl), ("eps_stages", c_i32), ("iters_per_stage", c_i32),
                ("tol", c_dbl), ("max_iter", c_i64), ("check_every", c_i32), ("use_graph", c_i32),
                ("v0", c_vp), ("res_hist", c_vp), ("kernel_ms", ctypes.POINTER(c_dbl)),
                ("kernel_launches", ctypes.POINTER(c_i64)), ("grid_kernel", c_i32), ("dense_kernel", c_i32),
                ("rebalance_at", c_i32), ("reserved", c_i32)]


class UotResult(ctypes.Structure):
    _fields_ = [("iters", c_i64), ("residual", c_dbl), ("status", c_i32), ("reserved", c_i32),
                ("elapsed_ms", c_dbl), ("du_inf", c_dbl)]


class UotObjectiveValues(ctypes.Structure):
    _fields_ = [("primal", c_dbl), ("dual", c_dbl), ("gap", c_dbl), ("transport_cost", c_dbl),
                ("mass1", c_dbl), ("mass2", c_dbl), ("massK", c_dbl)]


class UotBaryProblem(ctypes.Structure):
    _fields_ = [("dtype", c_i32), ("n", c_i32), ("geom", UotGeom), ("p", c_vp),
                ("alpha", ctypes.POINTER(c_dbl)), ("dx", c_vp), ("dy", c_vp), ("F1", UotDiv), ("F2", UotDiv)]


class UotBatchProblem(ctypes.Structure):
    _fields_ = [("dtype", c_i32), ("dim", c_i32), ("B", c_i64), ("offN", ctypes.POINTER(c_i64)),
                ("offM", ctypes.POINTER(c_i64)), ("x", c_vp), ("y", c_vp), ("p", c_vp), ("q", c_vp),
                ("dx", c_vp), ("dy", c_vp), ("F1", UotDiv), ("F2", UotDiv)]


class UotBatchResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.POINTER(c_i64)), ("residual", ctypes.POINTER(c_dbl)),
                ("latency_ms", ctypes.POINTER(c_dbl)), ("status", ctypes.POINTER(c_i32)), ("iters_max", c_i64),
                ("n_converged", c_i64), ("elapsed_ms", c_dbl), ("tile_rows", c_i32), ("blocks_per_cu", c_i32),
                ("tune_ms", c_dbl), ("product", c_i32), ("reserved", c_i32)]


class UotFlowProblem(ctypes.Structure):
    _fields_ = [("dtype", c_i32), ("kind", c_i32), ("species", c_i32), ("reserved", c_i32), ("geom", UotGeom),
                ("p0", c_vp), ("q", c_vp), ("dx", c_vp), ("tau", c_dbl), ("alpha", c_dbl)]


class UotNet(ctypes.Structure):
    _fields_ = [("n_in", c_i32), ("width", c_i32), ("n_out", c_i32), ("reserved", c_i32), ("in_scale", ctypes.c_float),
                ("in_shift", ctypes.c_float), ("master", c_vp), ("wbf16", c_vp), ("adam_m", c_vp), ("adam_v", c_vp),
                ("step", c_i64)]


_lib = None


def lib():
    """Load libuot.so (once).  Raises if it is missing: there is no CPU path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libuot.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "uot_abi_version": (c_i32, []),
        "uot_status_string": (ctypes.c_char_p, [c_i32]),
        "uot_last_error": (ctypes.c_char_p, []),
        "uot_create": (c_i32, [P(c_vp), c_vp]),
        "uot_destroy": (c_i32, [c_vp]),
        "uot_workspace_size": (c_i32, [P(UotProblem), P(ctypes.c_size_t)]),
        "uot_solve": (c_i32, [c_vp, P(UotProblem), P(UotParams), c_vp, c_vp, c_vp, ctypes.c_size_t, P(UotResult)]),
        "uot_solve_async": (c_i32, [c_vp, P(UotProblem), P(UotParams), c_vp, c_vp, c_vp, ctypes.c_size_t]),
        "uot_sync_result": (c_i32, [c_vp, P(UotResult)]),
        "uot_half_step": (c_i32, [c_vp, P(UotProblem), c_dbl, c_i32, c_vp, c_vp, c_vp, P(c_dbl), c_vp,
                                  ctypes.c_size_t]),
        "uot_half_step_noalloc": (c_i32, [c_vp, P(UotProblem), c_dbl, c_i32, c_vp, c_vp, c_vp, P(c_dbl)]),
        "uot_objective": (c_i32, [c_vp, P(UotProblem), c_dbl, c_vp, c_vp, c_vp, c_vp, P(UotObjectiveValues), c_vp,
                                  ctypes.c_size_t]),
        "uot_bary_workspace_size": (c_i32, [P(UotBaryProblem), P(ctypes.c_size_t)]),
        "uot_barycenter": (c_i32, [c_vp, P(UotBaryProblem), P(UotParams), c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t,
                                   P(UotResult)]),
        "uot_time_half_step": (c_i32, [c_vp, P(UotProblem), c_dbl, c_vp, c_i32, P(c_dbl), P(c_i32), c_vp,
                                       ctypes.c_size_t, c_i32]),
        "uot_time_fields_half_step": (c_i32, [c_vp, P(UotProblem), c_i32, c_dbl, c_vp, c_i32, P(c_dbl), P(c_i32), c_vp,
                                       ctypes.c_size_t, c_i32]),
        "uot_probe_rates": (c_i32, [c_vp, P(c_dbl), P(c_dbl)]),
        "uot_tuning_export": (c_i32, [c_vp, ctypes.c_char_p, ctypes.c_size_t, P(ctypes.c_size_t)]),
        "uot_tuning_import": (c_i32, [c_vp, ctypes.c_char_p]),
        "uot_fields_workspace_size": (c_i32, [P(UotProblem), c_i32, P(ctypes.c_size_t)]),
        "uot_solve_fields": (c_i32, [c_vp, P(UotProblem), c_i32, P(UotParams), c_vp, c_vp, c_vp, ctypes.c_size_t,
                                     P(UotResult)]),
        "uot_solve_mass": (c_i32, [c_vp, P(UotProblem), P(UotDiv), c_dbl, P(UotParams), c_vp, c_vp, P(c_dbl), c_vp,
                                   ctypes.c_size_t, P(UotResult)]),
        "uot_batch_workspace_size": (c_i32, [P(UotBatchProblem), P(ctypes.c_size_t)]),
        "uot_net_param_count": (c_i32, [P(UotNet), P(c_i64)]),
        "uot_net_workspace_size": (c_i32, [P(UotNet), c_i64, P(ctypes.c_size_t)]),
        "uot_net_sync": (c_i32, [c_vp, P(UotNet)]),
        "uot_warmstart_infer": (c_i32, [c_vp, P(UotNet), c_vp, c_vp, c_i64, c_vp, ctypes.c_size_t]),
        "uot_net_grad": (c_i32, [c_vp, P(UotNet), c_vp, c_vp, c_i64, c_vp, P(c_dbl), c_vp, ctypes.c_size_t]),
        "uot_warmstart_train_step": (c_i32, [c_vp, P(UotNet), c_vp, c_vp, c_i64, ctypes.c_float, P(c_dbl), c_vp,
                                             ctypes.c_size_t]),
        "uot_warmstart_features": (c_i32, [c_vp, c_vp, c_vp, c_i64, c_i32, c_i32, c_vp]),
        "uot_grid_upsample": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_i32, c_vp]),
        "uot_bary_estimate": (c_i32, [c_vp, c_vp, c_i32, c_i64, P(c_dbl), c_dbl, P(UotDiv), c_vp]),
        "uot_gemm_workspace_size": (c_i32, [c_i32, c_i32, c_i32, P(ctypes.c_size_t)]),
        "uot_gemm_bf16": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64,
                                  c_vp, ctypes.c_size_t]),
        "uot_time_gemm_bf16": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64,
                                       c_i32, P(c_dbl), c_vp, ctypes.c_size_t]),
        "uot_bary_local_v0": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_i32, c_i32, c_dbl, c_dbl, c_dbl, c_dbl, c_vp]),
        "uot_batch_gibbs": (c_i32, [c_vp, P(UotBatchProblem), c_dbl, c_i32, c_i32, c_vp, c_vp, c_vp, ctypes.c_size_t]),
        "uot_cloud_features_workspace_size": (c_i32, [P(UotBatchProblem), P(ctypes.c_size_t)]),
        "uot_cloud_features": (c_i32, [c_vp, P(UotBatchProblem), c_dbl, P(ctypes.c_float), P(ctypes.c_float), c_vp,
                                       c_vp, ctypes.c_size_t]),
        "uot_cloud_v0": (c_i32, [c_vp, c_vp, c_i64, c_dbl, c_vp, c_dbl, c_dbl, c_vp]),
        "uot_batch_balance": (c_i32, [c_vp, P(UotBatchProblem), c_dbl, c_vp, c_vp, c_vp, ctypes.c_size_t]),
        "uot_solve_batched": (c_i32, [c_vp, P(UotBatchProblem), P(UotParams), c_vp, c_vp, c_vp, ctypes.c_size_t,
                                      P(UotBatchResult)]),
        "uot_flow_workspace_size": (c_i32, [P(UotFlowProblem), P(ctypes.c_size_t)]),
        "uot_barycentric_map": (c_i32, [c_vp, P(UotProblem), c_dbl, c_vp, c_vp, c_vp, ctypes.c_size_t]),
        "uot_flow": (c_i32, [c_vp, P(UotFlowProblem), P(UotParams), c_i32, c_vp, c_vp, c_vp, ctypes.c_size_t,
                             P(UotResult)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class UotError(RuntimeError):
    def __init__(self, code, where):
        L = lib()
        super().__init__("%s failed: %s (%d): %s" % (where, L.uot_status_string(code).decode(), code,
                                                     L.uot_last_error().decode()))
        self.code = code


def _check(code, where, allow_not_converged=True):
    if code == UOT_OK or (allow_not_converged and code == UOT_NOT_CONVERGED):
        return code
    raise UotError(code, where)


# ---------------------------------------------------------------------------
# divergences (Table proximalexplicit rows)
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Div:
    kind: int
    lam: float = 1.0
    alpha: float = 0.0
    beta: float = math.inf

    def c(self) -> UotDiv:
        return UotDiv(self.kind, 0, float(self.lam), float(self.alpha), float(self.beta))


def EQ():
    return Div(UOT_DIV_EQ)


def KL(lam):
    return Div(UOT_DIV_KL, lam=float(lam))


def TV(lam):
    return Div(UOT_DIV_TV, lam=float(lam))


def RG(alpha, beta):
    return Div(UOT_DIV_RG, alpha=float(alpha), beta=float(beta))


def GROWTH(lam):
    """Growth functional of the WF gradient flow (lam = 2 tau alpha in [0, 1));
    the marginal's density is the cap."""
    return Div(UOT_DIV_GROWTH, lam=float(lam))


# ---------------------------------------------------------------------------
# costs: squared Euclidean, or WF (-log cos^2 with the cut locus at `cut`)
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Cost:
    kind: int = UOT_COST_SQEUCLID
    cut: float = 0.0


SQEUCLID = Cost()


def WF(cut):
    return Cost(UOT_COST_WF, float(cut))


def _grid_geom(shape, h, cost: Cost) -> UotGeom:
    size = int(math.prod(shape))
    n = list(shape) + [1] * (3 - len(shape))
    hh = list(h) + [0.0] * (3 - len(h))
    return UotGeom(UOT_GEOM_GRID, len(shape), size, size, c_vp(), c_vp(), (c_i64 * 3)(*n), (c_dbl * 3)(*hh),
                   cost.kind, 0, cost.cut)


# ---------------------------------------------------------------------------
# context and helpers
# ---------------------------------------------------------------------------
class Context:
    """A libuot context bound to torch's current stream on the current device."""

    def __init__(self, stream: Optional[torch.cuda.Stream] = None):
        L = lib()
        s = stream if stream is not None else torch.cuda.current_stream()
        self._h = c_vp()
        _check(L.uot_create(ctypes.byref(self._h), c_vp(s.cuda_stream)), "uot_create", False)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().uot_destroy(self._h)
            self._h = c_vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context() -> Context:
    key = (torch.cuda.current_device(), torch.cuda.current_stream().cuda_stream)
    if key not in _default_ctx:
        _default_ctx[key] = Context()
    return _default_ctx[key]


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return UOT_F32
    if t.dtype == torch.float64:
        return UOT_F64
    raise TypeError("tensors must be float32 or float64, got %s" % t.dtype)


def _dev(t: torch.Tensor, dtype, n=None, name="tensor") -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return t


def _ptr(t):
    return c_vp(t.data_ptr()) if t is not None else c_vp()


def workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + max(int(nbytes), 256)]


class Problem:
    """A UOT problem: geometry + densities + reference weights + penalties.
    Holds references to every tensor it points to."""

    def __init__(self, geom: UotGeom, dtype, p, q, dx, dy, F1: Div, F2: Div, keep=()):
        self.dtype = dtype
        self.p, self.q, self.dx, self.dy = p, q, dx, dy
        self._keep = keep
        self.N, self.M = p.numel(), q.numel()
        self.c = UotProblem(_dt(p), 0, geom, _ptr(p), _ptr(q), _ptr(dx), _ptr(dy), F1.c(), F2.c())
        self.F1, self.F2 = F1, F2
        self._ws = None

    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            n = ctypes.c_size_t()
            _check(lib().uot_workspace_size(ctypes.byref(self.c), ctypes.byref(n)), "uot_workspace_size", False)
            self._ws = workspace(n.value, self.p.device)
        return self._ws


def _coord_major(x, n, layout, name):
    """(d, n) view of point coordinates given as (n, d) ("nd") or (d, n)
    ("dn"); with layout None the shape decides, and a square shape above
    1 x 1, which fits both readings, is an error."""
    if x.dim() == 1:
        return x[None, :] if layout == "dn" else x[:, None].t()
    if layout is None:
        if x.shape[0] == x.shape[1] and x.shape[0] > 1:
            raise ValueError("%s is %d x %d: pass layout='nd' (points in rows) or 'dn' (coordinate-major)"
                             % (name, x.shape[0], x.shape[1]))
        layout = "nd" if x.shape[0] == n else "dn"
    if layout not in ("nd", "dn"):
        raise ValueError("layout must be 'nd' or 'dn'")
    xs = x.t() if layout == "nd" else x
    if xs.shape[1] != n:
        raise ValueError("%s has shape %s, which does not hold %d points in layout %r" % (name, tuple(x.shape), n,
                                                                                         layout))
    return xs


def points_problem(x, y, p, q, dx, dy, F1: Div, F2: Div, cost: Cost = SQEUCLID, layout: Optional[str] = None) -> Problem:
    """Point clouds x (N points) and y (M points), given as (N, d) tensors
    (layout "nd", points in rows) or coordinate-major (d, N) ("dn"); stored
    coordinate-major for the kernels.  Without a layout the shape decides,
    and a square shape (N = d) raises ValueError."""
    dtype = p.dtype
    N, M = p.numel(), q.numel()
    x = _coord_major(x, N, layout, "x")
    y = _coord_major(y, M, layout, "y")
    xs = _dev(x.contiguous(), dtype, name="x")
    ys = _dev(y.contiguous(), dtype, name="y")
    d = xs.shape[0]
    if ys.shape[0] != d:
        raise ValueError("x and y must have the same dimension")
    for t, n, nm in ((p, N, "p"), (q, M, "q"), (dx, N, "dx"), (dy, M, "dy")):
        _dev(t, dtype, n, nm)
    g = UotGeom(UOT_GEOM_POINTS, d, N, M, _ptr(xs), _ptr(ys), (c_i64 * 3)(0, 0, 0), (c_dbl * 3)(0, 0, 0),
                cost.kind, 0, cost.cut)
    return Problem(g, dtype, p, q, dx, dy, F1, F2, keep=(xs, ys))


def grid_problem(shape: Sequence[int], h: Sequence[float], p, q, dx, dy, F1: Div, F2: Div,
                 cost: Cost = SQEUCLID) -> Problem:
    dtype = p.dtype
    size = int(math.prod(shape))
    for t, nm in ((p, "p"), (q, "q"), (dx, "dx"), (dy, "dy")):
        _dev(t, dtype, size, nm)
    return Problem(_grid_geom(shape, h, cost), dtype, p, q, dx, dy, F1, F2)


GRID_AUTO, GRID_DIRECT, GRID_MFMA, GRID_MFMA16, GRID_MIXED = 0, 1, 2, 3, 4
DENSE_AUTO, DENSE_DIRECT, DENSE_TF, DENSE_MF, DENSE_MF3 = 0, 1, 2, 3, 4


def params(eps, tol=1e-6, max_iter=10000, eps0=None, eps_stages=10, iters_per_stage=100, check_every=50,
           use_graph=True, v0=None, res_hist=None, kernel_ms=None, kernel_launches=None,
           grid_kernel=GRID_AUTO, dense_kernel=0, rebalance_at=0) -> UotParams:
    return UotParams(float(eps), float(eps0 or 0.0), int(eps_stages if eps0 else 0), int(iters_per_stage),
                     float(tol), int(max_iter), int(check_every), int(bool(use_graph)), _ptr(v0), _ptr(res_hist),
                     kernel_ms, kernel_launches, int(grid_kernel), int(dense_kernel), int(rebalance_at), 0)


def solve(prob: Problem, eps, ctx: Optional[Context] = None, v0=None, record=False, time_kernels=False, **kw):
    """Scaling iterations until residual <= tol.  Returns (u, v, info).
    time_kernels: run without graphs and report per-class kernel times
    (HIP events around every launch) in info["kernel_ms"] / ["kernel_launches"]."""
    ctx = ctx or default_context()
    dev = prob.p.device
    u = torch.empty(prob.N, dtype=prob.dtype, device=dev)
    v = torch.empty(prob.M, dtype=prob.dtype, device=dev)
    max_iter = kw.get("max_iter", 10000)
    hist = torch.full((max_iter,), float("nan"), dtype=torch.float64, device=dev) if record else None
    if v0 is not None:
        _dev(v0, prob.dtype, prob.M, "v0")
    kms = (c_dbl * 4)() if time_kernels else None
    kcnt = (c_i64 * 4)() if time_kernels else None
    pr = params(eps, v0=v0, res_hist=hist, kernel_ms=kms, kernel_launches=kcnt, **kw)
    res = UotResult()
    ws = prob.workspace()
    code = lib().uot_solve(ctx.handle, ctypes.byref(prob.c), ctypes.byref(pr), _ptr(u), _ptr(v), _ptr(ws),
                           ws.numel(), ctypes.byref(res))
    _check(code, "uot_solve")
    info = dict(iters=res.iters, residual=res.residual, du_inf=res.du_inf, status=res.status,
                elapsed_ms=res.elapsed_ms, converged=(code == UOT_OK))
    if record:
        info["res_hist"] = hist[:res.iters].cpu()
    if time_kernels:
        info["kernel_ms"] = [kms[k] for k in range(4)]
        info["kernel_launches"] = [kcnt[k] for k in range(4)]
    return u, v, info


class PendingSolve:
    """An asynchronous solve (uot_solve_async): u and v fill in on the
    context's stream; result() waits (uot_sync_result) and returns the info
    dict of solve.  Holds the workspace and v0 until then."""

    def __init__(self, ctx, u, v, keep):
        self.ctx, self.u, self.v, self._keep = ctx, u, v, keep
        self._info = None

    def result(self):
        if self._info is None:
            res = UotResult()
            code = lib().uot_sync_result(self.ctx.handle, ctypes.byref(res))
            self._keep = None
            _check(code, "uot_sync_result")
            self._info = dict(iters=res.iters, residual=res.residual, du_inf=res.du_inf, status=res.status,
                              elapsed_ms=res.elapsed_ms, converged=(code == UOT_OK))
        return self._info


def solve_async(prob: Problem, eps, ctx: Optional[Context] = None, v0=None, **kw) -> PendingSolve:
    """solve without waiting: enqueues ceil(max_iter / check_every) chunks of
    iterations (no-ops after the stop) and returns a PendingSolve."""
    ctx = ctx or default_context()
    dev = prob.p.device
    u = torch.empty(prob.N, dtype=prob.dtype, device=dev)
    v = torch.empty(prob.M, dtype=prob.dtype, device=dev)
    if v0 is not None:
        _dev(v0, prob.dtype, prob.M, "v0")
    pr = params(eps, v0=v0, **kw)
    ws = prob.workspace()
    _check(lib().uot_solve_async(ctx.handle, ctypes.byref(prob.c), ctypes.byref(pr), _ptr(u), _ptr(v), _ptr(ws),
                                 ws.numel()), "uot_solve_async", False)
    return PendingSolve(ctx, u, v, (ws, v0))


def half_step(prob: Problem, eps, side, pot_in, pot_old, ctx: Optional[Context] = None):
    """One half-step from a given state.  side 0: pot_in = v, pot_old = u;
    returns (u_new, S, r).  side 1: pot_in = u; returns (v_new, T, 0.0)."""
    ctx = ctx or default_context()
    n_out = prob.N if side == 0 else prob.M
    n_in = prob.M if side == 0 else prob.N
    _dev(pot_in, prob.dtype, n_in, "pot_in")
    out = _dev(pot_old, prob.dtype, n_out, "pot_old").clone()
    lse = torch.empty(n_out, dtype=prob.dtype, device=out.device)
    r = c_dbl()
    ws = prob.workspace()
    _check(lib().uot_half_step(ctx.handle, ctypes.byref(prob.c), float(eps), int(side), _ptr(pot_in), _ptr(out),
                               _ptr(lse), ctypes.byref(r), _ptr(ws), ws.numel()), "uot_half_step", False)
    return out, lse, r.value


def half_step_noalloc(prob: Problem, eps, side, pot_in, pot_old, ctx: Optional[Context] = None):
    """half_step on the library's static scratch memory (uot_half_step_noalloc):
    no workspace is allocated.  Same arguments and results as half_step."""
    ctx = ctx or default_context()
    n_out = prob.N if side == 0 else prob.M
    n_in = prob.M if side == 0 else prob.N
    _dev(pot_in, prob.dtype, n_in, "pot_in")
    out = _dev(pot_old, prob.dtype, n_out, "pot_old").clone()
    lse = torch.empty(n_out, dtype=prob.dtype, device=out.device)
    r = c_dbl()
    _check(lib().uot_half_step_noalloc(ctx.handle, ctypes.byref(prob.c), float(eps), int(side), _ptr(pot_in),
                                       _ptr(out), _ptr(lse), ctypes.byref(r)), "uot_half_step_noalloc", False)
    return out, lse, r.value


def objective(prob: Problem, eps, u, v, ctx: Optional[Context] = None, marginals=False):
    """Primal / dual / gap / <C,R> / masses at (u, v), FP64 reductions."""
    ctx = ctx or default_context()
    _dev(u, prob.dtype, prob.N, "u")
    _dev(v, prob.dtype, prob.M, "v")
    pi1 = torch.empty(prob.N, dtype=prob.dtype, device=u.device) if marginals else None
    pi2 = torch.empty(prob.M, dtype=prob.dtype, device=u.device) if marginals else None
    o = UotObjectiveValues()
    ws = prob.workspace()
    _check(lib().uot_objective(ctx.handle, ctypes.byref(prob.c), float(eps), _ptr(u), _ptr(v), _ptr(pi1), _ptr(pi2),
                               ctypes.byref(o), _ptr(ws), ws.numel()), "uot_objective", False)
    d = {k: getattr(o, k) for k, _ in UotObjectiveValues._fields_}
    if marginals:
        d["pi1"], d["pi2"] = pi1, pi2
    return d


def barycentric_map(prob: Problem, eps, v, ctx: Optional[Context] = None):
    """Barycentric projection T (dim x N) of the plan of (u, v) (u cancels):
    T_i = sum_j R_ij dy_j y_j / sum_j R_ij dy_j; NaN only where K(b dy) vanishes."""
    ctx = ctx or default_context()
    _dev(v, prob.dtype, prob.M, "v")
    T = torch.empty(prob.c.geom.dim, prob.N, dtype=prob.dtype, device=v.device)
    ws = prob.workspace()
    _check(lib().uot_barycentric_map(ctx.handle, ctypes.byref(prob.c), float(eps), _ptr(v), _ptr(T), _ptr(ws),
                                     ws.numel()), "uot_barycentric_map", False)
    return T


def solve_mass(prob: Problem, F3: Div, mass, eps, ctx: Optional[Context] = None, record=False, **kw):
    """Algorithm 4: the scaling iteration with F3 on the total mass of the plan
    (reference value `mass`).  Returns (u, v, log_z, info)."""
    ctx = ctx or default_context()
    dev = prob.p.device
    u = torch.empty(prob.N, dtype=prob.dtype, device=dev)
    v = torch.empty(prob.M, dtype=prob.dtype, device=dev)
    ws = prob.workspace()
    max_iter = kw.get("max_iter", 10000)
    hist = torch.full((max_iter,), float("nan"), dtype=torch.float64, device=dev) if record else None
    pr = params(eps, res_hist=hist, **kw)
    res = UotResult()
    lz = c_dbl()
    f3 = F3.c()
    code = lib().uot_solve_mass(ctx.handle, ctypes.byref(prob.c), ctypes.byref(f3), float(mass), ctypes.byref(pr),
                                _ptr(u), _ptr(v), ctypes.byref(lz), _ptr(ws), ws.numel(), ctypes.byref(res))
    _check(code, "uot_solve_mass")
    info = dict(iters=res.iters, residual=res.residual, du_inf=res.du_inf, status=res.status,
                elapsed_ms=res.elapsed_ms, converged=(code == UOT_OK))
    if record:
        info["res_hist"] = hist[:res.iters].cpu()
    return u, v, lz.value, info


def barycenter(shape, h, p, alpha, dx, dy, F1: Div, F2: Div, eps, ctx: Optional[Context] = None, v0=None,
               record=False, cost: Cost = SQEUCLID, **kw):
    """Unbalanced barycentre of n densities p (n x size) on a grid.
    Returns (u, v, logh, info)."""
    ctx = ctx or default_context()
    dtype = p.dtype
    nm = p.shape[0]
    size = int(math.prod(shape))
    _dev(p, dtype, nm * size, "p")
    _dev(dx, dtype, size, "dx")
    _dev(dy, dtype, size, "dy")
    g = _grid_geom(shape, h, cost)
    al = (c_dbl * nm)(*[float(a) for a in alpha])
    bp = UotBaryProblem(_dt(p), nm, g, _ptr(p), ctypes.cast(al, ctypes.POINTER(c_dbl)), _ptr(dx), _ptr(dy),
                        F1.c(), F2.c())
    nb = ctypes.c_size_t()
    _check(lib().uot_bary_workspace_size(ctypes.byref(bp), ctypes.byref(nb)), "uot_bary_workspace_size", False)
    ws = workspace(nb.value, p.device)
    u = torch.empty(nm, size, dtype=dtype, device=p.device)
    v = torch.empty(nm, size, dtype=dtype, device=p.device)
    logh = torch.empty(size, dtype=dtype, device=p.device)
    max_iter = kw.get("max_iter", 10000)
    hist = torch.full((max_iter,), float("nan"), dtype=torch.float64, device=p.device) if record else None
    pr = params(eps, v0=v0, res_hist=hist, **kw)
    res = UotResult()
    code = lib().uot_barycenter(ctx.handle, ctypes.byref(bp), ctypes.byref(pr), _ptr(u), _ptr(v), _ptr(logh),
                                _ptr(ws), ws.numel(), ctypes.byref(res))
    _check(code, "uot_barycenter")
    info = dict(iters=res.iters, residual=res.residual, du_inf=res.du_inf, status=res.status,
                elapsed_ms=res.elapsed_ms, converged=(code == UOT_OK))
    if record:
        info["res_hist"] = hist[:res.iters].cpu()
    return u, v, logh, info


def time_half_step(prob: Problem, eps, v, reps=50, ctx: Optional[Context] = None, grid_kernel=0):
    """Average ms of each Gibbs-product kernel of one X half-step (HIP events)."""
    ctx = ctx or default_context()
    _dev(v, prob.dtype, prob.M, "v")
    ms = (c_dbl * 4)()
    nk = c_i32()
    ws = prob.workspace()
    _check(lib().uot_time_half_step(ctx.handle, ctypes.byref(prob.c), float(eps), _ptr(v), int(reps), ms,
                                    ctypes.byref(nk), _ptr(ws), ws.numel(), int(grid_kernel)),
           "uot_time_half_step", False)
    return [ms[k] for k in range(nk.value)]


def time_fields_half_step(shape, h, p, dx, dy, F1: Div, eps, v, reps=20, ctx: Optional[Context] = None,
                          grid_kernel=0, cost: Cost = SQEUCLID):
    """time_half_step over nb fields on one grid (p, v: nb x size); every
    timed launch processes all fields."""
    ctx = ctx or default_context()
    nb = p.shape[0]
    size = int(math.prod(shape))
    dtype = p.dtype
    _dev(p, dtype, nb * size, "p")
    _dev(v, dtype, nb * size, "v")
    _dev(dx, dtype, size, "dx")
    _dev(dy, dtype, size, "dy")
    g = _grid_geom(shape, h, cost)
    pb = UotProblem(_dt(p), 0, g, _ptr(p), _ptr(p), _ptr(dx), _ptr(dy), F1.c(), F1.c())
    nbytes = ctypes.c_size_t()
    _check(lib().uot_fields_workspace_size(ctypes.byref(pb), nb, ctypes.byref(nbytes)), "uot_fields_workspace_size",
           False)
    ws = workspace(nbytes.value, p.device)
    ms = (c_dbl * 4)()
    nk = c_i32()
    _check(lib().uot_time_fields_half_step(ctx.handle, ctypes.byref(pb), nb, float(eps), _ptr(v), int(reps), ms,
                                           ctypes.byref(nk), _ptr(ws), ws.numel(), int(grid_kernel)),
           "uot_time_fields_half_step", False)
    return [ms[k] for k in range(nk.value)]


def probe_rates(ctx: Optional[Context] = None):
    """(exp2 results/s, fp32 add results/s) measured on the current device."""
    ctx = ctx or default_context()
    e, a = c_dbl(), c_dbl()
    _check(lib().uot_probe_rates(ctx.handle, ctypes.byref(e), ctypes.byref(a)), "uot_probe_rates", False)
    return e.value, a.value


def export_tuning(ctx: Optional[Context] = None) -> str:
    """The context's tuning table (uot_tuning_export) as text."""
    ctx = ctx or default_context()
    n = ctypes.c_size_t()
    lib().uot_tuning_export(ctx.handle, None, 0, ctypes.byref(n))   # asks for the size
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().uot_tuning_export(ctx.handle, buf, n.value, ctypes.byref(n)), "uot_tuning_export", False)
    return buf.value.decode()


def import_tuning(text: str, ctx: Optional[Context] = None) -> None:
    """Merge a tuning table (uot_tuning_import) into the context."""
    ctx = ctx or default_context()
    _check(lib().uot_tuning_import(ctx.handle, text.encode()), "uot_tuning_import", False)


class BatchProblem:
    """B independent point-cloud problems of uneven sizes, concatenated.

    xs, ys: lists of (N_b, d) / (M_b, d) tensors (or one concatenated tensor
    each with sizes Ns / Ms); p, q, dx, dy likewise concatenated."""

    def __init__(self, Ns, Ms, x, y, p, q, dx, dy, F1: Div, F2: Div, layout: Optional[str] = None):
        import numpy as np
        dtype = p.dtype
        self.B = len(Ns)
        self.offN = np.zeros(self.B + 1, dtype=np.int64)
        self.offM = np.zeros(self.B + 1, dtype=np.int64)
        self.offN[1:] = np.cumsum(np.asarray(Ns, dtype=np.int64))
        self.offM[1:] = np.cumsum(np.asarray(Ms, dtype=np.int64))
        totN, totM = int(self.offN[-1]), int(self.offM[-1])
        x = _coord_major(x, totN, layout, "x")
        y = _coord_major(y, totM, layout, "y")
        self.x = _dev(x.contiguous(), dtype, name="x")
        self.y = _dev(y.contiguous(), dtype, name="y")
        d = self.x.shape[0]
        for t, n, nm in ((p, totN, "p"), (q, totM, "q"), (dx, totN, "dx"), (dy, totM, "dy")):
            _dev(t, dtype, n, nm)
        self.p, self.q, self.dx, self.dy = p, q, dx, dy
        self.dtype = dtype
        self.totN, self.totM = totN, totM
        self._offN_c = self.offN.ctypes.data_as(ctypes.POINTER(c_i64))
        self._offM_c = self.offM.ctypes.data_as(ctypes.POINTER(c_i64))
        self.c = UotBatchProblem(_dt(p), d, self.B, self._offN_c, self._offM_c, _ptr(self.x), _ptr(self.y), _ptr(p),
                                 _ptr(q), _ptr(dx), _ptr(dy), F1.c(), F2.c())
        self._ws = None

    def workspace(self):
        if self._ws is None:
            n = ctypes.c_size_t()
            _check(lib().uot_batch_workspace_size(ctypes.byref(self.c), ctypes.byref(n)), "uot_batch_workspace_size",
                   False)
            self._ws = workspace(n.value, self.p.device)
        return self._ws


def solve_batched(bp: BatchProblem, eps, ctx: Optional[Context] = None, v0=None, time_kernels=False, **kw):
    """Solve every problem of the batch.  Returns (u, v, info) with u, v
    concatenated and per-problem arrays in info."""
    import numpy as np
    ctx = ctx or default_context()
    dev = bp.p.device
    u = torch.empty(bp.totN, dtype=bp.dtype, device=dev)
    v = torch.empty(bp.totM, dtype=bp.dtype, device=dev)
    if v0 is not None:
        _dev(v0, bp.dtype, bp.totM, "v0")
    kms = (c_dbl * 4)() if time_kernels else None
    kcnt = (c_i64 * 4)() if time_kernels else None
    pr = params(eps, v0=v0, kernel_ms=kms, kernel_launches=kcnt, **kw)
    it = np.zeros(bp.B, dtype=np.int64)
    rs = np.zeros(bp.B, dtype=np.float64)
    lat = np.zeros(bp.B, dtype=np.float64)
    st = np.zeros(bp.B, dtype=np.int32)
    res = UotBatchResult(it.ctypes.data_as(ctypes.POINTER(c_i64)), rs.ctypes.data_as(ctypes.POINTER(c_dbl)),
                         lat.ctypes.data_as(ctypes.POINTER(c_dbl)), st.ctypes.data_as(ctypes.POINTER(c_i32)))
    ws = bp.workspace()
    code = lib().uot_solve_batched(ctx.handle, ctypes.byref(bp.c), ctypes.byref(pr), _ptr(u), _ptr(v), _ptr(ws),
                                   ws.numel(), ctypes.byref(res))
    _check(code, "uot_solve_batched")
    info = dict(iters=it, residual=rs, latency_ms=lat, status=st, iters_max=res.iters_max,
                n_converged=res.n_converged, elapsed_ms=res.elapsed_ms, tile_rows=res.tile_rows,
                blocks_per_cu=res.blocks_per_cu, tune_ms=res.tune_ms, product=res.product,
                converged=(code == UOT_OK))
    if time_kernels:
        info["kernel_ms"] = [kms[k] for k in range(4)]
        info["kernel_launches"] = [kcnt[k] for k in range(4)]
    return u, v, info


def batch_gibbs(bp: BatchProblem, eps, rows, cols, w, ctx: Optional[Context] = None):
    """out_r = log sum_c exp(w_c - |row_r - col_c|^2 / eps) per problem
    (uot_batch_gibbs); rows, cols: 0 for X, 1 for Y."""
    ctx = ctx or default_context()
    _dev(w, bp.dtype, bp.totM if cols else bp.totN, "w")
    out = torch.empty(bp.totM if rows else bp.totN, dtype=bp.dtype, device=w.device)
    ws = bp.workspace()
    _check(lib().uot_batch_gibbs(ctx.handle, ctypes.byref(bp.c), float(eps), int(rows), int(cols), _ptr(w), _ptr(out),
                                 _ptr(ws), ws.numel()), "uot_batch_gibbs", False)
    return out


def batch_balance(bp: BatchProblem, eps, v0, ctx: Optional[Context] = None, with_shift=False):
    """Mass balance of a starting potential v0 (device, totM, FP32; KL on both
    marginals), in place (uot_batch_balance): v0 <- v0 - s per problem.
    Returns v0, or (v0, s) with s the per-problem shifts when with_shift."""
    ctx = ctx or default_context()
    _dev(v0, torch.float32, bp.totM, "v0")
    shift = torch.empty(bp.B, dtype=torch.float32, device=v0.device) if with_shift else None
    ws = bp.workspace()
    _check(lib().uot_batch_balance(ctx.handle, ctypes.byref(bp.c), float(eps), _ptr(v0),
                                   _ptr(shift) if shift is not None else None, _ptr(ws), ws.numel()),
           "uot_batch_balance", False)
    return (v0, shift) if with_shift else v0


CLOUD_FEATURES = 16


def cloud_features(bp: BatchProblem, eps, shift, scale, ctx: Optional[Context] = None):
    """Warm-start features of every point of the Y clouds (uot_cloud_features):
    (totM x 16) FP32, normalised as (c - shift) * scale."""
    import numpy as np
    ctx = ctx or default_context()
    sh = np.ascontiguousarray(np.asarray(shift, dtype=np.float32).reshape(CLOUD_FEATURES))
    sc = np.ascontiguousarray(np.asarray(scale, dtype=np.float32).reshape(CLOUD_FEATURES))
    n = ctypes.c_size_t()
    _check(lib().uot_cloud_features_workspace_size(ctypes.byref(bp.c), ctypes.byref(n)),
           "uot_cloud_features_workspace_size", False)
    ws = workspace(n.value, bp.p.device)
    x = torch.empty(bp.totM, CLOUD_FEATURES, dtype=torch.float32, device=bp.p.device)
    fp = ctypes.POINTER(ctypes.c_float)
    _check(lib().uot_cloud_features(ctx.handle, ctypes.byref(bp.c), float(eps), sh.ctypes.data_as(fp),
                                    sc.ctypes.data_as(fp), _ptr(x), _ptr(ws), ws.numel()), "uot_cloud_features", False)
    return x


def cloud_v0(q, zeps, y, out_scale, out_shift, ctx: Optional[Context] = None):
    """v0 = zeps log q + out_scale y + out_shift (uot_cloud_v0), FP32."""
    ctx = ctx or default_context()
    n = q.numel()
    _dev(q, torch.float32, n, "q")
    _dev(y, torch.float32, n, "y")
    v0 = torch.empty(n, dtype=torch.float32, device=q.device)
    _check(lib().uot_cloud_v0(ctx.handle, _ptr(q), n, float(zeps), _ptr(y), float(out_scale), float(out_shift),
                              _ptr(v0)), "uot_cloud_v0", False)
    return v0


def solve_fields(shape, h, p, q, dx, dy, F1: Div, F2: Div, eps, ctx: Optional[Context] = None, v0=None,
                 record=False, cost: Cost = SQEUCLID, **kw):
    """nb independent UOT problems on one grid (p, q: nb x size).  Returns
    (u, v, info) with u, v of shape (nb, size)."""
    ctx = ctx or default_context()
    nb = p.shape[0]
    size = int(math.prod(shape))
    dtype = p.dtype
    _dev(p, dtype, nb * size, "p")
    _dev(q, dtype, nb * size, "q")
    _dev(dx, dtype, size, "dx")
    _dev(dy, dtype, size, "dy")
    g = _grid_geom(shape, h, cost)
    pb = UotProblem(_dt(p), 0, g, _ptr(p), _ptr(q), _ptr(dx), _ptr(dy), F1.c(), F2.c())
    nbytes = ctypes.c_size_t()
    _check(lib().uot_fields_workspace_size(ctypes.byref(pb), nb, ctypes.byref(nbytes)), "uot_fields_workspace_size",
           False)
    ws = workspace(nbytes.value, p.device)
    u = torch.empty(nb, size, dtype=dtype, device=p.device)
    v = torch.empty(nb, size, dtype=dtype, device=p.device)
    if v0 is not None:
        _dev(v0, dtype, nb * size, "v0")
    max_iter = kw.get("max_iter", 10000)
    hist = torch.full((max_iter,), float("nan"), dtype=torch.float64, device=p.device) if record else None
    pr = params(eps, v0=v0, res_hist=hist, **kw)
    res = UotResult()
    code = lib().uot_solve_fields(ctx.handle, ctypes.byref(pb), nb, ctypes.byref(pr), _ptr(u), _ptr(v), _ptr(ws),
                                  ws.numel(), ctypes.byref(res))
    _check(code, "uot_solve_fields")
    info = dict(iters=res.iters, residual=res.residual, du_inf=res.du_inf, status=res.status,
                elapsed_ms=res.elapsed_ms, converged=(code == UOT_OK))
    if record:
        info["res_hist"] = hist[:res.iters].cpu()
    return u, v, info


# ---------------------------------------------------------------------------
# warm-start network
# ---------------------------------------------------------------------------
def bf16_bits(t: torch.Tensor) -> torch.Tensor:
    """BF16 bit patterns (int16 view) of a float tensor, round to nearest even."""
    return t.to(torch.bfloat16).view(torch.int16)


def _gemm_workspace(M, N, K, device):
    n = ctypes.c_size_t()
    _check(lib().uot_gemm_workspace_size(M, N, K, ctypes.byref(n)), "uot_gemm_workspace_size", False)
    return workspace(n.value, device) if n.value else None


def gemm_bf16(A_bits, B_bits, M, N, K, ta=False, tb=False, lda=None, ldb=None, ctx: Optional[Context] = None,
              split=True):
    """C = op(A) op(B) on BF16 bits (uot_gemm_bf16); split=False runs it
    without K splits (no workspace)."""
    ctx = ctx or default_context()
    C = torch.empty(M, N, dtype=torch.float32, device=A_bits.device)
    lda = lda if lda is not None else (M if ta else K)
    ldb = ldb if ldb is not None else (K if tb else N)
    ws = _gemm_workspace(M, N, K, A_bits.device) if split else None
    _check(lib().uot_gemm_bf16(ctx.handle, int(ta), int(tb), M, N, K, _ptr(A_bits), lda, _ptr(B_bits), ldb, _ptr(C),
                               N, _ptr(ws), 0 if ws is None else ws.numel()), "uot_gemm_bf16", False)
    return C


def time_gemm_bf16(A_bits, B_bits, M, N, K, ta=False, tb=False, reps=20, ctx: Optional[Context] = None):
    """Average ms of gemm_bf16 with these operands (HIP events, library stream)."""
    ctx = ctx or default_context()
    C = torch.empty(M, N, dtype=torch.float32, device=A_bits.device)
    lda = M if ta else K
    ldb = K if tb else N
    ms = c_dbl()
    ws = _gemm_workspace(M, N, K, A_bits.device)
    _check(lib().uot_time_gemm_bf16(ctx.handle, int(ta), int(tb), M, N, K, _ptr(A_bits), lda, _ptr(B_bits), ldb,
                                    _ptr(C), N, int(reps), ctypes.byref(ms), _ptr(ws), 0 if ws is None else ws.numel()),
           "uot_time_gemm_bf16", False)
    return ms.value


class WarmStartNet:
    """4-layer MLP of the C ABI: parameters, BF16 copy and Adam state on the
    device; every computation runs in libuot's kernels."""

    def __init__(self, n_in, width, n_out, device, seed=0, in_scale=1.0, in_shift=0.0, params=None):
        import numpy as np
        self.c = UotNet(n_in, width, n_out, 0, in_scale, in_shift)
        cnt = c_i64()
        _check(lib().uot_net_param_count(ctypes.byref(self.c), ctypes.byref(cnt)), "uot_net_param_count", False)
        self.n_params = cnt.value
        if params is None:
            params = init_params(n_in, width, n_out, seed)
        self.master = torch.tensor(np.asarray(params, dtype=np.float32), device=device)
        assert self.master.numel() == self.n_params
        self.wbf16 = torch.empty(self.n_params, dtype=torch.int16, device=device)
        self.m = torch.zeros(self.n_params, dtype=torch.float32, device=device)
        self.v = torch.zeros(self.n_params, dtype=torch.float32, device=device)
        self.c.master, self.c.wbf16 = self.master.data_ptr(), self.wbf16.data_ptr()
        self.c.adam_m, self.c.adam_v = self.m.data_ptr(), self.v.data_ptr()
        self._ws = {}
        _check(lib().uot_net_sync(default_context().handle, ctypes.byref(self.c)), "uot_net_sync", False)

    def _workspace(self, batch):
        if batch not in self._ws:
            n = ctypes.c_size_t()
            _check(lib().uot_net_workspace_size(ctypes.byref(self.c), batch, ctypes.byref(n)),
                   "uot_net_workspace_size", False)
            self._ws = {batch: workspace(n.value, self.master.device)}
        return self._ws[batch]

    def infer(self, x, ctx: Optional[Context] = None):
        ctx = ctx or default_context()
        batch = x.shape[0]
        _dev(x, torch.float32, batch * self.c.n_in, "x")
        y = torch.empty(batch, self.c.n_out, dtype=torch.float32, device=x.device)
        ws = self._workspace(batch)
        _check(lib().uot_warmstart_infer(ctx.handle, ctypes.byref(self.c), _ptr(x), _ptr(y), batch, _ptr(ws),
                                         ws.numel()), "uot_warmstart_infer", False)
        return y

    def grad(self, x, t, ctx: Optional[Context] = None):
        ctx = ctx or default_context()
        batch = x.shape[0]
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = c_dbl()
        ws = self._workspace(batch)
        _check(lib().uot_net_grad(ctx.handle, ctypes.byref(self.c), _ptr(x), _ptr(t), batch, _ptr(g),
                                  ctypes.byref(loss), _ptr(ws), ws.numel()), "uot_net_grad", False)
        return g, loss.value

    def train_step(self, x, t, lr, want_loss=False, ctx: Optional[Context] = None):
        ctx = ctx or default_context()
        batch = x.shape[0]
        loss = c_dbl()
        ws = self._workspace(batch)
        _check(lib().uot_warmstart_train_step(ctx.handle, ctypes.byref(self.c), _ptr(x), _ptr(t), batch,
                                              ctypes.c_float(lr), ctypes.byref(loss) if want_loss else None,
                                              _ptr(ws), ws.numel()), "uot_warmstart_train_step", False)
        return loss.value if want_loss else None


def init_params(n_in, width, n_out, seed):
    """He-normal weights, zero biases, in the layout of the C ABI."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for fi, fo in ((n_in, width), (width, width), (width, width), (width, n_out)):
        out.append(rng.standard_normal(fi * fo) * np.sqrt(2.0 / fi))
        out.append(np.zeros(fo))
    return np.concatenate(out).astype(np.float32)


def warmstart_features(p, q, R, r, ctx: Optional[Context] = None):
    """x (nb x 2 r^2): log of the r x r average-pooled densities p and q."""
    ctx = ctx or default_context()
    nb = p.shape[0]
    x = torch.empty(nb, 2 * r * r, dtype=torch.float32, device=p.device)
    _check(lib().uot_warmstart_features(ctx.handle, _ptr(p), _ptr(q), nb, R, r, _ptr(x)), "uot_warmstart_features",
           False)
    return x


def grid_upsample(y, r, R, ctx: Optional[Context] = None):
    ctx = ctx or default_context()
    nb = y.shape[0]
    out = torch.empty(nb, R * R, dtype=torch.float32, device=y.device)
    _check(lib().uot_grid_upsample(ctx.handle, _ptr(y), nb, r, R, _ptr(out)), "uot_grid_upsample", False)
    return out


def bary_local_v0(p, h0, shape, h, lam, eps, ctx: Optional[Context] = None):
    """Local (no transport) warm start of a KL(lam) barycentre on a 2-D grid
    (uot_bary_local_v0): p (n x size), h0 (size) -> v0 (n x size), FP32."""
    ctx = ctx or default_context()
    n = p.shape[0]
    n1, n2 = shape
    _dev(p, torch.float32, n * n1 * n2, "p")
    _dev(h0, torch.float32, n1 * n2, "h0")
    v0 = torch.empty(n, n1 * n2, dtype=torch.float32, device=p.device)
    _check(lib().uot_bary_local_v0(ctx.handle, _ptr(p), _ptr(h0), n, n1, n2, float(h[0]), float(h[1]), float(lam),
                                   float(eps), _ptr(v0)), "uot_bary_local_v0", False)
    return v0


def bary_estimate(p, alpha, eps, F2: Div, ctx: Optional[Context] = None):
    """Pointwise Table estimatebary combination of the inputs (n x size) -> h (size)."""
    ctx = ctx or default_context()
    n, size = p.shape
    h = torch.empty(size, dtype=torch.float32, device=p.device)
    al = (c_dbl * n)(*[float(a) for a in alpha])
    f = F2.c()
    _check(lib().uot_bary_estimate(ctx.handle, _ptr(p), n, size, al, float(eps), ctypes.byref(f), _ptr(h)),
           "uot_bary_estimate", False)
    return h


# ---------------------------------------------------------------------------
# gradient flows (uot_flow)
# ---------------------------------------------------------------------------
FLOW_HEAT, FLOW_CROWD, FLOW_GROWTH = 0, 1, 2
_FLOW_KINDS = {"heat": FLOW_HEAT, "crowd": FLOW_CROWD, "growth": FLOW_GROWTH}


def flow(kind, p0, q, dx, tau, eps, n_steps, shape=None, h=None, x=None, alpha=0.0, cost: Cost = SQEUCLID,
         ctx: Optional[Context] = None, v0=None, record=False, **kw):
    """A gradient flow of n_steps steps (uot_flow): kind "heat", "crowd" or
    "growth" on a grid (shape, h) or on one point cloud x (N x d, X = Y).
    p0: (species, N) or (N,) initial densities w.r.t. dx; q: (N,) reference
    (heat) or cap (crowd, growth).  Per-step solver settings (tol, max_iter,
    eps0, check_every, grid_kernel ...) come through **kw.
    Returns (dens (n_steps+1, species, N), v (species, N), steps, info) with
    steps a list of per-step dicts (iters, residual, status, elapsed_ms)."""
    ctx = ctx or default_context()
    k = _FLOW_KINDS[kind] if isinstance(kind, str) else int(kind)
    dtype = q.dtype
    p0 = p0.reshape(-1, q.numel()) if p0.dim() == 1 else p0
    S, N = p0.shape
    _dev(p0, dtype, S * N, "p0")
    _dev(q, dtype, N, "q")
    _dev(dx, dtype, N, "dx")
    keep = ()
    if shape is not None:
        g = _grid_geom(shape, h, cost)
    else:
        xs = x if x.dim() == 2 else x[:, None]
        if xs.shape[0] == N and xs.shape[1] != N:
            xs = xs.t()
        xs = _dev(xs.contiguous(), dtype, name="x")
        g = UotGeom(UOT_GEOM_POINTS, xs.shape[0], N, N, _ptr(xs), _ptr(xs), (c_i64 * 3)(0, 0, 0),
                    (c_dbl * 3)(0, 0, 0), cost.kind, 0, cost.cut)
        keep = (xs,)
    fp = UotFlowProblem(_dt(q), k, S, 0, g, _ptr(p0), _ptr(q), _ptr(dx), float(tau), float(alpha))
    nbytes = ctypes.c_size_t()
    _check(lib().uot_flow_workspace_size(ctypes.byref(fp), ctypes.byref(nbytes)), "uot_flow_workspace_size", False)
    ws = workspace(nbytes.value, q.device)
    dens = torch.empty(n_steps + 1, S, N, dtype=dtype, device=q.device)
    v = torch.empty(S, N, dtype=dtype, device=q.device)
    if v0 is not None:
        _dev(v0, dtype, S * N, "v0")
    max_iter = kw.get("max_iter", 10000)
    hist = torch.full((max_iter,), float("nan"), dtype=torch.float64, device=q.device) if record else None
    pr = params(eps, v0=v0, res_hist=hist, **kw)
    steps = (UotResult * max(n_steps, 1))()
    code = lib().uot_flow(ctx.handle, ctypes.byref(fp), ctypes.byref(pr), int(n_steps), _ptr(dens), _ptr(v),
                          _ptr(ws), ws.numel(), steps)
    _check(code, "uot_flow")
    del keep
    out = [dict(iters=steps[i].iters, residual=steps[i].residual, status=steps[i].status,
                elapsed_ms=steps[i].elapsed_ms) for i in range(n_steps)]
    info = dict(converged=(code == UOT_OK), elapsed_ms=sum(o["elapsed_ms"] for o in out))
    if record:
        info["res_hist"] = hist.cpu()
    return dens, v, out, info
