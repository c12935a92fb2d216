"""CPU checks of the C-ABI boundary: the library loads, exports every entry
point include/uot.h declares, the ctypes structs match the C layout, and the
host-side validation rejects bad input before any GPU work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "uot.h")

uot = pytest.importorskip("paper_1607_05816_amd.uot")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(uot_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = uot.lib()
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", uot.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (uot_\w+)", out))
    assert set(names) <= exported


def test_abi_version_and_status_strings():
    L = uot.lib()
    assert L.uot_abi_version() == 3
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert len(L.uot_status_string(code)) > 0


_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "uot.h"
#define S(T) printf(#T " %zu\n", sizeof(T));
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  S(uot_div) S(uot_geom) S(uot_problem) S(uot_params) S(uot_result) S(uot_objective_values) S(uot_bary_problem)
  S(uot_batch_problem) S(uot_batch_result) S(uot_flow_problem)
  O(uot_geom, cost) O(uot_geom, cut) O(uot_flow_problem, geom) O(uot_flow_problem, p0) O(uot_flow_problem, tau)
  O(uot_flow_problem, alpha)
  O(uot_batch_problem, F2) O(uot_batch_problem, dy) O(uot_batch_result, tune_ms) O(uot_batch_result, tile_rows) O(uot_batch_result, product)
  O(uot_geom, n) O(uot_geom, h) O(uot_problem, geom) O(uot_problem, F1) O(uot_problem, F2)
  O(uot_params, v0) O(uot_params, res_hist) O(uot_params, check_every) O(uot_params, kernel_ms) O(uot_params, kernel_launches) O(uot_params, grid_kernel) O(uot_params, rebalance_at)
  O(uot_bary_problem, alpha) O(uot_bary_problem, F2) O(uot_result, elapsed_ms)
  return 0;
}
"""


def test_ctypes_layout_matches_c_header():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write(_PROBE)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    c = {}
    for line in out.splitlines():
        k, v = line.split()
        c[k] = int(v)
    py = {"uot_div": uot.UotDiv, "uot_geom": uot.UotGeom, "uot_problem": uot.UotProblem,
          "uot_params": uot.UotParams, "uot_result": uot.UotResult,
          "uot_objective_values": uot.UotObjectiveValues, "uot_bary_problem": uot.UotBaryProblem,
          "uot_batch_problem": uot.UotBatchProblem, "uot_batch_result": uot.UotBatchResult,
          "uot_flow_problem": uot.UotFlowProblem}
    for k, T in py.items():
        assert ctypes.sizeof(T) == c[k], k
    pyname = {"F1": "F1", "F2": "F2"}
    for key, val in c.items():
        if "." in key:
            s, f = key.split(".")
            assert getattr(py[s], pyname.get(f, f)).offset == val, key


def _geom_points(N, M, d=2):
    g = uot.UotGeom()
    g.kind, g.dim, g.N, g.M = uot.UOT_GEOM_POINTS, d, N, M
    g.x = ctypes.c_void_p(0x1000)
    g.y = ctypes.c_void_p(0x2000)
    return g


def test_workspace_size_and_validation_on_host():
    L = uot.lib()
    pb = uot.UotProblem()
    pb.dtype = uot.UOT_F32
    pb.geom = _geom_points(1000, 700, 3)
    n = ctypes.c_size_t()
    assert L.uot_workspace_size(ctypes.byref(pb), ctypes.byref(n)) == 0
    assert n.value > 4 * (1000 + 700)
    # grid geometry: size grows with the grid
    pg = uot.UotProblem()
    pg.dtype = uot.UOT_F32
    pg.geom.kind, pg.geom.dim = uot.UOT_GEOM_GRID, 2
    pg.geom.n[0], pg.geom.n[1] = 64, 48
    pg.geom.h[0], pg.geom.h[1] = 1 / 64, 1 / 48
    assert L.uot_workspace_size(ctypes.byref(pg), ctypes.byref(n)) == 0
    small = n.value
    pg.geom.n[0] = 256
    assert L.uot_workspace_size(ctypes.byref(pg), ctypes.byref(n)) == 0
    assert n.value > small
    # invalid: dimension 4, zero spacing, bad dtype
    pb.geom.dim = 4
    assert L.uot_workspace_size(ctypes.byref(pb), ctypes.byref(n)) == -2
    pg.geom.h[1] = 0.0
    assert L.uot_workspace_size(ctypes.byref(pg), ctypes.byref(n)) == -1
    pb.geom.dim = 2
    pb.dtype = 7
    assert L.uot_workspace_size(ctypes.byref(pb), ctypes.byref(n)) == -1
    assert b"dtype" in L.uot_last_error()


def test_solve_rejects_bad_arguments_before_gpu_work():
    """Argument checks run on the host and return an error code; a NULL
    context is rejected without touching the device."""
    L = uot.lib()
    pb = uot.UotProblem()
    pr = uot.UotParams()
    res = uot.UotResult()
    assert L.uot_solve(None, ctypes.byref(pb), ctypes.byref(pr), None, None, None, 0, ctypes.byref(res)) == -1
    assert L.uot_destroy(None) == 0


def test_binding_has_no_cpu_fallback(monkeypatch, tmp_path):
    """With the shared library absent the binding raises instead of computing."""
    import importlib
    mod = importlib.import_module("paper_1607_05816_amd.uot")
    monkeypatch.setattr(mod, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(mod, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        mod.lib()


def test_batch_workspace_and_validation():
    import numpy as np
    L = uot.lib()
    Ns = np.array([0, 64, 1000, 4096], dtype=np.int64)
    Ms = np.array([0, 100, 3000, 3064], dtype=np.int64)
    bp = uot.UotBatchProblem()
    bp.dtype, bp.dim, bp.B = uot.UOT_F32, 2, 3
    bp.offN = Ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    bp.offM = Ms.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    n = ctypes.c_size_t()
    assert L.uot_batch_workspace_size(ctypes.byref(bp), ctypes.byref(n)) == 0
    assert n.value > 4 * 3 * (4096 + 3064)
    bad = np.array([0, 64, 64, 100], dtype=np.int64)        # an empty problem
    bp.offN = bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    assert L.uot_batch_workspace_size(ctypes.byref(bp), ctypes.byref(n)) == -1
    assert b"N, M >= 1" in L.uot_last_error()


def test_wf_cost_and_flow_validation_on_host():
    """WF cost and gradient-flow arguments are checked on the host."""
    L = uot.lib()
    n = ctypes.c_size_t()
    # WF cost: a cut > 0 is needed, and grids must be 1-D (not separable)
    pg = uot.UotProblem()
    pg.dtype = uot.UOT_F32
    pg.geom.kind, pg.geom.dim = uot.UOT_GEOM_GRID, 1
    pg.geom.n[0], pg.geom.h[0] = 300, 1 / 300
    pg.geom.cost, pg.geom.cut = uot.UOT_COST_WF, 0.2
    assert L.uot_workspace_size(ctypes.byref(pg), ctypes.byref(n)) == 0
    pg.geom.cut = 0.0
    assert L.uot_workspace_size(ctypes.byref(pg), ctypes.byref(n)) == -1
    pg.geom.cut = 0.2
    pg.geom.dim = 2
    pg.geom.n[1], pg.geom.h[1] = 64, 1 / 64
    assert L.uot_workspace_size(ctypes.byref(pg), ctypes.byref(n)) == -2
    assert b"separable" in L.uot_last_error()
    pg.geom.cost = 5
    assert L.uot_workspace_size(ctypes.byref(pg), ctypes.byref(n)) == -1
    # flows
    fp = uot.UotFlowProblem()
    fp.dtype, fp.kind, fp.species = uot.UOT_F32, uot.FLOW_GROWTH, 1
    fp.geom.kind, fp.geom.dim = uot.UOT_GEOM_GRID, 1
    fp.geom.n[0], fp.geom.h[0] = 3000, 1 / 3000
    fp.geom.cost, fp.geom.cut = uot.UOT_COST_WF, 1.5707963267948966
    fp.p0 = fp.q = fp.dx = ctypes.c_void_p(0x1000)
    fp.tau, fp.alpha = 0.006, 1.0
    assert L.uot_flow_workspace_size(ctypes.byref(fp), ctypes.byref(n)) == 0
    assert n.value > 4 * 3000 * 4
    fp.species = 2
    assert L.uot_flow_workspace_size(ctypes.byref(fp), ctypes.byref(n)) == 0
    fp.alpha = 100.0                                  # 2 tau alpha >= 1
    assert L.uot_flow_workspace_size(ctypes.byref(fp), ctypes.byref(n)) == -1
    fp.alpha = 1.0
    fp.kind = uot.FLOW_HEAT                           # several species: growth only
    assert L.uot_flow_workspace_size(ctypes.byref(fp), ctypes.byref(n)) == -2
    fp.kind, fp.species = uot.FLOW_CROWD, 1
    fp.geom.kind, fp.geom.dim, fp.geom.N, fp.geom.M = uot.UOT_GEOM_POINTS, 2, 100, 100
    fp.geom.x, fp.geom.y = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    assert L.uot_flow_workspace_size(ctypes.byref(fp), ctypes.byref(n)) == -1    # X != Y
    assert b"same points" in L.uot_last_error()
    fp.geom.y = fp.geom.x
    assert L.uot_flow_workspace_size(ctypes.byref(fp), ctypes.byref(n)) == 0
    pr = uot.UotParams()
    assert L.uot_flow(None, ctypes.byref(fp), ctypes.byref(pr), 1, None, None, None, 0, None) == -1
    # the growth divergence: 0 <= lambda < 1
    # (the problem check fails before the context or the zeroed params are used)
    pb = uot.UotProblem()
    pb.p = pb.q = pb.dx = pb.dy = ctypes.c_void_p(0x1000)
    pb.F1 = uot.KL(1.0).c()
    pb.F2 = uot.GROWTH(1.2).c()
    assert L.uot_solve(ctypes.c_void_p(1), ctypes.byref(pb), ctypes.byref(pr), None, None, None, 0,
                       ctypes.byref(uot.UotResult())) == -1
    assert b"growth" in L.uot_last_error()


def test_point_layout_is_explicit_when_the_shape_is_square():
    """Coordinates may come as (N, d) or (d, N); a square array fits both and
    must name its layout instead of being guessed."""
    import torch
    from paper_1607_05816_amd.uot import _coord_major
    a = torch.arange(6.0).reshape(3, 2)                   # 3 points in R^2
    assert torch.equal(_coord_major(a, 3, None, "x"), a.t())
    assert torch.equal(_coord_major(a.t(), 3, None, "x"), a.t())
    sq = torch.arange(4.0).reshape(2, 2)                  # 2 points in R^2
    with pytest.raises(ValueError, match="layout"):
        _coord_major(sq, 2, None, "x")
    assert torch.equal(_coord_major(sq, 2, "nd", "x"), sq.t())
    assert torch.equal(_coord_major(sq, 2, "dn", "x"), sq)
    assert _coord_major(torch.arange(5.0), 5, None, "x").shape == (1, 5)
    with pytest.raises(ValueError):
        _coord_major(a, 4, None, "x")
