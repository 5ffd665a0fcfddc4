"""ctypes binding of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product package never imports it.

Build with `python -m oracle.build` (or `__graft_entry__.build()`).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

FIXPOINT, FAILED = 0, 1
SCHED_GS, SCHED_JACOBI, SCHED_PERM, SCHED_SELECT, SCHED_REVERSE = 0, 1, 2, 3, 4
ENUMERATE, MINIMIZE = 0, 1
FIRST_FAIL, INPUT_ORDER, EXPERT, MLP = 0, 1, 2, 3
OUT_ALL, OUT_OPTIMAL, OUT_UNSAT, OUT_LIMIT = 0, 1, 2, 3
OUTCOME_NAMES = {OUT_ALL: "all", OUT_OPTIMAL: "optimal", OUT_UNSAT: "unsat",
                 OUT_LIMIT: "limit"}

_P32 = C.POINTER(C.c_int32)


class _Model(C.Structure):
    _fields_ = [("nvars", C.c_int32), ("lb0", _P32), ("ub0", _P32),
                ("nrows", C.c_int32), ("row_ptr", _P32), ("coef", _P32),
                ("var", _P32), ("rhs", _P32), ("nreif", C.c_int32),
                ("reif", _P32), ("ndec", C.c_int32), ("dec", _P32),
                ("objective", C.c_int32), ("ncmd", C.c_int32), ("cmd", _P32),
                ("cmd_gptr", _P32), ("guard", _P32), ("cmd_tptr", _P32),
                ("cterm", _P32)]


_PF = C.POINTER(C.c_float)


class _FModel(C.Structure):
    _fields_ = [("nvars", C.c_int32), ("lb0", _PF), ("ub0", _PF), ("nrows", C.c_int32),
                ("row_ptr", _P32), ("coef", _PF), ("var", _P32), ("rhs", _PF)]


class _Stats(C.Structure):
    _fields_ = [("nodes", C.c_int64), ("fails", C.c_int64),
                ("solutions", C.c_int64), ("max_depth", C.c_int64),
                ("sweeps", C.c_int64), ("best", C.c_int32),
                ("outcome", C.c_int32), ("sol_hash", C.c_uint64)]


_lib = None


def use_library(path):
    """Load the oracle from `path` instead of LIB_PATH (the benchmark's
    CPU baseline times a copy built with -march=native on its host)."""
    global _lib
    _lib = _load(path)
    return _lib


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library not built: {LIB_PATH} "
                               "(run `python -m oracle.build`)")
        _lib = _load(LIB_PATH)
    return _lib


def _load(path):
    L = C.CDLL(path)
    MP = C.POINTER(_Model)
    L.orc_validate.argtypes = [MP]
    L.orc_validate.restype = C.c_int32
    L.orc_propagate.argtypes = [MP, _P32, _P32, C.c_int32, C.c_uint64,
                                C.POINTER(C.c_int64)]
    L.orc_propagate.restype = C.c_int32
    L.orc_jacobi_step.argtypes = [MP, _P32, _P32]
    L.orc_jacobi_step.restype = C.c_int32
    L.orc_gs_step.argtypes = [MP, _P32, _P32]
    L.orc_gs_step.restype = C.c_int32
    L.orc_solve.argtypes = [MP, C.c_int32, C.c_int32, C.c_int64, _P32,
                            C.c_int64, _P32, C.POINTER(_Stats)]
    L.orc_solve.restype = C.c_int32
    L.orc_solution_hash.argtypes = [_P32, C.c_int32]
    L.orc_solution_hash.restype = C.c_uint64
    L.orc_brute_points.argtypes = [MP, _P32, C.c_int64, C.POINTER(C.c_uint64)]
    L.orc_brute_points.restype = C.c_int64
    L.orc_brute_rcpsp.argtypes = [C.c_int32, _P32, C.c_int32, _P32, C.c_int32,
                                  _P32, _P32, C.c_int32, _P32]
    L.orc_brute_rcpsp.restype = C.c_int32
    L.orc_check_schedule.argtypes = [C.c_int32, _P32, C.c_int32, _P32,
                                     C.c_int32, _P32, _P32, _P32, _P32]
    L.orc_check_schedule.restype = C.c_int32
    PD = C.POINTER(C.c_double)
    L.orc_features.argtypes = [MP, _P32, _P32, PD]
    L.orc_features.restype = C.c_int32
    L.orc_mlp_forward.argtypes = [PD, PD, C.c_int64, PD]
    L.orc_mlp_forward.restype = C.c_int32
    L.orc_mlp_loss_grad.argtypes = [PD, PD, _P32, PD, C.c_int32, PD, PD]
    L.orc_mlp_loss_grad.restype = C.c_int32
    L.orc_trace.argtypes = [MP, C.c_int32, C.c_int64, C.POINTER(C.c_float), PD, _P32,
                            _P32, _P32, C.c_int64, C.c_int64, C.POINTER(C.c_int64)]
    L.orc_trace.restype = C.c_int64
    L.orc_set_mlp_params.argtypes = [PD]
    L.orc_set_mlp_params.restype = None
    L.orc_mlp_choice.argtypes = [MP, PD, _P32, _P32]
    L.orc_mlp_choice.restype = C.c_int32
    L.orc_floor_div.argtypes = [C.c_int64, C.c_int64]
    L.orc_floor_div.restype = C.c_int64
    L.orc_ceil_div.argtypes = [C.c_int64, C.c_int64]
    L.orc_ceil_div.restype = C.c_int64
    L.orc_solve_timed.argtypes = [C.POINTER(MP), C.c_int32, C.c_int32, C.c_int32, C.c_int64,
                                  C.c_int32, C.POINTER(C.c_int64), PD, _P32, _P32, PD]
    L.orc_solve_timed.restype = C.c_int32
    L.orc_adam_step.argtypes = [PD, PD, PD, PD, C.c_int32, C.c_double, C.c_int32]
    L.orc_adam_step.restype = C.c_int32
    FP = C.POINTER(_FModel)
    L.orc_fvalidate.argtypes = [FP]
    L.orc_fvalidate.restype = C.c_int32
    L.orc_fpropagate.argtypes = [FP, _PF, _PF, C.c_int32, C.c_uint64, C.POINTER(C.c_int64)]
    L.orc_fpropagate.restype = C.c_int32
    L.orc_fjacobi_step.argtypes = [FP, _PF, _PF]
    L.orc_fjacobi_step.restype = C.c_int32
    L.orc_fsame.argtypes = [C.c_int32, _PF, _PF]
    L.orc_fsame.restype = C.c_int32
    return L


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P32)


class OracleModel:
    """Holds int32 copies of a `Model`'s arrays and the C struct over them."""

    def __init__(self, model):
        self.model = model
        self._keep = [_i32(model.lb), _i32(model.ub), _i32(model.lin_ptr),
                      _i32(model.lin_coef), _i32(model.lin_var), _i32(model.lin_rhs),
                      _i32(model.reif).reshape(-1), _i32(model.decision),
                      _i32(model.cmd).reshape(-1), _i32(model.cmd_gptr),
                      _i32(model.cmd_guard).reshape(-1), _i32(model.cmd_tptr),
                      _i32(model.cmd_term).reshape(-1)]
        lb, ub, ptr, coef, var, rhs, reif, dec, cmd, gptr, guard, tptr, cterm = self._keep
        self.s = _Model(model.nvars, _ptr(lb), _ptr(ub), model.nrows, _ptr(ptr),
                        _ptr(coef), _ptr(var), _ptr(rhs), model.nreif, _ptr(reif),
                        int(dec.shape[0]), _ptr(dec), int(model.objective),
                        model.ncmd, _ptr(cmd), _ptr(gptr), _ptr(guard), _ptr(tptr),
                        _ptr(cterm))

    def ref(self):
        return C.byref(self.s)


def _om(model) -> OracleModel:
    return model if isinstance(model, OracleModel) else OracleModel(model)


def validate(model) -> int:
    return int(lib().orc_validate(_om(model).ref()))


def propagate(model, lb=None, ub=None, sched=SCHED_GS, seed=0):
    """Fixed point above (lb, ub) (default: the model's initial box).
    Returns (status, lb, ub, sweeps); status FIXPOINT or FAILED."""
    om = _om(model)
    m = om.model
    lb = np.array(m.lb if lb is None else lb, dtype=np.int32, copy=True)
    ub = np.array(m.ub if ub is None else ub, dtype=np.int32, copy=True)
    sw = C.c_int64(0)
    st = lib().orc_propagate(om.ref(), _ptr(lb), _ptr(ub), int(sched),
                             C.c_uint64(seed & (2**64 - 1)), C.byref(sw))
    if st < 0:
        raise ValueError(f"orc_propagate error {st}")
    return int(st), lb, ub, int(sw.value)


def jacobi_step(model, lb, ub):
    om = _om(model)
    lb = np.array(lb, dtype=np.int32, copy=True)
    ub = np.array(ub, dtype=np.int32, copy=True)
    st = lib().orc_jacobi_step(om.ref(), _ptr(lb), _ptr(ub))
    if st < 0:
        raise ValueError(f"orc_jacobi_step error {st}")
    return int(st), lb, ub


def gs_step(model, lb, ub):
    om = _om(model)
    lb = np.array(lb, dtype=np.int32, copy=True)
    ub = np.array(ub, dtype=np.int32, copy=True)
    st = lib().orc_gs_step(om.ref(), _ptr(lb), _ptr(ub))
    if st < 0:
        raise ValueError(f"orc_gs_step error {st}")
    return int(st), lb, ub


def solve(model, mode=None, branching=FIRST_FAIL, node_limit=0, sol_cap=0):
    """Depth-first search.  Returns a dict with nodes, fails, solutions,
    max_depth, sweeps, best, outcome, sol_hash, solutions_list, best_assign."""
    om = _om(model)
    m = om.model
    mode = m.mode if mode is None else mode
    nd = int(m.decision.shape[0])
    buf = np.zeros((max(sol_cap, 1), max(nd, 1)), dtype=np.int32)
    best = np.zeros(max(nd, 1), dtype=np.int32)
    st = _Stats()
    rc = lib().orc_solve(om.ref(), int(mode), int(branching), int(node_limit),
                         _ptr(buf) if sol_cap > 0 else None, int(sol_cap),
                         _ptr(best), C.byref(st))
    if rc < 0:
        raise ValueError(f"orc_solve error {rc}")
    nsol = int(min(st.solutions, sol_cap))
    return dict(nodes=st.nodes, fails=st.fails, solutions=st.solutions,
                max_depth=st.max_depth, sweeps=st.sweeps,
                best=None if st.best == 2**31 - 1 else int(st.best),
                outcome=int(st.outcome), sol_hash=int(st.sol_hash),
                solutions_list=buf[:nsol, :nd].copy(),
                best_assign=best[:nd].copy() if st.best != 2**31 - 1 else None)


def solve_timed(models, threads, mode=MINIMIZE, branching=FIRST_FAIL, node_limit=0):
    """orc_solve on independent instances, `threads` POSIX threads, timed in
    C (CLOCK_MONOTONIC).  Returns dict(nodes, secs, outcome, best per
    instance; wall_s for the set)."""
    oms = [_om(m) for m in models]
    n = len(oms)
    arr = (C.POINTER(_Model) * max(n, 1))(*[C.pointer(o.s) for o in oms])
    nodes = np.zeros(max(n, 1), dtype=np.int64)
    secs = np.zeros(max(n, 1), dtype=np.float64)
    out = np.zeros(max(n, 1), dtype=np.int32)
    best = np.zeros(max(n, 1), dtype=np.int32)
    wall = C.c_double(0.0)
    rc = lib().orc_solve_timed(arr, n, int(mode), int(branching), int(node_limit), int(threads),
                               nodes.ctypes.data_as(C.POINTER(C.c_int64)), _pd(secs), _ptr(out),
                               _ptr(best), C.byref(wall))
    if rc < 0:
        raise ValueError(f"orc_solve_timed error {rc}")
    return dict(nodes=nodes[:n].copy(), secs=secs[:n].copy(), outcome=out[:n].copy(),
                best=[None if b == 2**31 - 1 else int(b) for b in best[:n]],
                wall_s=float(wall.value))


def solution_hash(vals) -> int:
    v = _i32(vals)
    return int(lib().orc_solution_hash(_ptr(v), int(v.shape[0])))


def brute_points(model, cap=0):
    """(count, hash, solutions[:cap]) of all points of the initial box."""
    om = _om(model)
    nd = int(om.model.decision.shape[0])
    buf = np.zeros((max(cap, 1), max(nd, 1)), dtype=np.int32)
    h = C.c_uint64(0)
    n = lib().orc_brute_points(om.ref(), _ptr(buf) if cap > 0 else None, int(cap),
                               C.byref(h))
    if n < 0:
        raise ValueError("orc_brute_points: invalid model")
    return int(n), int(h.value), buf[:min(n, cap), :nd].copy()


def _raw(meta):
    n = len(meta["durations"])
    dur = _i32(meta["durations"])
    edges = _i32(np.asarray(meta["edges"], dtype=np.int32).reshape(-1))
    dem = _i32(np.asarray(meta["demands"], dtype=np.int32).reshape(-1))
    cap = _i32(meta["capacities"])
    return n, dur, edges, dem, cap


def brute_rcpsp(meta):
    """Minimum makespan of the raw RCPSP in `meta` (None if infeasible)."""
    n, dur, edges, dem, cap = _raw(meta)
    best_s = np.zeros(max(n, 1), dtype=np.int32)
    b = lib().orc_brute_rcpsp(n, _ptr(dur), int(edges.shape[0] // 2), _ptr(edges),
                              len(meta["capacities"]), _ptr(dem), _ptr(cap),
                              int(meta["horizon"]), _ptr(best_s))
    if b == -2:
        raise ValueError("edges must go from lower to higher task index")
    return (None, None) if b < 0 else (int(b), best_s[:n].copy())


def check_schedule(meta, s):
    n, dur, edges, dem, cap = _raw(meta)
    s = _i32(s)
    ms = C.c_int32(0)
    ok = lib().orc_check_schedule(n, _ptr(dur), int(edges.shape[0] // 2), _ptr(edges),
                                  len(meta["capacities"]), _ptr(dem), _ptr(cap),
                                  _ptr(s), C.cast(C.pointer(ms), _P32))
    return bool(ok), int(ms.value)


def floor_div(a: int, b: int) -> int:
    return int(lib().orc_floor_div(a, b))


def ceil_div(a: int, b: int) -> int:
    return int(lib().orc_ceil_div(a, b))


# ---------------------------------------------------------------- learned
NFEAT, NHID = 6, 64
NPARAM = NHID * NFEAT + NHID + NHID + 1


def _pd(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def features(model, lb, ub):
    """[ndecision, 6] float64 features of a store."""
    om = _om(model)
    lb, ub = _i32(lb), _i32(ub)
    out = np.zeros((max(int(om.model.decision.shape[0]), 1), NFEAT), dtype=np.float64)
    rc = lib().orc_features(om.ref(), _ptr(lb), _ptr(ub), _pd(out))
    if rc < 0:
        raise ValueError(f"orc_features error {rc}")
    return out[:int(om.model.decision.shape[0])]


def mlp_forward(params, x):
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, NFEAT)
    out = np.zeros(max(x.shape[0], 1), dtype=np.float64)
    lib().orc_mlp_forward(_pd(p), _pd(x), x.shape[0], _pd(out))
    return out[:x.shape[0]]


def one_hot(node_off, label):
    t = np.zeros(int(node_off[-1]), dtype=np.float64)
    t[np.asarray(node_off[:-1]) + np.asarray(label)] = 1.0
    return t


def mlp_loss_grad(params, x, node_off, target):
    """Loss and gradient; `target` is a distribution per node over its
    candidates ([C] floats), e.g. one_hot(off, label)."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, NFEAT)
    off = _i32(node_off)
    t = np.ascontiguousarray(target, dtype=np.float64)
    assert t.shape == (x.shape[0],)
    g = np.zeros(NPARAM, dtype=np.float64)
    loss = C.c_double(0.0)
    lib().orc_mlp_loss_grad(_pd(p), _pd(x), _ptr(off), _pd(t), int(off.shape[0] - 1),
                            C.byref(loss), _pd(g))
    return float(loss.value), g


def adam_step(p, g, m, v, lr, step):
    """One Adam step; returns new (p, m, v) as float64 arrays."""
    p = np.array(p, dtype=np.float64, copy=True)
    m = np.array(m, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    g = np.ascontiguousarray(g, dtype=np.float64)
    rc = lib().orc_adam_step(_pd(p), _pd(g), _pd(m), _pd(v), int(p.shape[0]), float(lr), int(step))
    if rc < 0:
        raise ValueError(f"orc_adam_step error {rc}")
    return p, m, v


def trace(model, node_limit, mode=None, cap_nodes=100000, cap_cand=4000000):
    """Expert-labelled search trace: dict(feat [C,6] f32, cand [C], off [N+1],
    label [N])."""
    om = _om(model)
    mode = om.model.mode if mode is None else mode
    feat = np.zeros((cap_cand, NFEAT), dtype=np.float32)
    score = np.zeros(cap_cand, dtype=np.float64)
    cand = np.zeros(cap_cand, dtype=np.int32)
    off = np.zeros(cap_nodes + 1, dtype=np.int32)
    lab = np.zeros(cap_nodes, dtype=np.int32)
    nc = C.c_int64(0)
    n = lib().orc_trace(om.ref(), int(mode), int(node_limit),
                        feat.ctypes.data_as(C.POINTER(C.c_float)), _pd(score), _ptr(cand), _ptr(off),
                        _ptr(lab), cap_nodes, cap_cand, C.byref(nc))
    if n < 0:
        raise ValueError(f"orc_trace error {n}")
    c = int(nc.value)
    return dict(feat=feat[:c].copy(), score=score[:c].copy(), cand=cand[:c].copy(),
                off=off[:n + 1].copy(), label=lab[:n].copy())


def mlp_choice(model, params, lb, ub):
    """Decision-list position the network branches on at the store (lb, ub)
    (the earliest of equal scores; fixed candidates skipped), or -1."""
    om = _om(model)
    p = np.ascontiguousarray(params, dtype=np.float64)
    assert p.shape == (NPARAM,)
    lb, ub = _i32(lb), _i32(ub)
    return int(lib().orc_mlp_choice(om.ref(), _pd(p), _ptr(lb), _ptr(ub)))


_mlp_keep = None


def set_mlp_params(params):
    """Parameters for MLP branching in solve(..., branching=MLP)."""
    global _mlp_keep
    _mlp_keep = np.ascontiguousarray(params, dtype=np.float64)
    lib().orc_set_mlp_params(_pd(_mlp_keep))


# ---------------------------------------------------------------- float stores
def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _pf(a: np.ndarray):
    return a.ctypes.data_as(_PF)


class OracleFModel:
    """float32 / int32 copies of an `FModel`'s arrays and the C struct."""

    def __init__(self, model):
        self.model = model
        self._keep = [_f32(model.lb), _f32(model.ub), _i32(model.row_ptr), _f32(model.coef),
                      _i32(model.var), _f32(model.rhs)]
        lb, ub, ptr, coef, var, rhs = self._keep
        self.s = _FModel(model.nvars, _pf(lb), _pf(ub), model.nrows, _ptr(ptr), _pf(coef),
                         _ptr(var), _pf(rhs))

    def ref(self):
        return C.byref(self.s)


def _ofm(model) -> OracleFModel:
    return model if isinstance(model, OracleFModel) else OracleFModel(model)


def fvalidate(model) -> int:
    return int(lib().orc_fvalidate(_ofm(model).ref()))


def fpropagate(model, lb=None, ub=None, sched=SCHED_GS, seed=0):
    """Fixed point of a float interval store above (lb, ub) (default: the
    model's box).  Returns (status, lb, ub, sweeps) with float32 arrays."""
    om = _ofm(model)
    m = om.model
    lb = np.array(m.lb if lb is None else lb, dtype=np.float32, copy=True)
    ub = np.array(m.ub if ub is None else ub, dtype=np.float32, copy=True)
    sw = C.c_int64(0)
    st = lib().orc_fpropagate(om.ref(), _pf(lb), _pf(ub), int(sched),
                              C.c_uint64(seed & (2**64 - 1)), C.byref(sw))
    if st < 0:
        raise ValueError(f"orc_fpropagate error {st}")
    return int(st), lb, ub, int(sw.value)


def fjacobi_step(model, lb, ub):
    om = _ofm(model)
    lb = np.array(lb, dtype=np.float32, copy=True)
    ub = np.array(ub, dtype=np.float32, copy=True)
    st = lib().orc_fjacobi_step(om.ref(), _pf(lb), _pf(ub))
    if st < 0:
        raise ValueError(f"orc_fjacobi_step error {st}")
    return int(st), lb, ub
