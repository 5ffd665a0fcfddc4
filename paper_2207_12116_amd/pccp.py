"""ctypes binding of libpccp (include/pccp.h): argument marshalling only.

Every step of propagation and search runs in the library's HIP kernels.  If
the library is not built, importing the binding raises; there is no
fallback.  Device memory and streams come from PyTorch: `stream` defaults to
torch's current stream, and the batch-propagation entry point takes int32
CUDA tensors.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .instances import Model, MODE_ENUMERATE, MODE_MINIMIZE

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpccp.so")

OK = 0
E_INVALID_ARG, E_MODEL, E_OVERFLOW, E_NOMEM, E_DEVICE = -1, -2, -3, -4, -5
E_LDS_CAPACITY, E_STATE, E_UNSUPPORTED, E_DEPTH = -6, -7, -8, -9
FIXPOINT, FAILED = 0, 1
ENUMERATE, MINIMIZE = MODE_ENUMERATE, MODE_MINIMIZE
OUT_ALL, OUT_OPTIMAL, OUT_UNSAT, OUT_LIMIT, OUT_CANCELLED = 0, 1, 2, 3, 4
OUTCOME_NAMES = {OUT_ALL: "all", OUT_OPTIMAL: "optimal", OUT_UNSAT: "unsat",
                 OUT_LIMIT: "limit", OUT_CANCELLED: "cancelled"}
BRANCH_FIRST_FAIL, BRANCH_INPUT_ORDER, BRANCH_MLP = 0, 1, 2

_P32 = C.POINTER(C.c_int32)
_I32, _I64, _VP = C.c_int32, C.c_int64, C.c_void_p
_PF = C.POINTER(C.c_float)


class Config(C.Structure):
    """pccp_config; zero fields select the defaults."""
    _fields_ = [("wg_size", _I32), ("num_wgs", _I32), ("desc_lds", _I32),
                ("root_lds", _I32), ("max_depth", _I32), ("queue_cap", _I32),
                ("sol_cap", _I64), ("launch", _I32), ("live", _I32),
                ("occupancy", _I32), ("dep", _I32), ("trail_cap", _I32)]


class Limits(C.Structure):
    _fields_ = [("node_limit", _I64), ("time_limit_s", C.c_double), ("cancel", _VP),
                ("inst_node_limit", _I64)]


class Stats(C.Structure):
    _fields_ = [("nodes", _I64), ("fails", _I64), ("solutions", _I64), ("sweeps", _I64),
                ("donations", _I64), ("subtrees", _I64), ("max_depth", _I64),
                ("prop_linear2", _I64), ("prop_reified", _I64), ("prop_linear", _I64),
                ("prop_terms", _I64), ("sol_hash", C.c_uint64), ("best", _I32),
                ("outcome", _I32), ("kernel_ms", C.c_double), ("ttpo_ms", C.c_double),
                ("grid", _I32), ("block", _I32), ("desc_lds", _I32), ("root_lds", _I32),
                ("lds_bytes", _I64), ("live", _I32), ("occupancy", _I32), ("dep", _I32),
                ("pad", _I32), ("atomics", _I64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["best"] = None if d["best"] == 2**31 - 1 else int(d["best"])
        return d


class TuneOpts(C.Structure):
    """pccp_tune_opts; zero fields select the defaults."""
    _fields_ = [("budget_s", C.c_double), ("whole_run", _I32), ("finalists", _I32),
                ("modes", _I32), ("wg_sizes", _I32), ("max_depth", _I32), ("pad", _I32)]


class TuneResult(C.Structure):
    _fields_ = [("cfg", Config), ("nodes_per_s", C.c_double), ("nodes_per_s_long", C.c_double),
                ("grid", _I32), ("status", _I32)]


class LdsPeaks(C.Structure):
    _fields_ = [("read_gbs", C.c_double), ("atomic_gops", C.c_double),
                ("atomic_ret_gops", C.c_double), ("ms", C.c_double * 3), ("num_cus", _I32),
                ("grid", _I32), ("block", _I32), ("pad", _I32)]


EXPORTS = [
    "pccp_model_create", "pccp_model_destroy", "pccp_model_add_vars",
    "pccp_model_add_linear_le", "pccp_model_add_reified_overlap",
    "pccp_model_set_decision_vars", "pccp_model_set_objective", "pccp_model_info",
    "pccp_solver_create", "pccp_solver_destroy", "pccp_propagate", "pccp_get_domains",
    "pccp_propagate_batch", "pccp_solve", "pccp_batch_solve", "pccp_get_stats",
    "pccp_get_solution_count", "pccp_get_solutions", "pccp_get_best",
    "pccp_set_branching", "pccp_solver_capacity", "pccp_last_error", "pccp_version",
    "pccp_node_features", "pccp_mlp_create", "pccp_mlp_destroy", "pccp_mlp_set_params",
    "pccp_mlp_get_params", "pccp_mlp_train_step", "pccp_mlp_get_grads", "pccp_mlp_scores",
    "pccp_mlp_weights", "pccp_model_save_file", "pccp_model_load_file",
    "pccp_get_solution_hash", "pccp_autotune", "pccp_measure_lds_peaks",
    "pccp_solve_noalloc", "pccp_propagate_batch_incr", "pccp_model_add_guarded",
    "pccp_fmodel_create", "pccp_fmodel_destroy", "pccp_fmodel_add_vars",
    "pccp_fmodel_add_linear_le", "pccp_fsolver_create", "pccp_fsolver_destroy",
    "pccp_fpropagate_batch",
]

_lib = None


class PccpError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().pccp_last_error().decode(errors="replace")
        super().__init__(f"{where}: error {code}: {msg}")
        self.code = code


def lib():
    """Load libpccp.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpccp.so is not built ({LIB_PATH}); run "
                          "`python -m paper_2207_12116_amd.build`")
    L = C.CDLL(LIB_PATH)
    sig = {
        "pccp_model_create": [C.POINTER(_VP)],
        "pccp_model_destroy": [_VP],
        "pccp_model_add_vars": [_VP, _I32, _P32, _P32, _P32],
        "pccp_model_add_linear_le": [_VP, _I32, _P32, _P32, _I32],
        "pccp_model_add_reified_overlap": [_VP, _I32, _I32, _I32, _I32],
        "pccp_model_set_decision_vars": [_VP, _I32, _P32],
        "pccp_model_set_objective": [_VP, _I32],
        "pccp_model_info": [_VP, _P32, _P32, _P32, _P32, _P32],
        "pccp_solver_create": [_VP, C.POINTER(Config), _VP, C.POINTER(_VP)],
        "pccp_solver_destroy": [_VP],
        "pccp_fmodel_create": [C.POINTER(_VP)],
        "pccp_fmodel_destroy": [_VP],
        "pccp_fmodel_add_vars": [_VP, _I32, _PF, _PF, _P32],
        "pccp_fmodel_add_linear_le": [_VP, _I32, _PF, _P32, C.c_float],
        "pccp_fsolver_create": [_VP, _I32, _VP, C.POINTER(_VP)],
        "pccp_fsolver_destroy": [_VP],
        "pccp_fpropagate_batch": [_VP, _I32, _VP, _VP, _VP, _VP, _VP, _VP],
        "pccp_propagate": [_VP, _P32, _P32, _P32],
        "pccp_get_domains": [_VP, _P32, _P32, _I32],
        "pccp_propagate_batch": [_VP, _I32, _VP, _VP, _VP, _VP, _VP, _VP],
        "pccp_propagate_batch_incr": [_VP, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP],
        "pccp_solve": [_VP, _I32, C.POINTER(Limits), _P32],
        "pccp_solve_noalloc": [_VP, _I32, C.POINTER(Limits), _P32],
        "pccp_model_add_guarded": [_VP, _I32, _I32, _I32, _I32, _I32, _P32, _P32, _P32, _I32,
                                   _P32, _P32],
        "pccp_batch_solve": [C.POINTER(_VP), _I32, _I32, C.POINTER(Config),
                             C.POINTER(Limits), _P32],
        "pccp_get_stats": [_VP, C.POINTER(Stats)],
        "pccp_get_solution_count": [_VP, C.POINTER(_I64)],
        "pccp_get_solutions": [_VP, _I64, _I64, _P32],
        "pccp_get_best": [_VP, _P32, _P32, _I32],
        "pccp_set_branching": [_VP, _I32, _VP],
        "pccp_solver_capacity": [_VP, _P32, _P32],
        "pccp_node_features": [_VP, _I32, _VP, _VP, _VP],
        "pccp_mlp_create": [C.c_uint64, _VP, C.POINTER(_VP)],
        "pccp_mlp_destroy": [_VP],
        "pccp_mlp_set_params": [_VP, C.POINTER(C.c_float)],
        "pccp_mlp_get_params": [_VP, C.POINTER(C.c_float)],
        "pccp_mlp_train_step": [_VP, _VP, _VP, _VP, _I32, _I32, _I32, C.c_float,
                                C.POINTER(C.c_float)],
        "pccp_mlp_get_grads": [_VP, C.POINTER(C.c_float)],
        "pccp_mlp_scores": [_VP, _VP, _I32, _VP, _I32],
        "pccp_mlp_weights": [_VP, C.POINTER(_VP)],
        "pccp_model_save_file": [_VP, C.c_char_p],
        "pccp_model_load_file": [C.c_char_p, C.POINTER(_VP)],
        "pccp_get_solution_hash": [_VP, C.POINTER(C.c_uint64)],
        "pccp_autotune": [C.POINTER(_VP), _I32, _I32, C.POINTER(TuneOpts), C.POINTER(Config),
                          C.POINTER(TuneResult), _I32, _P32],
        "pccp_measure_lds_peaks": [C.POINTER(LdsPeaks)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = _I32
    L.pccp_last_error.argtypes = []
    L.pccp_last_error.restype = C.c_char_p
    L.pccp_version.argtypes = []
    L.pccp_version.restype = C.c_char_p
    _lib = L
    return L


def _chk(rc, where):
    if rc != OK:
        raise PccpError(rc, where)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_P32)


def _current_stream():
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def _limits(node_limit=0, time_limit=0.0, cancel=None, inst_node_limit=0):
    lim = Limits(int(node_limit), float(time_limit), None, int(inst_node_limit))
    if cancel is not None:          # a pinned int32 torch tensor
        lim.cancel = C.c_void_p(int(cancel.data_ptr()))
    return lim


class ModelHandle:
    """A pccp_model built from an `instances.Model`."""

    def __init__(self, model: Model):
        L = lib()
        h = _VP()
        _chk(L.pccp_model_create(C.byref(h)), "pccp_model_create")
        self.h = h
        lb, ub = _i32(model.lb), _i32(model.ub)
        _chk(L.pccp_model_add_vars(h, model.nvars, _p(lb), _p(ub), None), "add_vars")
        ptr, coef, var, rhs = (_i32(model.lin_ptr), _i32(model.lin_coef),
                               _i32(model.lin_var), _i32(model.lin_rhs))
        for r in range(model.nrows):
            a, b = int(ptr[r]), int(ptr[r + 1])
            cc, vv = coef[a:b], var[a:b]
            _chk(L.pccp_model_add_linear_le(h, b - a, _p(cc), _p(vv), int(rhs[r])),
                 "add_linear_le")
        for b_, si, sj, d in _i32(model.reif).reshape(-1, 4).tolist():
            _chk(L.pccp_model_add_reified_overlap(h, b_, si, sj, d), "add_reified_overlap")
        if model.ncmd:
            cmd = _i32(model.cmd).reshape(-1, 4)
            gptr, tptr = _i32(model.cmd_gptr), _i32(model.cmd_tptr)
            guard = _i32(model.cmd_guard).reshape(-1, 3)
            term = _i32(model.cmd_term).reshape(-1, 2)
            for q in range(model.ncmd):
                x, side, k, div = (int(v) for v in cmd[q])
                g = guard[gptr[q]:gptr[q + 1]]
                t = term[tptr[q]:tptr[q + 1]]
                gv, gs, gc = (np.ascontiguousarray(g[:, i]) for i in range(3))
                ta, ty = np.ascontiguousarray(t[:, 0]), np.ascontiguousarray(t[:, 1])
                _chk(L.pccp_model_add_guarded(h, x, side, k, div, int(g.shape[0]), _p(gv), _p(gs),
                                              _p(gc), int(t.shape[0]), _p(ta), _p(ty)),
                     "add_guarded")
        dec = _i32(model.decision)
        _chk(L.pccp_model_set_decision_vars(h, int(dec.shape[0]), _p(dec)), "set_decision_vars")
        _chk(L.pccp_model_set_objective(h, int(model.objective)), "set_objective")

    @classmethod
    def from_file(cls, path: str) -> "ModelHandle":
        """A model read by pccp_model_load_file."""
        self = cls.__new__(cls)
        h = _VP()
        _chk(lib().pccp_model_load_file(os.fsencode(path), C.byref(h)), "pccp_model_load_file")
        self.h = h
        return self

    def save(self, path: str):
        _chk(lib().pccp_model_save_file(self.h, os.fsencode(path)), "pccp_model_save_file")

    def info(self) -> dict:
        v = [_I32(0) for _ in range(5)]
        _chk(lib().pccp_model_info(self.h, *[C.cast(C.byref(x), _P32) for x in v]),
             "pccp_model_info")
        return dict(zip(("nvars", "nlinear", "nterms", "nreified", "ndecision"),
                        [int(x.value) for x in v]))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pccp_model_destroy(self.h)
            self.h = None


class Solver:
    """A model compiled and uploaded to the current HIP device."""

    def __init__(self, model: Model, config: Config | None = None, stream=None,
                 handle: ModelHandle | None = None, **cfg):
        """`handle`: an already built library model (e.g. read from a file)
        whose content is `model`'s; by default one is built from `model`."""
        L = lib()
        self.model = model
        self.cfg = config if config is not None else Config(**cfg)
        self._mh = handle if handle is not None else ModelHandle(model)
        self.stream = _current_stream() if stream is None else int(stream)
        h = _VP()
        _chk(L.pccp_solver_create(self._mh.h, C.byref(self.cfg), C.c_void_p(self.stream),
                                  C.byref(h)), "pccp_solver_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pccp_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # ---- propagation
    def propagate(self, lb=None, ub=None):
        """Fixed point of a host box (default: the model's initial box).
        Returns (status, lb, ub)."""
        L = lib()
        st = C.c_int32(0)
        if lb is None:
            _chk(L.pccp_propagate(self.h, None, None, C.byref(st)), "pccp_propagate")
        else:
            lb, ub = _i32(lb), _i32(ub)
            _chk(L.pccp_propagate(self.h, _p(lb), _p(ub), C.byref(st)), "pccp_propagate")
        V = self.model.nvars
        olb = np.zeros(V, dtype=np.int32)
        oub = np.zeros(V, dtype=np.int32)
        _chk(L.pccp_get_domains(self.h, _p(olb), _p(oub), V), "pccp_get_domains")
        return int(st.value), olb, oub

    def propagate_batch(self, lb_in, ub_in, lb_out, ub_out, status, sweeps=None):
        """Fixed points of many boxes; int32 CUDA tensors of shape [nbox, nvars]
        (status, sweeps: [nbox]).  Enqueued on the solver's stream."""
        nbox = int(lb_in.shape[0])
        for t in (lb_in, ub_in, lb_out, ub_out):
            assert t.is_cuda and t.is_contiguous() and t.shape == (nbox, self.model.nvars)
        assert status.is_cuda and status.numel() >= nbox
        _chk(lib().pccp_propagate_batch(
            self.h, nbox, C.c_void_p(lb_in.data_ptr()), C.c_void_p(ub_in.data_ptr()),
            C.c_void_p(lb_out.data_ptr()), C.c_void_p(ub_out.data_ptr()),
            C.c_void_p(status.data_ptr()),
            C.c_void_p(sweeps.data_ptr()) if sweeps is not None else None),
            "pccp_propagate_batch")

    def propagate_batch_incr(self, lb_in, ub_in, dvar, dlo, dhi, lb_out, ub_out, status,
                             sweeps=None):
        """Fixed points of fixed-point boxes joined with one decision each
        (lb(dvar) >= dlo, ub(dvar) <= dhi), by dependency-driven propagation;
        int32 CUDA tensors [nbox, nvars] and [nbox].  Enqueued on the solver's
        stream."""
        nbox = int(lb_in.shape[0])
        for t in (lb_in, ub_in, lb_out, ub_out):
            assert t.is_cuda and t.is_contiguous() and t.shape == (nbox, self.model.nvars)
        for t in (dvar, dlo, dhi, status):
            assert t.is_cuda and t.is_contiguous() and t.numel() >= nbox
        if sweeps is not None:
            assert sweeps.is_cuda and sweeps.numel() >= nbox
        v = lambda t: C.c_void_p(t.data_ptr())
        _chk(lib().pccp_propagate_batch_incr(
            self.h, nbox, v(lb_in), v(ub_in), v(dvar), v(dlo), v(dhi), v(lb_out), v(ub_out),
            v(status), v(sweeps) if sweeps is not None else None), "pccp_propagate_batch_incr")

    # ---- search
    def solve(self, mode=None, node_limit=0, time_limit=0.0, cancel=None):
        mode = self.model.mode if mode is None else mode
        out = C.c_int32(0)
        lim = _limits(node_limit, time_limit, cancel)
        _chk(lib().pccp_solve(self.h, int(mode), C.byref(lim), C.byref(out)), "pccp_solve")
        return int(out.value)

    def solve_noalloc(self, mode=None, node_limit=0, time_limit=0.0, cancel=None):
        """pccp_solve_noalloc: the search with its workspace in the library's
        static device array (no allocation; no solution list kept)."""
        mode = self.model.mode if mode is None else mode
        out = C.c_int32(0)
        lim = _limits(node_limit, time_limit, cancel)
        _chk(lib().pccp_solve_noalloc(self.h, int(mode), C.byref(lim), C.byref(out)),
             "pccp_solve_noalloc")
        return int(out.value)

    def stats(self) -> dict:
        st = Stats()
        _chk(lib().pccp_get_stats(self.h, C.byref(st)), "pccp_get_stats")
        return st.as_dict()

    def solution_hash(self) -> int:
        h = C.c_uint64(0)
        _chk(lib().pccp_get_solution_hash(self.h, C.byref(h)), "pccp_get_solution_hash")
        return int(h.value)

    def solution_count(self) -> int:
        n = C.c_int64(0)
        _chk(lib().pccp_get_solution_count(self.h, C.byref(n)), "pccp_get_solution_count")
        return int(n.value)

    def solutions(self, count=None) -> np.ndarray:
        nd = int(self.model.decision.shape[0])
        n = min(self.solution_count(), int(self.cfg.sol_cap)) if count is None else count
        out = np.zeros((max(n, 1), max(nd, 1)), dtype=np.int32)
        if n > 0:
            _chk(lib().pccp_get_solutions(self.h, 0, n, _p(out)), "pccp_get_solutions")
        return out[:n, :nd]

    def best(self):
        nd = int(self.model.decision.shape[0])
        obj = C.c_int32(0)
        vals = np.zeros(max(nd, 1), dtype=np.int32)
        _chk(lib().pccp_get_best(self.h, C.byref(obj), _p(vals), max(nd, 1)), "pccp_get_best")
        if obj.value == 2**31 - 1:
            return None, None
        return int(obj.value), vals[:nd]

    def set_branching(self, kind, weights_ptr=None):
        _chk(lib().pccp_set_branching(self.h, int(kind),
                                      C.c_void_p(weights_ptr) if weights_ptr else None),
             "pccp_set_branching")

    def node_features(self, lb, ub, out):
        """Features of stores (int32 CUDA tensors [nbox, nvars]) into out
        (float32 CUDA tensor [nbox, ndecision, 6])."""
        nbox = int(lb.shape[0])
        _chk(lib().pccp_node_features(self.h, nbox, C.c_void_p(lb.data_ptr()),
                                      C.c_void_p(ub.data_ptr()), C.c_void_p(out.data_ptr())),
             "pccp_node_features")

    def capacity(self):
        a, b = C.c_int32(0), C.c_int32(0)
        _chk(lib().pccp_solver_capacity(self.h, C.byref(a), C.byref(b)), "pccp_solver_capacity")
        return int(a.value), int(b.value)


def batch_solve(solvers, mode=MINIMIZE, config: Config | None = None, node_limit=0,
                time_limit=0.0, cancel=None, inst_node_limit=0):
    """One persistent launch over every solver's model; returns outcomes."""
    n = len(solvers)
    arr = (_VP * n)(*[s.h for s in solvers])
    outs = np.zeros(n, dtype=np.int32)
    lim = _limits(node_limit, time_limit, cancel, inst_node_limit)
    cfg_p = C.byref(config) if config is not None else None
    _chk(lib().pccp_batch_solve(arr, n, int(mode), cfg_p, C.byref(lim), _p(outs)),
         "pccp_batch_solve")
    return outs.tolist()


def autotune(solvers, mode=MINIMIZE, opts: TuneOpts | None = None, cap=256):
    """pccp_autotune: (chosen Config, list of candidate dicts in the order
    tried)."""
    n = len(solvers)
    arr = (_VP * n)(*[s.h for s in solvers])
    best = Config()
    res = (TuneResult * cap)()
    nres = _I32(0)
    _chk(lib().pccp_autotune(arr, n, int(mode), C.byref(opts) if opts is not None else None,
                             C.byref(best), res, cap, C.cast(C.byref(nres), _P32)),
         "pccp_autotune")
    out = []
    for r in res[:min(cap, nres.value)]:
        c = {k: getattr(r.cfg, k) for k, _ in Config._fields_}
        out.append({"config": c, "nodes_per_s": r.nodes_per_s,
                    "nodes_per_s_long": r.nodes_per_s_long, "grid": r.grid, "status": r.status})
    return best, out


def lds_peaks() -> dict:
    """pccp_measure_lds_peaks on the current device."""
    p = LdsPeaks()
    _chk(lib().pccp_measure_lds_peaks(C.byref(p)), "pccp_measure_lds_peaks")
    return {"read_GBs": p.read_gbs, "atomic_Gops": p.atomic_gops,
            "atomic_ret_Gops": p.atomic_ret_gops, "ms": list(p.ms), "num_cus": p.num_cus,
            "grid": p.grid, "block": p.block}


def version() -> str:
    return lib().pccp_version().decode()


NPARAM = 513


class MLP:
    """The learned branching network (pccp_mlp_*)."""

    def __init__(self, seed=0, stream=None):
        h = _VP()
        self.stream = _current_stream() if stream is None else int(stream)
        _chk(lib().pccp_mlp_create(C.c_uint64(seed), C.c_void_p(self.stream), C.byref(h)),
             "pccp_mlp_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pccp_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def params(self) -> np.ndarray:
        out = np.zeros(NPARAM, dtype=np.float32)
        _chk(lib().pccp_mlp_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float))),
             "pccp_mlp_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.shape == (NPARAM,)
        _chk(lib().pccp_mlp_set_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float))),
             "pccp_mlp_set_params")

    def grads(self) -> np.ndarray:
        out = np.zeros(NPARAM, dtype=np.float32)
        _chk(lib().pccp_mlp_get_grads(self.h, out.ctypes.data_as(C.POINTER(C.c_float))),
             "pccp_mlp_get_grads")
        return out

    def train_step(self, feat, off, target, max_cand, lr):
        """feat float32 [C, 6], off int32 [N+1], target float32 [C] (a
        distribution over each node's candidates): CUDA tensors."""
        loss = C.c_float(0.0)
        _chk(lib().pccp_mlp_train_step(
            self.h, C.c_void_p(feat.data_ptr()), C.c_void_p(off.data_ptr()),
            C.c_void_p(target.data_ptr()), int(off.shape[0]) - 1, int(feat.shape[0]),
            int(max_cand), C.c_float(lr), C.byref(loss)), "pccp_mlp_train_step")
        return float(loss.value)

    def scores(self, feat, out, bf16=True):
        _chk(lib().pccp_mlp_scores(self.h, C.c_void_p(feat.data_ptr()), int(feat.shape[0]),
                                   C.c_void_p(out.data_ptr()), 1 if bf16 else 0),
             "pccp_mlp_scores")

    def weights_ptr(self) -> int:
        w = _VP()
        _chk(lib().pccp_mlp_weights(self.h, C.byref(w)), "pccp_mlp_weights")
        return int(w.value)


# ---------------------------------------------------------------- float stores
class FSolver:
    """A float model (instances.FModel) built in the library and uploaded to
    the current HIP device."""

    def __init__(self, model, wg_size: int = 0, stream=None):
        L = lib()
        self.model = model
        mh = _VP()
        _chk(L.pccp_fmodel_create(C.byref(mh)), "pccp_fmodel_create")
        try:
            lb = np.ascontiguousarray(model.lb, dtype=np.float32)
            ub = np.ascontiguousarray(model.ub, dtype=np.float32)
            _chk(L.pccp_fmodel_add_vars(mh, model.nvars, lb.ctypes.data_as(_PF),
                                        ub.ctypes.data_as(_PF), None), "pccp_fmodel_add_vars")
            ptr = np.asarray(model.row_ptr, dtype=np.int32)
            coef = np.ascontiguousarray(model.coef, dtype=np.float32)
            var = np.ascontiguousarray(model.var, dtype=np.int32)
            for r in range(model.nrows):
                a, b = int(ptr[r]), int(ptr[r + 1])
                cc, vv = np.ascontiguousarray(coef[a:b]), np.ascontiguousarray(var[a:b])
                _chk(L.pccp_fmodel_add_linear_le(mh, b - a, cc.ctypes.data_as(_PF), _p(vv),
                                                 float(model.rhs[r])), "pccp_fmodel_add_linear_le")
            self.stream = _current_stream() if stream is None else int(stream)
            h = _VP()
            _chk(L.pccp_fsolver_create(mh, int(wg_size), C.c_void_p(self.stream), C.byref(h)),
                 "pccp_fsolver_create")
            self.h = h
        finally:
            L.pccp_fmodel_destroy(mh)

    def propagate_batch(self, lb_in, ub_in, lb_out, ub_out, status, sweeps=None):
        """Fixed points of float boxes: float32 CUDA tensors [nbox, nvars],
        int32 status / sweeps [nbox].  Enqueued on the solver's stream."""
        nbox = int(lb_in.shape[0])
        for t in (lb_in, ub_in, lb_out, ub_out):
            assert t.is_cuda and t.is_contiguous() and t.shape == (nbox, self.model.nvars)
        assert status.is_cuda and status.numel() >= nbox
        v = lambda t: C.c_void_p(t.data_ptr())
        _chk(lib().pccp_fpropagate_batch(self.h, nbox, v(lb_in), v(ub_in), v(lb_out), v(ub_out),
                                         v(status), v(sweeps) if sweeps is not None else None),
             "pccp_fpropagate_batch")

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.pccp_fsolver_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
