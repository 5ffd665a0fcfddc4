"""Seeded synthetic instances: the tiny CSP and the RCPSP family.

This module produces *input data only*: variable boxes, linear rows,
reified-overlap items, the decision-variable list and the objective.  It holds
none of the solving arithmetic (no propagation, no search); both the HIP
solver and the CPU oracle consume the `Model` it returns.

Randomness: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), uniform integers by rejection sampling so
that every draw is exactly uniform.

Model encoding of the RCPSP follows the PCCP model of §2 (variables s_i over
IZ(0,h), the n*n Boolean overlap variables b_ij over IZ(0,1), one precedence
per edge i << j, one reified overlap per ordered pair (i, j) including i = j,
one resource row per (resource k, task j)), plus a makespan variable m with
s_i + d_i <= m for every task (the paper names the objective but gives no
encoding for it).  The horizon is h = sum of durations, the example the paper
gives for it.

The paper's datasets (Patterson, PSPLIB j30) are not used; these generators
stand in for them with j30's shape (30 tasks, 4 renewable resources) and
larger sizes (60, 90, 120 tasks).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import hashlib

import numpy as np

MASK64 = (1 << 64) - 1

# Configuration ids mixed into the seed so that different workloads never
# share a random stream.
CFG_TINY_CSP = 1
CFG_RCPSP = 2
CFG_TINY_RCPSP = 3
CFG_PREC_ONLY = 4
CFG_JOBSHOP = 5
CFG_FLOAT_CSP = 6
CFG_FLOAT_NET = 7
CFG_FLOAT_EXTREME = 8


class SplitMix64:
    """SplitMix64 stream (Steele, Lea & Flood 2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def below(self, n: int) -> int:
        """Uniform integer in [0, n) by rejection sampling."""
        if n <= 0:
            raise ValueError("n must be positive")
        limit = (1 << 64) - ((1 << 64) % n)
        while True:
            r = self.next_u64()
            if r < limit:
                return r % n

    def uniform(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + self.below(hi - lo + 1)

    def shuffle(self, xs: list) -> None:
        """Fisher-Yates shuffle in place."""
        for i in range(len(xs) - 1, 0, -1):
            j = self.below(i + 1)
            xs[i], xs[j] = xs[j], xs[i]


def stream(config_id: int, seed: int) -> SplitMix64:
    return SplitMix64(((config_id & 0xFFFFFFFF) << 32) ^ (seed & 0xFFFFFFFF))


MODE_ENUMERATE = 0
MODE_MINIMIZE = 1


@dataclass
class Model:
    """A constraint model over int32 interval variables (lattice IZ, §2).

    lb, ub         int32[V]      initial box of every variable
    lin_ptr        int32[R+1]    CSR row pointer of the linear rows
    lin_coef       int32[T]      nonzero coefficients
    lin_var        int32[T]      variable of each term (distinct within a row)
    lin_rhs        int32[R]      row r means  sum_t coef_t * x_t <= rhs_r
    reif           int32[Q, 4]   (b, si, sj, d): b <=> (si <= sj  and  sj < si + d)
    decision       int32[D]      branching candidates, in tie-break order
    objective      int           variable to minimise, or -1
    mode           int           MODE_ENUMERATE or MODE_MINIMIZE
    meta           dict          generator parameters (durations, demands, ...)
    cmd            int32[C, 4]   guarded commands {guards} => x <- f (§3):
                                 (x, side, k, div); side 0 tells lb(x) >=
                                 ceil(f / div), side 1 tells ub(x) <=
                                 floor(f / div), f = k + sum a_t * y_t
    cmd_gptr       int32[C+1]    CSR pointer of the guards
    cmd_guard      int32[G, 3]   (y, side, c): side 0 is entailed(y >= c),
                                 side 1 is entailed(y <= c)
    cmd_tptr       int32[C+1]    CSR pointer of the terms of f
    cmd_term       int32[U, 2]   (a, y), a nonzero
    """

    lb: np.ndarray
    ub: np.ndarray
    lin_ptr: np.ndarray
    lin_coef: np.ndarray
    lin_var: np.ndarray
    lin_rhs: np.ndarray
    reif: np.ndarray
    decision: np.ndarray
    objective: int
    mode: int
    meta: dict = field(default_factory=dict)
    cmd: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), dtype=np.int32))
    cmd_gptr: np.ndarray = field(default_factory=lambda: np.zeros(1, dtype=np.int32))
    cmd_guard: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), dtype=np.int32))
    cmd_tptr: np.ndarray = field(default_factory=lambda: np.zeros(1, dtype=np.int32))
    cmd_term: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), dtype=np.int32))

    @property
    def nvars(self) -> int:
        return int(self.lb.shape[0])

    @property
    def nrows(self) -> int:
        return int(self.lin_rhs.shape[0])

    @property
    def nterms(self) -> int:
        return int(self.lin_coef.shape[0])

    @property
    def nreif(self) -> int:
        return int(self.reif.shape[0])

    @property
    def ncmd(self) -> int:
        return int(self.cmd.shape[0])

    def rows(self):
        """Yield (coef array, var array, rhs) per linear row."""
        for r in range(self.nrows):
            a, b = int(self.lin_ptr[r]), int(self.lin_ptr[r + 1])
            yield self.lin_coef[a:b], self.lin_var[a:b], int(self.lin_rhs[r])

    def content_hash(self) -> str:
        h = hashlib.sha256()
        for arr in (self.lb, self.ub, self.lin_ptr, self.lin_coef, self.lin_var,
                    self.lin_rhs, self.reif, self.decision):
            h.update(np.ascontiguousarray(arr, dtype=np.int32).tobytes())
        h.update(np.int64(self.objective).tobytes())
        h.update(np.int64(self.mode).tobytes())
        if self.ncmd:
            for arr in (self.cmd, self.cmd_gptr, self.cmd_guard, self.cmd_tptr, self.cmd_term):
                h.update(np.ascontiguousarray(arr, dtype=np.int32).tobytes())
        return h.hexdigest()[:16]


class _Builder:
    def __init__(self):
        self.lb: list[int] = []
        self.ub: list[int] = []
        self.ptr = [0]
        self.coef: list[int] = []
        self.var: list[int] = []
        self.rhs: list[int] = []
        self.reif: list[tuple[int, int, int, int]] = []
        self.cmd: list[tuple[int, int, int, int]] = []
        self.gptr = [0]
        self.guard: list[tuple[int, int, int]] = []
        self.tptr = [0]
        self.cterm: list[tuple[int, int]] = []

    def add_vars(self, n: int, lo: int, hi: int) -> int:
        first = len(self.lb)
        self.lb.extend([lo] * n)
        self.ub.extend([hi] * n)
        return first

    def add_row(self, coefs, vars_, rhs: int) -> None:
        pairs = [(int(a), int(v)) for a, v in zip(coefs, vars_) if int(a) != 0]
        if not pairs:
            return  # 0 <= rhs holds for every generated row (rhs >= 0)
        for a, v in pairs:
            self.coef.append(a)
            self.var.append(v)
        self.rhs.append(int(rhs))
        self.ptr.append(len(self.coef))

    def add_reif(self, b: int, si: int, sj: int, d: int) -> None:
        self.reif.append((b, si, sj, d))

    def add_cmd(self, guards, x: int, side: int, k: int, div: int, terms) -> None:
        """{guards} => x <- f: guards (y, side, c), terms (a, y) of f."""
        for y, gs, c in guards:
            self.guard.append((int(y), int(gs), int(c)))
        self.gptr.append(len(self.guard))
        for a, y in terms:
            if int(a) != 0:
                self.cterm.append((int(a), int(y)))
        self.tptr.append(len(self.cterm))
        self.cmd.append((int(x), int(side), int(k), int(div)))

    def finish(self, decision, objective, mode, meta) -> Model:
        i32 = lambda xs: np.asarray(xs, dtype=np.int32)
        reif = np.asarray(self.reif, dtype=np.int32).reshape(-1, 4)
        return Model(i32(self.lb), i32(self.ub), i32(self.ptr), i32(self.coef),
                     i32(self.var), i32(self.rhs), reif, i32(decision),
                     int(objective), int(mode), meta,
                     i32(self.cmd).reshape(-1, 4), i32(self.gptr),
                     i32(self.guard).reshape(-1, 3), i32(self.tptr),
                     i32(self.cterm).reshape(-1, 2))


def tiny_csp(seed: int, nvars: int = 8, dom: int = 20, nprec: int = 12) -> Model:
    """Tiny CSP: `nvars` variables over [0, dom], `nprec` random precedences
    x_u + d <= x_v (d uniform 1..5) along a random topological order (so the
    precedence graph is a DAG), and one row sum_i a_i x_i <= c with a_i
    uniform 1..4 and c = 60% of the largest possible sum (exactly
    0.6 * dom * sum a_i = 12 * sum a_i for dom = 20).  Enumerate all
    solutions, branching over every variable."""
    rng = stream(CFG_TINY_CSP, seed)
    b = _Builder()
    b.add_vars(nvars, 0, dom)
    perm = list(range(nvars))
    rng.shuffle(perm)
    pairs = [(p, q) for p in range(nvars) for q in range(p + 1, nvars)]
    rng.shuffle(pairs)
    precs = []
    for (p, q) in pairs[:nprec]:
        u, v = perm[p], perm[q]
        d = rng.uniform(1, 5)
        precs.append((u, v, d))
        b.add_row([1, -1], [u, v], -d)  # x_u - x_v <= -d
    a = [rng.uniform(1, 4) for _ in range(nvars)]
    c = (dom * sum(a) * 6) // 10
    b.add_row(a, list(range(nvars)), c)
    meta = dict(kind="tiny_csp", seed=seed, precedences=precs, weights=a, cap=c,
                dom=dom)
    return b.finish(list(range(nvars)), -1, MODE_ENUMERATE, meta)


def rcpsp_data(n: int, seed: int, nres: int = 4, cap: int = 10, dmax: int = 10,
               config_id: int = CFG_RCPSP):
    """Raw RCPSP data <T, P, R> (§2): durations, precedence edges, demands,
    capacities.  Durations uniform 1..dmax; each task i < n-1 gets 1..3
    distinct successors drawn uniformly from {i+1, ..., n-1} (all of them if
    fewer remain); each demand r_{k,i} is 0 with probability 1/2, else uniform
    1..10 (clipped to the capacity)."""
    rng = stream(config_id, (n << 20) ^ seed)
    dur = [rng.uniform(1, dmax) for _ in range(n)]
    edges = []
    for i in range(n - 1):
        cands = list(range(i + 1, n))
        k = rng.uniform(1, 3)
        if k >= len(cands):
            succ = cands
        else:
            rng.shuffle(cands)
            succ = sorted(cands[:k])
        edges.extend((i, j) for j in succ)
    dem = [[0] * n for _ in range(nres)]
    for k in range(nres):
        for i in range(n):
            if rng.below(2) == 1:
                dem[k][i] = min(cap, rng.uniform(1, 10))
    caps = [cap] * nres
    return dur, edges, dem, caps


def rcpsp_model(dur, edges, dem, caps, horizon: int | None = None,
                with_overlap: bool = True, meta: dict | None = None) -> Model:
    """The PCCP RCPSP model of §2 with the makespan objective.

    Variable layout: s_i = i (i < n); b_ij = n + i*n + j; m = n + n*n
    (or m = n when `with_overlap` is False, for precedence-only models)."""
    n = len(dur)
    h = sum(dur) if horizon is None else horizon
    b = _Builder()
    s0 = b.add_vars(n, 0, h)
    if with_overlap:
        b0 = b.add_vars(n * n, 0, 1)
    m = b.add_vars(1, 0, h)
    for (i, j) in edges:                       # s_i + d_i <= s_j
        b.add_row([1, -1], [s0 + i, s0 + j], -dur[i])
    for i in range(n):                         # s_i + d_i <= m
        b.add_row([1, -1], [s0 + i, m], -dur[i])
    if with_overlap:
        for j in range(n):
            for i in range(n):                 # b_ij <=> (s_i <= s_j < s_i + d_i)
                b.add_reif(b0 + i * n + j, s0 + i, s0 + j, dur[i])
        for k in range(len(caps)):
            for j in range(n):                 # sum_i r_ki * b_ij <= c_k
                b.add_row([dem[k][i] for i in range(n)],
                          [b0 + i * n + j for i in range(n)], caps[k])
    md = dict(kind="rcpsp", n=n, horizon=h, durations=list(dur), edges=list(edges),
              demands=[list(r) for r in dem], capacities=list(caps))
    if meta:
        md.update(meta)
    return b.finish([s0 + i for i in range(n)], m, MODE_MINIMIZE, md)


def rcpsp(n: int, seed: int) -> Model:
    """Synthetic project scheduling instance with n tasks and 4 resources."""
    dur, edges, dem, caps = rcpsp_data(n, seed)
    return rcpsp_model(dur, edges, dem, caps, meta=dict(seed=seed))


def tiny_rcpsp(n: int, seed: int, dmax: int = 3) -> Model:
    """Tiny RCPSP (n <= 6, short durations) small enough to brute-force."""
    dur, edges, dem, caps = rcpsp_data(n, seed, dmax=dmax, config_id=CFG_TINY_RCPSP)
    return rcpsp_model(dur, edges, dem, caps, meta=dict(seed=seed))


def precedence_only(n: int, seed: int) -> Model:
    """Precedences plus makespan only (no resources): its root fixed point has
    the critical-path closed form."""
    dur, edges, dem, caps = rcpsp_data(n, seed, config_id=CFG_PREC_ONLY)
    return rcpsp_model(dur, edges, dem, caps, with_overlap=False, meta=dict(seed=seed))


def batch_sizes(seed: int) -> int:
    """Mixed-size batch: the task count of seed s is (30, 60, 90)[s mod 3]."""
    return (30, 60, 90)[seed % 3]


def jobshop_data(n_jobs: int, n_mach: int, seed: int, dmax: int = 10):
    """Synthetic job shop: every job visits every machine once, in a random
    order, with durations uniform in 1..dmax.  Returns jobs[j] = list of
    (machine, duration) in the job's order."""
    rng = stream(CFG_JOBSHOP, seed)
    jobs = []
    for _ in range(n_jobs):
        order = list(range(n_mach))
        rng.shuffle(order)
        jobs.append([(m, rng.uniform(1, dmax)) for m in order])
    return jobs


def jobshop(n_jobs: int, n_mach: int, seed: int, guarded: bool = False) -> Model:
    """The job shop as a PCCP program (front-end in `lang`): start times s,
    makespan m; precedences along each job; for every pair of operations on
    one machine, a disjunction of their two orders.  Variable layout: the
    starts job by job, then m, then the auxiliaries of the disjunctions.
    guarded=True states each disjunction with guarded commands (disj_rows:
    once one order is impossible the other is told) instead of a reified
    difference with an implication."""
    from .lang import Program
    jobs = jobshop_data(n_jobs, n_mach, seed)
    h = sum(d for job in jobs for _, d in job)
    p = Program()
    s = [[p.var(0, h) for _ in job] for job in jobs]
    m = p.var(0, h)
    on = {k: [] for k in range(n_mach)}
    for j, job in enumerate(jobs):
        for k, (mach, d) in enumerate(job):
            nxt = s[j][k + 1] if k + 1 < len(job) else m
            p.tell([1, -1], [s[j][k], nxt], -d)            # s + d <= next
            on[mach].append((s[j][k], d))
    for ops in on.values():
        for a in range(len(ops)):
            for b in range(a + 1, len(ops)):
                (x, dx), (y, dy) = ops[a], ops[b]
                if guarded:
                    p.disj_rows([1, -1], [x, y], -dx, [1, -1], [y, x], -dy)
                else:
                    p.disj(x, y, -dx, y, x, -dy)           # x + dx <= y or y + dy <= x
    dec = [v for row in s for v in row]
    return p.compile(decision=dec, objective=m,
                     meta=dict(kind="jobshop", jobs=jobs, n_jobs=n_jobs, n_mach=n_mach,
                               horizon=h, seed=seed, guarded=bool(guarded)))


# ------------------------------------------------------------- model files
# The library's model-file layout (little-endian): the line "PCCP-MODEL 1",
# one line of JSON with nvars, nrows, nterms, nreif, ndec, objective,
# ncmd, nguards, ncterms (and here also the search mode and the generator's
# parameters as "meta"), then int32 arrays lb, ub, row_ptr, coef, var, rhs,
# reif (4 per item), dec, and when ncmd > 0 the guarded commands: cmd (4 per
# command), cmd_gptr, guards (3 per guard), cmd_tptr, terms (2 per term).
MODEL_MAGIC = b"PCCP-MODEL 1\n"


def save_model(model: Model, path: str) -> None:
    import json
    hdr = {"nvars": model.nvars, "nrows": model.nrows, "nterms": model.nterms,
           "nreif": model.nreif, "ndec": int(model.decision.shape[0]),
           "objective": int(model.objective), "ncmd": model.ncmd,
           "nguards": int(np.asarray(model.cmd_guard).reshape(-1, 3).shape[0]),
           "ncterms": int(np.asarray(model.cmd_term).reshape(-1, 2).shape[0]),
           "mode": int(model.mode), "meta": model.meta}
    arrays = [model.lb, model.ub, model.lin_ptr, model.lin_coef, model.lin_var,
              model.lin_rhs, model.reif, model.decision]
    if model.ncmd:
        arrays += [model.cmd, model.cmd_gptr, model.cmd_guard, model.cmd_tptr, model.cmd_term]
    with open(path, "wb") as f:
        f.write(MODEL_MAGIC)
        f.write(json.dumps(hdr, separators=(", ", ": ")).encode() + b"\n")
        for a in arrays:
            f.write(np.ascontiguousarray(a, dtype="<i4").tobytes())


def load_model(path: str) -> Model:
    import json
    with open(path, "rb") as f:
        if f.readline() != MODEL_MAGIC:
            raise ValueError(f"{path}: not a model file")
        hdr = json.loads(f.readline())
        body = np.frombuffer(f.read(), dtype="<i4")
    V, R, T, Q, D = (int(hdr[k]) for k in ("nvars", "nrows", "nterms", "nreif", "ndec"))
    NC, NG, NT = (int(hdr.get(k, 0)) for k in ("ncmd", "nguards", "ncterms"))
    sizes = [V, V, R + 1, T, T, R, 4 * Q, D]
    if NC:
        sizes += [4 * NC, NC + 1, 3 * NG, NC + 1, 2 * NT]
    if body.shape[0] != sum(sizes):
        raise ValueError(f"{path}: {body.shape[0]} values, expected {sum(sizes)}")
    parts, o = [], 0
    for n in sizes:
        parts.append(body[o:o + n].astype(np.int32))
        o += n
    lb, ub, ptr, coef, var, rhs, reif, dec = parts[:8]
    obj = int(hdr["objective"])
    mode = int(hdr.get("mode", MODE_MINIMIZE if obj >= 0 else MODE_ENUMERATE))
    m = Model(lb, ub, ptr, coef, var, rhs, reif.reshape(-1, 4), dec, obj, mode,
              dict(hdr.get("meta", {})))
    if NC:
        m.cmd = parts[8].reshape(-1, 4)
        m.cmd_gptr = parts[9]
        m.cmd_guard = parts[10].reshape(-1, 3)
        m.cmd_tptr = parts[11]
        m.cmd_term = parts[12].reshape(-1, 2)
    return m

# ---------------------------------------------------------------- float models
@dataclass
class FModel:
    """A model over float32 interval variables with linear rows over the
    reals (data only):

    lb, ub     float32[V]   initial box (finite)
    row_ptr    int32[R+1]   CSR pointer of the rows
    coef       float32[T]   nonzero coefficients
    var        int32[T]     variables (distinct within a row)
    rhs        float32[R]   sum_t coef[t] * x_var[t] <= rhs
    """

    lb: np.ndarray
    ub: np.ndarray
    row_ptr: np.ndarray
    coef: np.ndarray
    var: np.ndarray
    rhs: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nvars(self) -> int:
        return int(self.lb.shape[0])

    @property
    def nrows(self) -> int:
        return int(self.rhs.shape[0])

    @property
    def nterms(self) -> int:
        return int(self.coef.shape[0])


def _f32(v) -> float:
    return float(np.float32(v))


def _fmodel(lb, ub, rows, meta) -> FModel:
    ptr, coef, var, rhs = [0], [], [], []
    for a, x, c in rows:
        coef.extend(a)
        var.extend(x)
        rhs.append(c)
        ptr.append(len(coef))
    f32 = lambda v: np.asarray(v, dtype=np.float32)
    return FModel(f32(lb), f32(ub), np.asarray(ptr, dtype=np.int32), f32(coef),
                  np.asarray(var, dtype=np.int32), f32(rhs), meta)


def _unit(rng: SplitMix64) -> float:
    """Uniform in [0, 1) with 24 random bits (exactly a float32)."""
    return (rng.next_u64() >> 40) / float(1 << 24)


def float_csp(seed: int, nvars: int = 8, dom: float = 20.0, nprec: int = 12) -> FModel:
    """The tiny CSP over the reals: `nvars` variables in [0, dom],
    `nprec` precedences x_u + d <= x_v (d uniform in [1, 5]) along a random
    topological order, and one row sum_i a_i x_i <= c with a_i uniform in
    [1, 4] and c = 60% of the largest possible sum."""
    rng = stream(CFG_FLOAT_CSP, seed)
    perm = list(range(nvars))
    rng.shuffle(perm)
    pairs = [(p, q) for p in range(nvars) for q in range(p + 1, nvars)]
    rng.shuffle(pairs)
    rows = []
    for (p, q) in pairs[:nprec]:
        d = _f32(1.0 + 4.0 * _unit(rng))
        rows.append(([1.0, -1.0], [perm[p], perm[q]], -d))
    a = [_f32(1.0 + 3.0 * _unit(rng)) for _ in range(nvars)]
    c = _f32(0.6 * dom * sum(a))
    rows.append((a, list(range(nvars)), c))
    return _fmodel([0.0] * nvars, [dom] * nvars, rows,
                   dict(kind="float_csp", seed=seed, dom=dom))


def float_network(n: int, seed: int, rows_per_var: int = 2, kmax: int = 6,
                  dom: float = 100.0) -> FModel:
    """A sparse system over the reals: n variables in [-dom, dom] and
    rows_per_var * n rows of 2..kmax distinct variables with coefficients
    uniform in +-[0.25, 4] and a right-hand side that a random point of the
    box satisfies with a slack uniform in [0, dom / 4] (so the root is not
    failed, and propagation tightens the box)."""
    rng = stream(CFG_FLOAT_NET, seed)
    pt = [_f32(dom * (2.0 * _unit(rng) - 1.0) * 0.5) for _ in range(n)]
    rows = []
    for _ in range(rows_per_var * n):
        k = rng.uniform(2, kmax)
        xs = set()
        while len(xs) < k:
            xs.add(rng.below(n))
        xs = sorted(xs)
        a = []
        for _x in xs:
            mag = 0.25 + 3.75 * _unit(rng)
            a.append(_f32(mag if rng.below(2) else -mag))
        val = sum(ai * pt[x] for ai, x in zip(a, xs))
        rows.append((a, xs, _f32(val + dom / 4.0 * _unit(rng))))
    return _fmodel([-dom] * n, [dom] * n, rows, dict(kind="float_network", n=n, seed=seed))


# magnitudes for float_extreme: subnormal, tiny, ordinary, huge and the top
# of the float32 range
_EXT_COEF = (1.4e-45, 3e-39, 1e-30, 0.5, 1.0, 3.0, 7e5, 1e30, 3.4e38)
_EXT_BOUND = (-3.4e38, -1e30, -1e5, -1.0, -1e-40, 0.0, 1e-40, 1.0, 1e5, 1e30, 3.4e38)
_EXT_SLACK = (0.0, 1e-42, 1e-20, 1.0, 1e10, 1e30)


def float_extreme(seed: int, n: int = 30, nrows: int = 50, kmax: int = 10) -> FModel:
    """A small system over the reals whose bounds, coefficients and
    right-hand sides span the float32 range, from subnormals to 3.4e38, so
    that products and sums overflow, underflow and cancel: n variables with
    bounds drawn from a fixed ladder of magnitudes, up to nrows rows of
    1..kmax distinct variables, each row's right-hand side the float at or
    above what a random point of the box gives it plus a slack (rows whose
    right-hand side would leave the float range are dropped)."""
    rng = stream(CFG_FLOAT_EXTREME, seed)
    pick = lambda xs: xs[rng.below(len(xs))]
    lb, ub, pt = [], [], []
    for _ in range(n):
        a, b = sorted((pick(_EXT_BOUND), pick(_EXT_BOUND)))
        lb.append(a)
        ub.append(b)
        pt.append(_f32(a + (b - a) * _unit(rng)))
    rows = []
    for _ in range(nrows):
        k = rng.uniform(1, kmax)
        xs = set()
        while len(xs) < k:
            xs.add(rng.below(n))
        xs = sorted(xs)
        a = [_f32(pick(_EXT_COEF) * (1.0 if rng.below(2) else -1.0)) for _ in xs]
        val = sum(ai * pt[x] for ai, x in zip(a, xs))
        c = val + abs(val) * pick((0.0, 1e-6, 0.5)) + pick(_EXT_SLACK)
        if not abs(c) < 3.4e38:
            continue
        cf = np.float32(c)
        if float(cf) < c:
            cf = np.nextafter(cf, np.float32(np.inf))
        rows.append((a, xs, float(cf)))
    return _fmodel(lb, ub, rows, dict(kind="float_extreme", seed=seed))
