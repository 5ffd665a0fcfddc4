"""A small PCCP front-end: programs built from tells, asks, reified
difference constraints and disjunctions over interval variables (§2), compiled
to the guarded normal form the library runs (§3: a program becomes a parallel
composition of guarded commands).

Constructs and what they compile to (every one lands on the library's two
constraint forms, the linear row and the reified overlap item):

  tell(sum a x <= c)          one linear row
  iff(b, x - y <= c)          b <=> (x - y <= c): a shifted copy x' = x - c
                              (two difference rows) and one reified item
                              (b, x', y, D) with D past the span of y - x', so
                              that its second conjunct is always entailed
  implies(b, sum a x <= c)    ask(b) -> tell(row): the row with b weighted by a
                              constant M that makes it void while b = 0
                              (sum a x + M b <= c + M); with neg(b) for
                              "when b is false"
  neg(b)                      a Boolean b' with b + b' = 1 (two rows)
  disj(x - y <= c, u - v <= d)
                              b <=> (x - y <= c) and neg(b) -> (u - v <= d)
  ask(x - y <= c, row)        a fresh b with iff(b, x - y <= c), then
                              implies(b, row): the row is told once the
                              guard is entailed (§2 ask; interval entailment
                              decides b)

Constructs on the library's guarded-command kind (§3 guarded normal form:
a set of commands {g_1..g_n} => x <- f run in parallel; the gnf function of
§3 lifts nested asks by duplicating their guards):

  when(guards, sum a x <= c)  {guards} => one command per term: the term's
                              bound told from the other terms' bounds
                              (guards are bound tests (y, ">=", c) or
                              (y, "<=", c), i.e. entailed(y >= c) etc.)
  view(sum a x)               an auxiliary t with t <- sum a x on both
                              bounds (two unguarded commands): lb(t) and
                              ub(t) are the least and greatest value of the
                              sum over the box, so entailed(sum a x <= c) is
                              ub(t) <= c and entailed(not sum a x <= c) is
                              lb(t) >= c + 1 (§2 entailment of a linear sum)
  ask_row(guard row, body row)
                              if entailed(guard) then tell(body)
  iff_row(b, row)             b <=> row, §2's four processes for phi <=> psi:
                              entailed(row) -> b; entailed(b) -> row;
                              entailed(not row) -> not b; entailed(not b) ->
                              not row
  disj_rows(row1, row2)       entailed(not row1) -> row2 and entailed(not
                              row2) -> row1

The program keeps its own variables first (in creation order) and appends
the auxiliary ones; `decision` defaults to the program's own variables.
"""
from __future__ import annotations

from .instances import MODE_ENUMERATE, MODE_MINIMIZE, Model, _Builder

_INT16 = 32767


class Program:
    def __init__(self):
        self._lo: list[int] = []
        self._hi: list[int] = []
        self._rows: list[tuple[list[int], list[int], int]] = []
        self._reif: list[tuple[int, int, int, int]] = []
        self._cmds: list[tuple] = []
        self._own: list[int] = []
        self._aux_from = None

    # ---- variables
    def var(self, lo: int, hi: int) -> int:
        """A program variable with the interval [lo, hi]."""
        if lo > hi:
            raise ValueError("empty interval")
        if self._aux_from is not None:
            raise ValueError("program variables must be created before any construct that adds auxiliaries")
        self._lo.append(int(lo))
        self._hi.append(int(hi))
        self._own.append(len(self._lo) - 1)
        return len(self._lo) - 1

    def boolean(self) -> int:
        return self.var(0, 1)

    def _aux(self, lo: int, hi: int) -> int:
        if self._aux_from is None:
            self._aux_from = len(self._lo)
        self._lo.append(int(lo))
        self._hi.append(int(hi))
        return len(self._lo) - 1

    def _bool(self, b: int):
        if not (self._lo[b] >= 0 and self._hi[b] <= 1):
            raise ValueError(f"variable {b} is not Boolean")

    # ---- constructs
    def tell(self, coefs, vars_, c: int):
        """tell(sum coefs[i] * vars_[i] <= c)."""
        coefs, vars_ = [int(a) for a in coefs], [int(v) for v in vars_]
        if len(coefs) != len(vars_) or len(set(vars_)) != len(vars_):
            raise ValueError("a row needs one coefficient per distinct variable")
        self._rows.append((coefs, vars_, int(c)))

    def iff(self, b: int, x: int, y: int, c: int):
        """b <=> (x - y <= c)."""
        self._bool(b)
        xs = self._aux(self._lo[x] - c, self._hi[x] - c)        # xs = x - c
        self.tell([1, -1], [xs, x], -c)
        self.tell([-1, 1], [xs, x], c)
        d = self._hi[y] - self._lo[xs] + 1
        if d < 1:
            d = 1
        if d > _INT16:
            raise ValueError("domains too wide for a reified difference (span over 32766)")
        self._reif.append((b, xs, y, d))

    def neg(self, b: int) -> int:
        """A Boolean equal to 1 - b."""
        self._bool(b)
        nb = self._aux(0, 1)
        self.tell([1, 1], [b, nb], 1)
        self.tell([-1, -1], [b, nb], -1)
        return nb

    def implies(self, b: int, coefs, vars_, c: int):
        """ask(b = 1) -> tell(sum coefs * vars_ <= c)."""
        self._bool(b)
        coefs, vars_ = [int(a) for a in coefs], [int(v) for v in vars_]
        # the largest value the row's left side can take, so that with b = 0
        # the row is entailed
        top = sum(a * (self._hi[v] if a > 0 else self._lo[v]) for a, v in zip(coefs, vars_))
        m = max(0, top - int(c))
        if m > _INT16:
            raise ValueError("domains too wide for an implication (big-M over int16)")
        self.tell(coefs + [m], vars_ + [b], int(c) + m)

    def disj(self, x: int, y: int, c: int, u: int, v: int, d: int) -> int:
        """(x - y <= c) or (u - v <= d); returns the Boolean of the first."""
        b = self._aux(0, 1)
        self.iff(b, x, y, c)
        self.implies(self.neg(b), [1, -1], [u, v], d)
        return b

    def ask(self, x: int, y: int, c: int, coefs, vars_, rhs: int) -> int:
        """ask(x - y <= c) -> tell(sum coefs * vars_ <= rhs); returns the
        guard's Boolean."""
        b = self._aux(0, 1)
        self.iff(b, x, y, c)
        self.implies(b, coefs, vars_, rhs)
        return b

    # ---- guarded commands
    @staticmethod
    def _guards(guards):
        out = []
        for y, op, c in guards:
            if op not in (">=", "<="):
                raise ValueError("a guard is (var, '>=' or '<=', constant)")
            out.append((int(y), 0 if op == ">=" else 1, int(c)))
        return out

    def _check_row(self, coefs, vars_):
        coefs, vars_ = [int(a) for a in coefs], [int(v) for v in vars_]
        if len(coefs) != len(vars_) or len(set(vars_)) != len(vars_) or 0 in coefs:
            raise ValueError("a row needs one nonzero coefficient per distinct variable")
        return coefs, vars_

    def when(self, guards, coefs, vars_, c: int):
        """{guards} => tell(sum coefs * vars_ <= c), one command per term:
        a_i > 0: ub(x_i) <= floor((c - sum_{j != i} a_j x_j) / a_i);
        a_i < 0: lb(x_i) >= ceil((sum_{j != i} a_j x_j - c) / -a_i)."""
        g = self._guards(guards)
        coefs, vars_ = self._check_row(coefs, vars_)
        for i, (a, x) in enumerate(zip(coefs, vars_)):
            rest = [(aj, xj) for j, (aj, xj) in enumerate(zip(coefs, vars_)) if j != i]
            if a > 0:
                self._cmds.append((g, x, 1, int(c), a, [(-aj, xj) for aj, xj in rest]))
            else:
                self._cmds.append((g, x, 0, -int(c), -a, rest))

    def view(self, coefs, vars_) -> int:
        """An auxiliary t whose bounds are the least and greatest value of
        sum coefs * vars_ over the box (two unguarded commands)."""
        coefs, vars_ = self._check_row(coefs, vars_)
        lo = sum(a * (self._lo[v] if a > 0 else self._hi[v]) for a, v in zip(coefs, vars_))
        hi = sum(a * (self._hi[v] if a > 0 else self._lo[v]) for a, v in zip(coefs, vars_))
        t = self._aux(lo, hi)
        terms = list(zip(coefs, vars_))
        self._cmds.append(([], t, 0, 0, 1, terms))      # lb(t) >= sum of least terms
        self._cmds.append(([], t, 1, 0, 1, terms))      # ub(t) <= sum of greatest terms
        return t

    def ask_row(self, gcoefs, gvars, gc: int, coefs, vars_, c: int, guards=()):
        """if entailed(sum gcoefs * gvars <= gc) then tell(sum coefs * vars_ <= c)."""
        t = self.view(gcoefs, gvars)
        self.when(list(guards) + [(t, "<=", int(gc))], coefs, vars_, c)
        return t

    def iff_row(self, b: int, coefs, vars_, c: int):
        """b <=> (sum coefs * vars_ <= c)."""
        self._bool(b)
        coefs, vars_ = self._check_row(coefs, vars_)
        t = self.view(coefs, vars_)
        self._cmds.append(([(t, 1, int(c))], b, 0, 1, 1, []))     # entailed(row) -> lb(b) >= 1
        self._cmds.append(([(t, 0, int(c) + 1)], b, 1, 0, 1, []))  # entailed(not row) -> ub(b) <= 0
        self.when([(b, ">=", 1)], coefs, vars_, c)                # entailed(b) -> row
        self.when([(b, "<=", 0)], [-a for a in coefs], vars_, -int(c) - 1)  # entailed(not b) -> not row
        return t

    def disj_rows(self, c1, v1, r1: int, c2, v2, r2: int):
        """(sum c1 * v1 <= r1) or (sum c2 * v2 <= r2)."""
        t1 = self.view(c1, v1)
        t2 = self.view(c2, v2)
        self.when([(t1, ">=", int(r1) + 1)], c2, v2, r2)
        self.when([(t2, ">=", int(r2) + 1)], c1, v1, r1)
        return t1, t2

    # ---- compile
    def compile(self, decision=None, objective: int = -1, meta: dict | None = None) -> Model:
        bld = _Builder()
        for lo, hi in zip(self._lo, self._hi):
            bld.add_vars(1, lo, hi)
        for coefs, vars_, c in self._rows:
            bld.add_row(coefs, vars_, c)
        for it in self._reif:
            bld.add_reif(*it)
        for g, x, side, k, div, terms in self._cmds:
            bld.add_cmd(g, x, side, k, div, terms)
        dec = list(self._own) if decision is None else [int(v) for v in decision]
        mode = MODE_MINIMIZE if objective >= 0 else MODE_ENUMERATE
        return bld.finish(dec, objective, mode, dict(meta or {}, kind="pccp_program"))
