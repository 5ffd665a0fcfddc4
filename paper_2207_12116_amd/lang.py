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

    # ---- compile
    def compile(self, decision=None, objective: int = -1, meta: dict | None = None) -> Model:
        bld = _Builder()
        for lo, hi in zip(self._lo, self._hi):
            bld.add_vars(1, lo, hi)
        for coefs, vars_, c in self._rows:
            bld.add_row(coefs, vars_, c)
        for it in self._reif:
            bld.add_reif(*it)
        dec = list(self._own) if decision is None else [int(v) for v in decision]
        mode = MODE_MINIMIZE if objective >= 0 else MODE_ENUMERATE
        return bld.finish(dec, objective, mode, dict(meta or {}, kind="pccp_program"))
