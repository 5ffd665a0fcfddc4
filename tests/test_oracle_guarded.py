"""Pins of the oracle's general guarded command ({guards} => x <- f, §3
guarded normal form; guards are entailments of bound constraints, §2 ask).

  - hand-worked fixed points, each derived below from the definition;
  - a linear row stated as unguarded commands (one per term, what the
    front-end's `when([], row)` emits) reaches the same fixed point as the
    row kind on random boxes, and the row kind is pinned on its own by the
    bound-consistency hull tests;
  - soundness and tightness against brute force on tiny boxes: the fixed
    point of a single guarded command keeps every point that satisfies it,
    and when its guard is entailed and f has one term, the told bound is
    the exact bound of the points (a one-term tell is bound-consistent).
The meaning of the commands on complete points is pinned in test_lang.py
(random programs against direct evaluation)."""
import itertools
import random

import numpy as np
import pytest

import oracle as O
from paper_2207_12116_amd.lang import Program


def fix(p, lb=None, ub=None):
    m = p.compile()
    st, l, u, _ = O.propagate(m, lb, ub)
    return m, st, l, u


def test_hand_guard_entailed_or_not():
    # x, y in [0, 10], b in [0, 1]; y >= 3; {lb(b) >= 1} => x + y <= 7.
    p = Program()
    x, y, b = p.var(0, 10), p.var(0, 10), p.boolean()
    p.tell([-1], [y], -3)
    p.when([(b, ">=", 1)], [1, 1], [x, y], 7)
    # b not entailed: nothing but y >= 3
    m, st, l, u = fix(p)
    assert st == O.FIXPOINT and (l[x], u[x], l[y], u[y]) == (0, 10, 3, 10)
    # b = 1: ub(x) <= 7 - lb(y) = 4, ub(y) <= 7 - lb(x) = 7
    lb0, ub0 = m.lb.copy(), m.ub.copy()
    lb0[b] = 1
    st, l, u, _ = O.propagate(m, lb0, ub0)
    assert st == O.FIXPOINT and (l[x], u[x], l[y], u[y]) == (0, 4, 3, 7)
    # b = 1 and x >= 5: ub(y) <= 7 - 5 = 2 < lb(y) = 3, failed
    lb0[x] = 5
    st, l, u, _ = O.propagate(m, lb0, ub0)
    assert st == O.FAILED


def test_hand_division_rounding():
    # 2x + 3y <= 20 with y >= 3: ub(x) <= floor((20 - 9) / 2) = 5,
    # ub(y) <= floor((20 - 0) / 3) = 6
    p = Program()
    x, y = p.var(0, 10), p.var(3, 10)
    p.when([], [2, 3], [x, y], 20)
    _, st, l, u = fix(p)
    assert st == O.FIXPOINT and (l[x], u[x], l[y], u[y]) == (0, 5, 3, 6)


def test_hand_negative_coefficient_and_ub_guard():
    # {ub(x) <= 5} => -2y + z <= -3, i.e. y >= (z + 3) / 2 and z <= 2y - 3.
    # z in [4, 9]: lb(y) >= ceil((4 + 3) / 2) = 4; ub(z) <= 2 * 10 - 3 = 17
    # (no change).  With x in [0, 8] the guard is not entailed.
    p = Program()
    x, y, z = p.var(0, 5), p.var(0, 10), p.var(4, 9)
    p.when([(x, "<=", 5)], [-2, 1], [y, z], -3)
    _, st, l, u = fix(p)
    assert st == O.FIXPOINT and (l[y], u[y], l[z], u[z]) == (4, 10, 4, 9)
    q = Program()
    x, y, z = q.var(0, 8), q.var(0, 10), q.var(4, 9)
    q.when([(x, "<=", 5)], [-2, 1], [y, z], -3)
    _, st, l, u = fix(q)
    assert (l[y], u[y]) == (0, 10)
    # the same with y <= 3: lb(y) >= 4 > 3, failed once the guard holds
    r = Program()
    x, y, z = r.var(0, 5), r.var(0, 3), r.var(4, 9)
    r.when([(x, "<=", 5)], [-2, 1], [y, z], -3)
    _, st, _, _ = fix(r)
    assert st == O.FAILED


def test_hand_view_and_iff_row():
    # t = x + y over x in [1, 4], y in [2, 3]: lb(t) = 3, ub(t) = 7.
    # b <=> (x + y <= 7) is entailed true: lb(b) = 1.
    p = Program()
    x, y, b = p.var(1, 4), p.var(2, 3), p.boolean()
    p.iff_row(b, [1, 1], [x, y], 7)
    _, st, l, u = fix(p)
    assert st == O.FIXPOINT and (l[b], u[b]) == (1, 1)
    # b <=> (x + y <= 2) is entailed false (lb(t) = 3 >= 3): ub(b) = 0
    q = Program()
    x, y, b = q.var(1, 4), q.var(2, 3), q.boolean()
    q.iff_row(b, [1, 1], [x, y], 2)
    _, st, l, u = fix(q)
    assert (l[b], u[b]) == (0, 0)
    # b = 1 told: x + y <= 4 gives ub(x) <= 4 - 2 = 2, ub(y) <= 4 - 1 = 3
    r = Program()
    x, y, b = r.var(1, 4), r.var(2, 3), r.var(1, 1)
    r.iff_row(b, [1, 1], [x, y], 4)
    _, st, l, u = fix(r)
    assert (l[x], u[x], l[y], u[y]) == (1, 2, 2, 3)


def _random_row(rng, n, lo, hi):
    p = Program()
    xs = [p.var(lo, hi) for _ in range(n)]
    a = [rng.choice([-3, -2, -1, 1, 2, 3]) for _ in range(n)]
    c = rng.randint(-4, 8)
    return p, xs, a, c


@pytest.mark.parametrize("seed", range(40))
def test_row_as_commands_equals_row_kind(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 4)
    p1, xs, a, c = _random_row(rng, n, -5, 6)
    p1.tell(a, xs, c)
    p2, xs2, _, _ = _random_row(random.Random(seed), n, -5, 6)
    p2.when([], a, xs2, c)
    m1, m2 = p1.compile(), p2.compile()
    assert m2.ncmd == n and m1.ncmd == 0
    for k in range(20):
        lb = np.array([rng.randint(-5, 2) for _ in range(n)], np.int32)
        ub = np.array([rng.randint(int(l), 6) for l in lb], np.int32)
        r1 = O.propagate(m1, lb, ub)
        r2 = O.propagate(m2, lb, ub)
        assert r1[0] == r2[0]
        if r1[0] == O.FIXPOINT:
            assert np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])


@pytest.mark.parametrize("seed", range(30))
def test_single_command_sound_and_exact_on_one_term(seed):
    """{y >= g} => div * x >= k + a * z (or <=): over every sub-box of a
    tiny box, the fixed point keeps every satisfying point; when the guard
    is entailed, the told bound of x is the least (greatest) x of the
    points of the box that satisfy it, or the box fails when none does."""
    rng = random.Random(seed)
    side = rng.randint(0, 1)
    a = rng.choice([-2, -1, 1, 2, 3])
    k, div, g = rng.randint(-3, 3), rng.randint(1, 3), rng.randint(0, 2)
    def build(lx, ux, ly, uy, lz, uz):
        p = Program()
        x, y, z = p.var(lx, ux), p.var(ly, uy), p.var(lz, uz)
        p._cmds.append(([(y, 0, g)], x, side, k, div, [(a, z)]))
        return p, x, y, z
    def sat(px, py, pz):
        if py < g:
            return True
        return div * px >= k + a * pz if side == 0 else div * px <= k + a * pz
    vals = range(-2, 3)
    for lx, ux in itertools.combinations_with_replacement(vals, 2):
        for lz, uz in itertools.combinations_with_replacement(vals, 2):
            for ly, uy in ((0, 2), (g, 2), (g, g)):
                if ly > uy:
                    continue
                p, x, y, z = build(lx, ux, ly, uy, lz, uz)
                _, st, l, u = fix(p)
                pts = [(px, py, pz) for px in range(lx, ux + 1) for py in range(ly, uy + 1)
                       for pz in range(lz, uz + 1) if sat(px, py, pz)]
                if st == O.FAILED:
                    assert not pts
                    continue
                for px, py, pz in pts:
                    assert l[x] <= px <= u[x] and l[y] <= py <= u[y] and l[z] <= pz <= u[z]
                if ly >= g:   # guard entailed: bound of x exact over the points
                    if side == 0:
                        assert l[x] == min(px for px, _, _ in pts)
                    else:
                        assert u[x] == max(px for px, _, _ in pts)
