"""The PCCP front-end (paper_2207_12116_amd.lang) on the CPU.

Pins, each independent of the compilation:
  - tiny random programs (tells, reified differences, implications on b and
    on not-b, disjunctions, asks): the solutions the oracle enumerates on
    the compiled model, projected on the program's own variables, are
    exactly the points of the box where every construct holds, evaluated
    directly in Python;
  - job shops compiled from the front-end: the oracle's optimum equals the
    minimum over every machine's operation order of the longest path in the
    disjunctive graph (tests.models.jobshop_brute)."""
import itertools
import random

import pytest

import oracle as O
from paper_2207_12116_amd import instances as I
from paper_2207_12116_amd.lang import Program
from tests.models import jobshop_brute


def _row(coefs, vars_, c, pt):
    return sum(a * pt[v] for a, v in zip(coefs, vars_)) <= c


def _guard_holds(guards, pt):
    return all((pt[y] >= c) if op == ">=" else (pt[y] <= c) for y, op, c in guards)


def _random_program(rng, guarded=False):
    nx, nb = rng.randint(2, 3), rng.randint(1, 2)
    p = Program()
    xs = [p.var(rng.randint(-2, 0), rng.randint(1, 3)) for _ in range(nx)]
    bs = [p.boolean() for _ in range(nb)]
    cons = []

    def rrow():
        k = rng.randint(1, min(3, nx))
        vs = rng.sample(xs, k)
        return [rng.choice([-2, -1, 1, 2]) for _ in vs], vs, rng.randint(-2, 4)

    kinds = ["tell", "iff", "implies", "implies_not", "disj", "ask"]
    if guarded:
        kinds = ["tell", "when", "ask_row", "iff_row", "disj_rows"]
    for _ in range(rng.randint(2, 4)):
        kind = rng.choice(kinds)
        if kind == "tell":
            a, v, c = rrow()
            p.tell(a, v, c)
            cons.append(lambda pt, a=a, v=v, c=c: _row(a, v, c, pt))
        elif kind == "iff":
            b = rng.choice(bs)
            x, y = rng.sample(xs, 2)
            c = rng.randint(-2, 2)
            p.iff(b, x, y, c)
            cons.append(lambda pt, b=b, x=x, y=y, c=c: pt[b] == int(pt[x] - pt[y] <= c))
        elif kind in ("implies", "implies_not"):
            b = rng.choice(bs)
            a, v, c = rrow()
            if kind == "implies":
                p.implies(b, a, v, c)
                cons.append(lambda pt, b=b, a=a, v=v, c=c: pt[b] == 0 or _row(a, v, c, pt))
            else:
                p.implies(p.neg(b), a, v, c)
                cons.append(lambda pt, b=b, a=a, v=v, c=c: pt[b] == 1 or _row(a, v, c, pt))
        elif kind == "when":
            g = [(rng.choice(xs + bs), rng.choice([">=", "<="]), rng.randint(-1, 2))
                 for _ in range(rng.randint(1, 2))]
            a, v, c = rrow()
            p.when(g, a, v, c)
            cons.append(lambda pt, g=g, a=a, v=v, c=c: not _guard_holds(g, pt) or _row(a, v, c, pt))
        elif kind == "ask_row":
            ga, gv, gc = rrow()
            a, v, c = rrow()
            p.ask_row(ga, gv, gc, a, v, c)
            cons.append(lambda pt, ga=ga, gv=gv, gc=gc, a=a, v=v, c=c:
                        not _row(ga, gv, gc, pt) or _row(a, v, c, pt))
        elif kind == "iff_row":
            b = rng.choice(bs)
            a, v, c = rrow()
            p.iff_row(b, a, v, c)
            cons.append(lambda pt, b=b, a=a, v=v, c=c: pt[b] == int(_row(a, v, c, pt)))
        elif kind == "disj_rows":
            a1, v1, c1 = rrow()
            a2, v2, c2 = rrow()
            p.disj_rows(a1, v1, c1, a2, v2, c2)
            cons.append(lambda pt, a1=a1, v1=v1, c1=c1, a2=a2, v2=v2, c2=c2:
                        _row(a1, v1, c1, pt) or _row(a2, v2, c2, pt))
        elif kind == "disj":
            x, y = rng.sample(xs, 2)
            u, w = rng.sample(xs, 2)
            c, d = rng.randint(-2, 2), rng.randint(-2, 2)
            p.disj(x, y, c, u, w, d)
            cons.append(lambda pt, x=x, y=y, c=c, u=u, w=w, d=d:
                        pt[x] - pt[y] <= c or pt[u] - pt[w] <= d)
        else:
            x, y = rng.sample(xs, 2)
            c = rng.randint(-2, 2)
            a, v, r = rrow()
            p.ask(x, y, c, a, v, r)
            cons.append(lambda pt, x=x, y=y, c=c, a=a, v=v, r=r:
                        pt[x] - pt[y] > c or _row(a, v, r, pt))
    return p, xs + bs, cons


@pytest.mark.parametrize("guarded", [False, True], ids=["rows_reified", "guarded_commands"])
@pytest.mark.parametrize("seed", range(60))
def test_random_programs_solution_sets(seed, guarded):
    """Guarded commands (§3 guarded normal form) are pinned here by their
    meaning: the points the oracle's search keeps are exactly those where
    every construct holds, evaluated directly on the point."""
    rng = random.Random(seed + (1000 if guarded else 0))
    p, own, cons = _random_program(rng, guarded)
    model = p.compile()
    boxes = [range(model.lb[v], model.ub[v] + 1) for v in own]
    want = set()
    for vals in itertools.product(*boxes):
        pt = dict(zip(own, vals))
        if all(f(pt) for f in cons):
            want.add(tuple(vals))
    r = O.solve(model, mode=I.MODE_ENUMERATE, sol_cap=100000)
    got = {tuple(int(x) for x in row) for row in r["solutions_list"]}
    assert r["solutions"] == len(got)
    assert got == want, (seed, sorted(want - got)[:5], sorted(got - want)[:5])


@pytest.mark.parametrize("guarded", [False, True], ids=["reified", "guarded"])
@pytest.mark.parametrize("nj,nm", [(2, 2), (3, 2), (3, 3), (4, 2), (4, 3)])
@pytest.mark.parametrize("seed", range(3))
def test_jobshop_optimum_equals_disjunctive_graph_brute_force(nj, nm, seed, guarded):
    m = I.jobshop(nj, nm, seed, guarded=guarded)
    r = O.solve(m)
    assert r["outcome"] == O.OUT_OPTIMAL
    assert r["best"] == jobshop_brute(m.meta["jobs"])


def test_front_end_rejects_bad_programs():
    p = Program()
    x = p.var(0, 5)
    with pytest.raises(ValueError):
        p.var(3, 2)
    with pytest.raises(ValueError):
        p.iff(x, x, x, 0)                  # x is not Boolean
    b = p.boolean()
    p.neg(b)
    with pytest.raises(ValueError):
        p.var(0, 1)                        # own variables come before auxiliaries
    q = Program()
    u, w, bb = q.var(0, 40000), q.var(0, 40000), q.boolean()
    with pytest.raises(ValueError):
        q.iff(bb, u, w, 0)                 # span past the reified item's int16 d


def test_guarded_program_brute_points():
    """The oracle's independent point checker (orc_brute_points states each
    guarded command as a constraint on complete points) agrees with the
    direct evaluation on random guarded programs."""
    for seed in range(25):
        rng = random.Random(5000 + seed)
        p, own, cons = _random_program(rng, guarded=True)
        model = p.compile()
        # brute force runs over every variable: keep the auxiliaries'
        # boxes (views) as they are, they are determined by the own ones
        n, h, pts = O.brute_points(model, cap=100000)
        boxes = [range(model.lb[v], model.ub[v] + 1) for v in own]
        want = {vals for vals in itertools.product(*boxes)
                if all(f(dict(zip(own, vals))) for f in cons)}
        got = {tuple(int(x) for x in row) for row in pts}
        assert got == want, seed


def test_front_end_guarded_errors():
    p = Program()
    x, y = p.var(0, 5), p.var(0, 5)
    with pytest.raises(ValueError):
        p.when([(x, ">", 1)], [1], [y], 3)        # guards are >= or <=
    with pytest.raises(ValueError):
        p.when([], [1, 0], [x, y], 3)             # zero coefficient
    with pytest.raises(ValueError):
        p.iff_row(x, [1], [y], 2)                 # x is not Boolean
