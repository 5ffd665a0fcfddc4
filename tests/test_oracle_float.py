"""Pins of the oracle's floating-point interval propagation (oracle/fprop.c).

The store is float32 intervals (lb in FInc, ub in FDec, §2 with the IEEE
total order of its footnote); a linear row over the reals tells each term
the bound of §2's linear tell, rounded outward.  What fixes the result
independently of the oracle's code:
  - exact arithmetic (Python fractions): every tell of a single row lies on
    the sound side of the exact real bound and within the rounding error the
    operations can make; on dyadic data, where every operation is exact, the
    result is the exact bound;
  - closed form: on a precedence network with dyadic durations the fixed
    point is the critical-path schedule (earliest and latest starts);
  - soundness: a point that satisfies every row exactly stays inside the
    fixed point; a system with no real solution fails;
  - the lattice laws of §3: the same store under every schedule (Gauss-
    Seidel, Jacobi, random permutations, reversed), extensive, idempotent,
    monotone;
  - a planted mistake (round-to-nearest instead of outward rounding, in a
    restatement of the tell) fails the exact-arithmetic pin.
"""
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2207_12116_amd import instances as I

F = Fraction


def f32(x) -> float:
    return float(np.float32(x))


def ulp(x: float) -> float:
    x = np.float32(abs(x))
    return float(np.spacing(x)) if x != 0 else float(np.spacing(np.float32(0)))


def row_model(a, c, lb, ub):
    return I._fmodel(lb, ub, [(a, list(range(len(a))), c)], {})


def exact_bounds(a, c, lb, ub):
    """Exact real bound of every term of one row: (is_ub, value) per term."""
    out = []
    for t in range(len(a)):
        s = sum(F(a[u]) * F(lb[u] if a[u] > 0 else ub[u]) for u in range(len(a)) if u != t)
        out.append((a[t] > 0, (F(c) - s) / F(a[t])))
    return out


def _random_row(rng, n, dyadic):
    if dyadic:
        a = [rng.choice([-1, 1]) * rng.choice([0.25, 0.5, 1.0, 2.0, 4.0]) for _ in range(n)]
        lb = [rng.randint(-40, 0) / 2 for _ in range(n)]
        ub = [l + rng.randint(0, 40) / 2 for l in lb]
        c = rng.randint(-20, 40) / 4
    else:
        a = [f32(rng.choice([-1, 1]) * rng.uniform(0.1, 7.0)) for _ in range(n)]
        lb = [f32(rng.uniform(-30, 0)) for _ in range(n)]
        ub = [f32(l + rng.uniform(0, 30)) for l in lb]
        c = f32(rng.uniform(-20, 40))
    return a, c, lb, ub


def _tolerance(a, c, lb, ub, t):
    """What rounding can add to term t's bound: each of the n rounded
    operations is off by less than one float32 unit of its result, and the
    partial results are bounded by |c| + sum |m_u|; the division adds one
    unit of the quotient."""
    n = len(a)
    mags = abs(F(c)) + sum(abs(F(a[u]) * F(lb[u] if a[u] > 0 else ub[u])) for u in range(n))
    return (n + 2) * F(2) ** -23 * mags / abs(F(a[t]))


@pytest.mark.parametrize("dyadic", [True, False], ids=["dyadic", "float"])
def test_single_row_against_exact_arithmetic(dyadic):
    rng = random.Random(11 if dyadic else 12)
    nchecked = 0
    for _ in range(300):
        n = rng.randint(1, 5)
        a, c, lb, ub = _random_row(rng, n, dyadic)
        m = row_model(a, c, lb, ub)
        # one Jacobi step from the initial box: each term's tell on its own
        st, glb, gub = O.fjacobi_step(m, m.lb, m.ub)
        for t, (is_ub, exact) in enumerate(exact_bounds(a, c, lb, ub)):
            got = F(float(gub[t] if is_ub else glb[t]))
            old = F(float(ub[t] if is_ub else lb[t]))
            if is_ub:
                want = min(old, exact)
                assert got >= want, (a, c, lb, ub, t)                 # sound
                if exact < old:
                    assert got - exact <= _tolerance(a, c, lb, ub, t) + F(ulp(float(exact)))
                if dyadic:
                    assert got == want
            else:
                want = max(old, exact)
                assert got <= want, (a, c, lb, ub, t)
                if exact > old:
                    assert exact - got <= _tolerance(a, c, lb, ub, t) + F(ulp(float(exact)))
                if dyadic:
                    assert got == want
            nchecked += 1
    assert nchecked > 500


def test_single_row_reaches_its_hull_in_one_sweep():
    """A tell on a term changes only the bound that term's own tell moves,
    never a bound another term of the row reads: after one sweep the store
    is the row's fixed point."""
    rng = random.Random(5)
    for _ in range(200):
        a, c, lb, ub = _random_row(rng, rng.randint(1, 6), False)
        m = row_model(a, c, lb, ub)
        st, glb, gub, sweeps = O.fpropagate(m)
        st1, jlb, jub = O.fjacobi_step(m, m.lb, m.ub)
        if st == O.FIXPOINT:
            assert sweeps <= 2
            assert np.array_equal(glb.view(np.uint32), np.where(jlb == 0, np.float32(-0.0), jlb).view(np.uint32))


def _cpm(n, edges, dur, horizon):
    """Earliest and latest starts by the critical-path method (exact)."""
    es = [F(0)] * n
    order = list(range(n))                 # every edge goes from i to j > i
    for j in order:
        for (i, k) in edges:
            if k == j:
                es[j] = max(es[j], es[i] + F(dur[i]))
    ls = [F(horizon) - F(dur[i]) for i in range(n)]
    for i in reversed(order):
        for (k, j) in edges:
            if k == i:
                ls[i] = min(ls[i], ls[j] - F(dur[i]))
    return es, ls


@pytest.mark.parametrize("seed", range(8))
def test_precedence_network_is_critical_path(seed):
    """x_i + d_i <= x_j along a DAG (i < j), x in [0, H - d]: with dyadic
    durations every operation is exact and the fixed point is the
    critical-path schedule."""
    rng = random.Random(seed)
    n = rng.randint(5, 25)
    dur = [rng.randint(1, 40) / 8 for _ in range(n)]
    edges = []
    for i in range(n - 1):
        for j in rng.sample(range(i + 1, n), min(n - 1 - i, rng.randint(1, 3))):
            edges.append((i, j))
    horizon = sum(dur)
    rows = [([1.0, -1.0], [i, j], -dur[i]) for (i, j) in edges]
    m = I._fmodel([0.0] * n, [horizon - d for d in dur], rows, {})
    st, lb, ub, _ = O.fpropagate(m)
    assert st == O.FIXPOINT
    es, ls = _cpm(n, edges, dur, horizon)
    assert [F(float(x)) for x in lb] == es
    assert [F(float(x)) for x in ub] == ls


def _feasible(model, pt):
    for r in range(model.nrows):
        a0, a1 = model.row_ptr[r], model.row_ptr[r + 1]
        tot = sum(F(float(model.coef[t])) * F(float(pt[model.var[t]])) for t in range(a0, a1))
        if tot > F(float(model.rhs[r])):
            return False
    return True


@pytest.mark.parametrize("seed", range(12))
def test_hidden_solution_stays_inside(seed):
    """float_network builds its rows around a random point of the box; where
    that point satisfies every row exactly, it lies inside the fixed point."""
    import paper_2207_12116_amd.instances as inst
    m = I.float_network(30 + 10 * seed, seed, rows_per_var=3)
    rng = inst.stream(inst.CFG_FLOAT_NET, seed)
    pt = [inst._f32(100.0 * (2.0 * inst._unit(rng) - 1.0) * 0.5) for _ in range(m.nvars)]
    if not _feasible(m, pt):
        pytest.skip("the rounded right-hand side cut the hidden point off")
    st, lb, ub, _ = O.fpropagate(m)
    assert st == O.FIXPOINT
    for v, x in enumerate(pt):
        assert lb[v] <= x <= ub[v], (v, lb[v], x, ub[v])
    assert float((ub - lb).mean()) < 200.0          # and the box did shrink


def test_infeasible_system_fails():
    # x + y <= 1, -x <= -0.75, -y <= -0.5 has no real solution
    m = I._fmodel([0.0, 0.0], [10.0, 10.0],
                  [([1.0, 1.0], [0, 1], 1.0), ([-1.0], [0], -0.75), ([-1.0], [1], -0.5)], {})
    assert O.fpropagate(m)[0] == O.FAILED
    # touching at one point is not empty: x + y <= 1.25 leaves x = 0.75, y = 0.5
    m = I._fmodel([0.0, 0.0], [10.0, 10.0],
                  [([1.0, 1.0], [0, 1], 1.25), ([-1.0], [0], -0.75), ([-1.0], [1], -0.5)], {})
    st, lb, ub, _ = O.fpropagate(m)
    assert st == O.FIXPOINT and list(lb) == [0.75, 0.5] and list(ub) == [0.75, 0.5]


def test_zero_bounds_are_canonical():
    """A lower bound of zero is -0 and an upper bound of zero is +0 (the
    weaker zero of FInc and of FDec), so [0, 0] is not read as empty under
    the total order."""
    m = I._fmodel([0.0, -1.0], [1.0, 0.0], [([1.0, 1.0], [0, 1], 0.0), ([-1.0, -1.0], [0, 1], 0.0)], {})
    st, lb, ub, _ = O.fpropagate(m, lb=np.float32([0.0, -0.0]), ub=np.float32([-0.0, 0.0]))
    assert st == O.FIXPOINT
    assert np.signbit(lb[0]) and not np.signbit(ub[0]) and lb[0] == 0 and ub[0] == 0
    assert lb[1] == 0 and ub[1] == 0


FMODELS = [("csp%d" % s, lambda s=s: I.float_csp(s)) for s in range(6)] + \
          [("net%d" % s, lambda s=s: I.float_network(200, s)) for s in range(4)]


@pytest.mark.parametrize("name,mk", FMODELS, ids=[m[0] for m in FMODELS])
def test_schedules_agree_bit_for_bit(name, mk):
    m = mk()
    ref = O.fpropagate(m)
    for sched, seed in [(O.SCHED_JACOBI, 0), (O.SCHED_REVERSE, 0), (O.SCHED_PERM, 1),
                        (O.SCHED_PERM, 99)]:
        got = O.fpropagate(m, sched=sched, seed=seed)
        assert got[0] == ref[0], (name, sched)
        if ref[0] == O.FIXPOINT:
            assert np.array_equal(got[1].view(np.uint32), ref[1].view(np.uint32)), (name, sched)
            assert np.array_equal(got[2].view(np.uint32), ref[2].view(np.uint32)), (name, sched)


@pytest.mark.parametrize("name,mk", FMODELS, ids=[m[0] for m in FMODELS])
def test_extensive_idempotent_monotone(name, mk):
    m = mk()
    rng = random.Random(len(name))
    st, lb, ub, _ = O.fpropagate(m)
    if st != O.FIXPOINT:
        return
    assert (lb >= m.lb).all() and (ub <= m.ub).all()
    st2, lb2, ub2, sw = O.fpropagate(m, lb, ub)
    assert st2 == O.FIXPOINT and sw == 1
    assert np.array_equal(lb2.view(np.uint32), lb.view(np.uint32))
    for _ in range(10):
        # a sub-box of the root's box: its fixed point is inside the root's
        slb, sub = m.lb.copy(), m.ub.copy()
        for v in range(m.nvars):
            if rng.random() < 0.3:
                x = np.float32(rng.uniform(float(m.lb[v]), float(m.ub[v])))
                if rng.random() < 0.5:
                    slb[v] = x
                else:
                    sub[v] = x
        s3, lb3, ub3, _ = O.fpropagate(m, slb, sub)
        if s3 == O.FIXPOINT:
            assert (lb3 >= lb).all() and (ub3 <= ub).all()


def _tell_rn(a, c, lb, ub, t):
    """A restatement of the tell with a planted mistake: round-to-nearest
    float32 arithmetic instead of outward rounding."""
    s = np.float32(0)
    for u in range(len(a)):
        if u != t:
            s = np.float32(s + np.float32(a[u]) * np.float32(lb[u] if a[u] > 0 else ub[u]))
    return np.float32(np.float32(np.float32(c) - s) / np.float32(a[t]))


def test_planted_round_to_nearest_fails_the_exact_pin():
    rng = random.Random(12)
    caught = False
    for _ in range(300):
        n = rng.randint(1, 5)
        a, c, lb, ub = _random_row(rng, n, False)
        for t, (is_ub, exact) in enumerate(exact_bounds(a, c, lb, ub)):
            got = F(float(_tell_rn(a, c, lb, ub, t)))
            if (is_ub and got < exact) or (not is_ub and got > exact):
                caught = True
    assert caught
