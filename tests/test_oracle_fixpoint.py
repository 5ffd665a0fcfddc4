"""The oracle's propagation loop against the paper's theorems and closed
forms:
  - §3, Theorem 2: fix is a closure operator (extensive, monotone,
    idempotent) with a unique least fixed point;
  - §3, Proposition 3 and Theorem 6: sequential, parallel (Jacobi) and any
    fair schedule reach the same fixed point; one sequential pass is at least
    as strong as one parallel pass;
  - critical-path closed form on precedence-only models;
  - soundness: no solution is ever pruned (brute force)."""
import random

import numpy as np
import pytest

import oracle as O
from paper_2207_12116_amd import instances as I
from tests.models import random_subbox

SCHEDS = [(O.SCHED_GS, 0), (O.SCHED_JACOBI, 0), (O.SCHED_REVERSE, 0),
          (O.SCHED_PERM, 1), (O.SCHED_PERM, 2), (O.SCHED_PERM, 3),
          (O.SCHED_SELECT, 4), (O.SCHED_SELECT, 5)]


def leq(lb1, ub1, lb2, ub2):
    """Store order of IZ^n: (lb1,ub1) <= (lb2,ub2) iff every interval of the
    second is inside the first."""
    return bool(np.all(lb1 <= lb2) and np.all(ub1 >= ub2))


def models_small():
    return [("csp0", I.tiny_csp(0)), ("csp3", I.tiny_csp(3)),
            ("rcpsp6", I.tiny_rcpsp(6, 1)), ("rcpsp30", I.rcpsp(30, 2))]


@pytest.mark.parametrize("name,model", models_small(), ids=lambda x: x if isinstance(x, str) else "")
def test_schedule_independence(name, model):
    rng = random.Random(hash(name) & 0xffff)
    om = O.OracleModel(model)
    boxes = [(model.lb, model.ub)] + [random_subbox(model, rng) for _ in range(12)]
    for lb0, ub0 in boxes:
        ref = O.propagate(om, lb0, ub0, O.SCHED_GS)
        for sched, seed in SCHEDS[1:]:
            got = O.propagate(om, lb0, ub0, sched, seed)
            assert got[0] == ref[0], (name, sched, seed)
            if ref[0] == O.FIXPOINT:
                assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])


@pytest.mark.parametrize("name,model", models_small(), ids=lambda x: x if isinstance(x, str) else "")
def test_closure_operator(name, model):
    rng = random.Random(1 + (hash(name) & 0xffff))
    om = O.OracleModel(model)
    for _ in range(15):
        lb0, ub0 = random_subbox(model, rng)
        st, lb, ub, _ = O.propagate(om, lb0, ub0)
        if st == O.FAILED:
            continue
        assert leq(lb0, ub0, lb, ub)                       # extensive
        st2, lb2, ub2, sw = O.propagate(om, lb, ub)        # idempotent
        assert st2 == O.FIXPOINT and sw == 1
        assert np.array_equal(lb, lb2) and np.array_equal(ub, ub2)
        # monotone: a stronger input gives a stronger (or failed) output
        lb1, ub1 = random_subbox(model, rng)
        lb1 = np.maximum(lb1, lb0)
        ub1 = np.minimum(ub1, ub0)
        st3, lb3, ub3, _ = O.propagate(om, lb1, ub1)
        if st3 == O.FIXPOINT:
            assert leq(lb, ub, lb3, ub3)


@pytest.mark.parametrize("name,model", models_small(), ids=lambda x: x if isinstance(x, str) else "")
def test_sequential_pass_dominates_parallel_pass(name, model):
    """§3 (after Proposition 3): one sequential pass over all processes is at
    least as strong as one parallel pass."""
    rng = random.Random(2 + (hash(name) & 0xffff))
    om = O.OracleModel(model)
    for _ in range(15):
        lb0, ub0 = random_subbox(model, rng)
        sj, ljb, ujb = O.jacobi_step(om, lb0, ub0)
        sg, lgb, ugb = O.gs_step(om, lb0, ub0)
        if sg == O.FAILED:
            continue
        assert sj != O.FAILED
        assert leq(ljb, ujb, lgb, ugb)


def test_fixpoint_is_least():
    """Jacobi iteration from the initial box (the Kleene sequence of the
    parallel denotation D(P), §3) climbs to the same point: the least fixed
    point above the box."""
    for model in [I.tiny_csp(1), I.tiny_rcpsp(5, 2), I.rcpsp(30, 3)]:
        lb, ub = model.lb.copy(), model.ub.copy()
        for _ in range(10000):
            st, lb, ub = O.jacobi_step(model, lb, ub)
            if st != 2:
                break
        ref = O.propagate(model)
        assert st == ref[0]
        if st == O.FIXPOINT:
            assert np.array_equal(lb, ref[1]) and np.array_equal(ub, ref[2])


def _cpm(model):
    """Critical-path method on a precedence-only model (independent closed
    form): earliest starts forward in topological order, latest starts
    backward from the horizon."""
    meta = model.meta
    n, h, dur = meta["n"], meta["horizon"], meta["durations"]
    succ = [[] for _ in range(n)]
    pred = [[] for _ in range(n)]
    for i, j in meta["edges"]:
        succ[i].append(j)
        pred[j].append(i)
    es = [0] * n
    for j in range(n):                       # edges go i < j: index order is topological
        for i in pred[j]:
            es[j] = max(es[j], es[i] + dur[i])
    ls = [h - dur[i] for i in range(n)]      # every task ends by m <= h
    for i in reversed(range(n)):
        for j in succ[i]:
            ls[i] = min(ls[i], ls[j] - dur[i])
    cp = max(es[i] + dur[i] for i in range(n))
    return es, ls, cp


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("n", [10, 30, 120])
def test_precedence_fixpoint_is_critical_path(n, seed):
    model = I.precedence_only(n, seed)
    es, ls, cp = _cpm(model)
    st, lb, ub, _ = O.propagate(model)
    assert st == O.FIXPOINT
    assert lb[:n].tolist() == es
    assert ub[:n].tolist() == ls
    assert lb[n] == cp and ub[n] == model.meta["horizon"]


@pytest.mark.parametrize("seed", [0, 2, 5])
def test_root_fixpoint_keeps_every_solution(seed):
    """Soundness (§4, Theorem 8 at the level of the oracle): every point that
    satisfies the constraints survives propagation.  Checked against brute
    force on a smaller domain of the tiny CSP family."""
    model = I.tiny_csp(seed, dom=12)
    n, h, sols = O.brute_points(model, cap=10**6)
    assert n == len(sols)
    st, lb, ub, _ = O.propagate(model)
    if n == 0:
        return
    assert st == O.FIXPOINT
    assert np.all(sols.min(axis=0) >= lb) and np.all(sols.max(axis=0) <= ub)


def test_cycle_and_empty_box_fail():
    from tests.models import make_model
    cyc = make_model([(0, 1000), (0, 1000)],
                     [([1, -1], [0, 1], -1), ([-1, 1], [0, 1], -1)])
    for sched, seed in SCHEDS:
        assert O.propagate(cyc, sched=sched, seed=seed)[0] == O.FAILED
    # reified cycle: b forced true and the two disjuncts contradict
    m = make_model([(1, 1), (0, 50), (0, 50)],
                   [([1, -1], [2, 1], -1)], [(0, 1, 2, 3)])
    assert O.propagate(m)[0] == O.FAILED
    empty = make_model([(0, 5), (4, 3)], [([1, 1], [0, 1], 10)])
    assert O.propagate(empty)[0] == O.FAILED


def test_validation_rejects_bad_models():
    from tests.models import make_model
    assert O.validate(make_model([(0, 1)], [([1], [3], 0)])) == -2       # bad var
    assert O.validate(make_model([(0, 1), (0, 1)], [([1, 1], [0, 0], 0)])) == -2  # dup
    assert O.validate(make_model([(0, 1)], [([0], [0], 0)])) == -2       # zero coef
    assert O.validate(make_model([(0, 2**30)], [([4], [0], 0)])) == -3   # overflow
    assert O.validate(make_model([(0, 1)], [], [(0, 0, 5, 1)])) == -2    # bad reif var
    assert O.validate(I.rcpsp(30, 0)) == 0
