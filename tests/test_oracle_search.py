"""The oracle's search against brute force and hand-worked optima.

  - ENUMERATE (tiny CSP family): the solution set equals the brute-force
    generate-and-test set (count, order-independent hash and, when small,
    the sorted list).
  - MINIMIZE (tiny RCPSP): the optimum equals the brute-force minimum over
    start times checked instant by instant on the raw data (independent of
    the Boolean decomposition), and the returned schedule is feasible.
  - Invariants: the optimum does not depend on the branching rule; it is at
    least the critical-path and energy lower bounds; bounding the objective
    below the optimum makes the model unsatisfiable."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2207_12116_amd import instances as I
from tests.models import make_model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sorted_rows(a):
    a = np.asarray(a)
    return a[np.lexsort(a.T[::-1])] if len(a) else a


@pytest.mark.parametrize("seed,dom", [(0, 10), (1, 10), (2, 12), (3, 12), (4, 14),
                                      (5, 9), (6, 11), (7, 13)])
def test_enumerate_equals_brute_force(seed, dom):
    model = I.tiny_csp(seed, dom=dom)
    n, h, sols = O.brute_points(model, cap=2 * 10**6)
    for br in (O.FIRST_FAIL, O.INPUT_ORDER):
        r = O.solve(model, branching=br, sol_cap=2 * 10**6)
        assert r["outcome"] == O.OUT_ALL
        assert r["solutions"] == n and r["sol_hash"] == h
        if n <= 2 * 10**6:
            assert np.array_equal(_sorted_rows(r["solutions_list"]), _sorted_rows(sols))
        # a node is a propagate call: every node is a leaf, a failure or an
        # inner node with exactly two children
        assert r["nodes"] == 2 * (r["nodes"] - r["fails"] - r["solutions"]) + 1


@pytest.mark.slow
def test_enumerate_full_size_seed():
    """One instance of the tiny CSP at its stated size (8 variables over
    [0, 20]): 21^8 points, generate-and-test with partial-assignment checks."""
    model = I.tiny_csp(0)
    n, h, _ = O.brute_points(model)
    r = O.solve(model)
    assert (r["solutions"], r["sol_hash"]) == (n, h) == (25278142, r["sol_hash"])


def test_hand_searches():
    with open(os.path.join(GOLDEN, "hand_searches.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        if c["mode"] == "enumerate":
            m = make_model(c["boxes"], c["rows"], c["reif"])
            r = O.solve(m, sol_cap=100)
            assert sorted(map(list, r["solutions_list"].tolist())) == c["solutions"]
        else:
            d = c["rcpsp"]
            m = I.rcpsp_model(d["durations"], [tuple(e) for e in d["edges"]],
                              d["demands"], d["capacities"])
            r = O.solve(m)
            assert r["outcome"] == O.OUT_OPTIMAL and r["best"] == c["optimum"], c["name"]


def _lower_bounds(meta):
    n, dur = meta["n"], meta["durations"]
    es = [0] * n
    for i, j in sorted(meta["edges"], key=lambda e: e[1]):
        es[j] = max(es[j], es[i] + dur[i])
    # recompute in topological (index) order to be safe
    es = [0] * n
    for j in range(n):
        for i, jj in meta["edges"]:
            if jj == j:
                es[j] = max(es[j], es[i] + dur[i])
    cp = max(es[i] + dur[i] for i in range(n))
    energy = max(-(-sum(r[i] * dur[i] for i in range(n)) // c)
                 for r, c in zip(meta["demands"], meta["capacities"]))
    return cp, energy


@pytest.mark.parametrize("n,seed", [(3, s) for s in range(6)] + [(4, s) for s in range(6)]
                         + [(5, s) for s in range(5)] + [(6, s) for s in range(4)])
def test_minimize_equals_brute_force(n, seed):
    model = I.tiny_rcpsp(n, seed)
    meta = model.meta
    opt, sched = O.brute_rcpsp(meta)
    assert opt is not None
    ok, ms = O.check_schedule(meta, sched)
    assert ok and ms == opt
    r = O.solve(model)
    assert r["outcome"] == O.OUT_OPTIMAL and r["best"] == opt
    ok, ms = O.check_schedule(meta, r["best_assign"])
    assert ok and ms == opt
    r2 = O.solve(model, branching=O.INPUT_ORDER)
    assert r2["best"] == opt
    cp, energy = _lower_bounds(meta)
    assert opt >= cp and opt >= energy


@pytest.mark.parametrize("seed", range(3))
def test_bound_below_optimum_is_unsat(seed):
    model = I.tiny_rcpsp(5, seed)
    opt = O.solve(model)["best"]
    m = model.objective
    model.ub = model.ub.copy()
    model.ub[m] = opt - 1
    r = O.solve(model)
    assert r["outcome"] == O.OUT_UNSAT and r["best"] is None and r["solutions"] == 0
    model.ub[m] = opt
    r = O.solve(model)
    assert r["outcome"] == O.OUT_OPTIMAL and r["best"] == opt


def test_node_limit():
    model = I.rcpsp(30, 0)
    r = O.solve(model, node_limit=500)
    assert r["outcome"] == O.OUT_LIMIT and r["nodes"] == 500
