"""The remaining workload shapes through the C-ABI:
  - 120 tasks, one instance (about 14.5k variables, 15k propagators):
    single-workgroup search parity with the oracle on a node-limited prefix;
    whole-GPU searches are sound and input-order branching finds a schedule;
  - a mixed batch of 30-, 60- and 90-task instances in one persistent launch:
    every incumbent is feasible (checked instant by instant on the raw data),
    proven optima agree with the same instances searched one per launch, and
    the batch agrees with the same instances in a different order;
  - the batch of sixteen 30-task instances in the launch shape the node-rate
    measurement uses: the oracle's prefix on one workgroup, and sound
    incumbents at full size over the whole GPU."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2207_12116_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_12116_amd import pccp
    pccp.lib()
    return pccp


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_120_tasks_prefix_parity(P):
    model = I.rcpsp(120, 0)
    ref = O.solve(model, node_limit=150)
    s = P.Solver(model, num_wgs=1)
    say("120 tasks prefix")
    assert s.solve(node_limit=150, time_limit=120) == P.OUT_LIMIT
    st = s.stats()
    assert (st["nodes"], st["fails"], st["solutions"], st["best"], st["max_depth"]) == \
        (ref["nodes"], ref["fails"], ref["solutions"], ref["best"], ref["max_depth"])


DEEP = [(120, 1, dict(dep=2)), (120, 1, dict(dep=1)), (60, 1, dict(live=1)), (60, 2, dict(live=1)),
        (60, 1, dict(dep=1))]


@pytest.mark.parametrize("n,seed,mode", DEEP, ids=["120-tables", "120-dep", "60-lists", "60b-lists",
                                                   "60-dep"])
def test_deep_paths_prefix_parity(P, n, seed, mode):
    """Input-order branching dives hundreds of decisions deep (about a
    thousand at 120 tasks, about 400 at 60): a single-workgroup prefix whose
    path runs far past the decision levels kept in LDS (the rest live in
    global memory) gives the oracle's counters, depth included.  The item
    lists of the live mode share the control block with the stack's
    deepest-level word, so that mode is covered here too."""
    model = I.rcpsp(n, seed)
    ref = O.solve(model, branching=O.INPUT_ORDER, node_limit=1500)
    s = P.Solver(model, num_wgs=1, max_depth=4096, **mode)
    s.set_branching(P.BRANCH_INPUT_ORDER)
    say("deep prefix", n, seed, mode, ref["max_depth"])
    assert s.solve(node_limit=1500, time_limit=120) == P.OUT_LIMIT
    st = s.stats()
    assert st["live"] == (mode.get("live") == 1) and st["dep"] == (mode.get("dep") == 1)
    assert ref["max_depth"] > 300
    assert (st["nodes"], st["fails"], st["solutions"], st["best"], st["max_depth"]) == \
        (ref["nodes"], ref["fails"], ref["solutions"], ref["best"], ref["max_depth"])


def test_120_tasks_whole_gpu_incumbent_feasible(P):
    """First-fail on 120 tasks thrashes deep in the tree (the oracle finds no
    schedule in its first 20k nodes either), so its run is only checked for
    soundness; branching in input order (tasks are numbered along the
    precedence order, so x = lb places them one by one) must find a schedule."""
    model = I.rcpsp(120, 1)
    st, lb, ub, _ = O.propagate(model)
    for br in (P.BRANCH_FIRST_FAIL, P.BRANCH_INPUT_ORDER):
        # input order walks each start time up one value per right branch:
        # its paths run about a thousand decisions deep
        s = P.Solver(model, max_depth=4096 if br == P.BRANCH_INPUT_ORDER else 0)
        s.set_branching(br)
        out = s.solve(time_limit=3.0)
        obj, vals = s.best()
        say("120 tasks", br, P.OUTCOME_NAMES[out], obj, s.stats()["nodes"])
        assert out in (P.OUT_LIMIT, P.OUT_OPTIMAL)
        assert s.stats()["nodes"] > 0
        if br == P.BRANCH_INPUT_ORDER:
            assert obj is not None
        if obj is not None:
            ok, ms = O.check_schedule(model.meta, vals)
            assert ok and ms == obj
            assert obj >= lb[model.objective]          # never below the root bound


def test_mixed_batch(P):
    seeds = list(range(12))
    models = [I.rcpsp(I.batch_sizes(s), s) for s in seeds]
    assert sorted({m.meta["n"] for m in models}) == [30, 60, 90]
    solvers = [P.Solver(m) for m in models]
    say("mixed batch", len(models))
    outs = P.batch_solve(solvers, P.MINIMIZE, time_limit=4.0)
    for m, s, o in zip(models, solvers, outs):
        obj, vals = s.best()
        if obj is None:
            continue
        ok, ms = O.check_schedule(m.meta, vals)
        assert ok and ms == obj, m.meta["seed"]
    # same instances in reverse order: proven optima must agree
    rsolvers = [P.Solver(m) for m in models[::-1]]
    routs = P.batch_solve(rsolvers, P.MINIMIZE, time_limit=4.0)[::-1]
    rsolvers = rsolvers[::-1]
    for a, b, oa, ob in zip(solvers, rsolvers, outs, routs):
        if oa == P.OUT_OPTIMAL and ob == P.OUT_OPTIMAL:
            assert a.best()[0] == b.best()[0]


def test_mixed_batch_small_proven(P):
    """A batch the GPU proves completely: every optimum equals the oracle's."""
    models = [I.rcpsp_model(*I.rcpsp_data(n, s)[:4]) for n, s in
              [(8, 0), (10, 2), (12, 4), (9, 1), (11, 3), (10, 4), (12, 0), (8, 3)]]
    refs = [O.solve(m, node_limit=400000) for m in models]
    solvers = [P.Solver(m) for m in models]
    outs = P.batch_solve(solvers, P.MINIMIZE, time_limit=30)
    for m, s, o, r in zip(models, solvers, outs, refs):
        assert o == P.OUT_OPTIMAL
        if r["outcome"] == O.OUT_OPTIMAL:
            assert s.best()[0] == r["best"]
        ok, ms = O.check_schedule(m.meta, s.best()[1])
        assert ok and ms == s.best()[0]


# the batch of sixteen 30-task instances (seeds 0-15) in the launch shape
# the node-rate measurement settles on: workgroups of 128 threads, tables
# and subtree roots in HBM, the high-occupancy build, dependency-driven sweeps
HEADLINE = dict(wg_size=128, desc_lds=2, root_lds=2, occupancy=1, dep=1)


def test_headline_shape_single_wg_prefix(P):
    """The same kernel variant on one workgroup: the oracle's depth-first
    prefix, every counter equal."""
    for seed, limit in ((0, 2500), (7, 2000), (15, 2000)):
        m = I.rcpsp(30, seed)
        ref = O.solve(m, node_limit=limit)
        s = P.Solver(m, config=P.Config(num_wgs=1, **HEADLINE))
        out = s.solve(node_limit=limit, time_limit=60)
        st = s.stats()
        say("headline shape 1wg", seed, st["nodes"], ref["nodes"])
        assert out == P.OUT_LIMIT and ref["outcome"] == O.OUT_LIMIT
        assert (st["block"], st["occupancy"], st["dep"]) == (128, 1, 1)
        assert (st["nodes"], st["fails"], st["solutions"], st["best"], st["max_depth"]) == \
            (ref["nodes"], ref["fails"], ref["solutions"], ref["best"], ref["max_depth"])


def test_headline_batch_full_size_sound(P):
    """The whole batch at its full size in that shape (a persistent launch
    over the whole GPU): each incumbent is a feasible schedule on the raw
    data, with the makespan the kernel reports, never below the oracle's root
    bound; the counters are consistent; a second launch of the same solvers
    starts afresh and is just as sound."""
    models = [I.rcpsp(30, s) for s in range(16)]
    roots = [O.propagate(m) for m in models]
    cfg = P.Config(**HEADLINE)
    solvers = [P.Solver(m, config=cfg) for m in models]
    for rep in range(2):
        outs = P.batch_solve(solvers, P.MINIMIZE, config=cfg, time_limit=2.0)
        st0 = solvers[0].stats()
        say("headline batch", rep, st0["grid"], st0["block"],
            sum(s.stats()["nodes"] for s in solvers))
        assert st0["block"] == 128 and st0["grid"] >= 256 and st0["dep"] == 1
        found = 0
        for m, s, o, r in zip(models, solvers, outs, roots):
            st = s.stats()
            assert o in (P.OUT_LIMIT, P.OUT_OPTIMAL)
            assert 0 < st["nodes"] and st["fails"] <= st["nodes"]
            # dependency-driven sweeps run a fraction of the tables per node
            assert st["prop_linear2"] + st["prop_reified"] > 0
            obj, vals = s.best()
            if obj is None:
                continue
            found += 1
            ok, ms = O.check_schedule(m.meta, vals)
            assert ok and ms == obj == st["best"], m.meta["seed"]
            assert obj >= r[1][m.objective]
        assert found >= 8
