"""The search entry point that allocates nothing (pccp_solve_noalloc) against
pccp_solve on the same solvers: identical results on two calls in a row, the
second on a smaller instance, in the sequential order (one workgroup: every
counter is fixed) and over many workgroups (ENUMERATE: the node count,
solution count and hash are fixed; MINIMIZE: the optimum)."""
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


def counts(s):
    st = s.stats()
    return (st["nodes"], st["fails"], st["solutions"], st["sol_hash"], st["best"],
            st["max_depth"], st["outcome"])


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
def test_noalloc_sequential_matches_solve(P, dep):
    # first call: a node-limited prefix of a 30-task search; second call: a
    # smaller instance searched to its optimum
    for model, limit in [(I.rcpsp(30, 3), 3000), (I.tiny_rcpsp(10, 1), 0)]:
        say(f"noalloc sequential dep={dep} nvars={model.nvars} limit={limit}")
        a = P.Solver(model, num_wgs=1, dep=dep)
        b = P.Solver(model, num_wgs=1, dep=dep)
        oa = a.solve(P.MINIMIZE, node_limit=limit, time_limit=60)
        ob = b.solve_noalloc(P.MINIMIZE, node_limit=limit, time_limit=60)
        assert oa == ob
        assert counts(a) == counts(b)
        ba, bb = a.best(), b.best()
        assert ba[0] == bb[0]
        if ba[0] is not None:
            assert np.array_equal(ba[1], bb[1])
        if limit == 0:
            ref = O.solve(model)
            assert oa == P.OUT_OPTIMAL
            st = b.stats()
            assert (st["nodes"], st["fails"], st["solutions"], st["best"]) == \
                (ref["nodes"], ref["fails"], ref["solutions"], ref["best"])


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
def test_noalloc_many_workgroups(P, dep):
    for seed, dom in [(2, 14), (1, 12)]:
        model = I.tiny_csp(seed, dom=dom)
        ref = O.solve(model)
        say(f"noalloc enumerate dep={dep} seed={seed} dom={dom}")
        a = P.Solver(model, num_wgs=64, dep=dep)
        assert a.solve_noalloc(time_limit=60) == P.OUT_ALL
        st = a.stats()
        assert (st["nodes"], st["solutions"], st["sol_hash"]) == \
            (ref["nodes"], ref["solutions"], ref["sol_hash"])
        b = P.Solver(model, num_wgs=64, dep=dep)
        assert b.solve(time_limit=60) == P.OUT_ALL
        sb = b.stats()
        assert (sb["nodes"], sb["solutions"], sb["sol_hash"]) == \
            (st["nodes"], st["solutions"], st["sol_hash"])
    for n, seed in [(14, 2), (9, 0)]:
        model = I.tiny_rcpsp(n, seed)
        ref = O.solve(model)
        say(f"noalloc minimize dep={dep} n={n} seed={seed}")
        a = P.Solver(model, num_wgs=64, dep=dep)
        assert a.solve_noalloc(P.MINIMIZE, time_limit=60) == P.OUT_OPTIMAL
        b = P.Solver(model, num_wgs=64, dep=dep)
        assert b.solve(P.MINIMIZE, time_limit=60) == P.OUT_OPTIMAL
        assert a.best()[0] == b.best()[0] == ref["best"]


def test_noalloc_refuses_oversized_workspace(P):
    # 16 bytes per stack level per workgroup: 65536 levels over the default
    # grid is far past the 64 MiB array
    model = I.rcpsp(30, 0)
    s = P.Solver(model, max_depth=65536)
    with pytest.raises(P.PccpError) as e:
        s.solve_noalloc(P.MINIMIZE, node_limit=100)
    assert e.value.code == P.E_NOMEM and "workspace" in str(e.value)
    # the entry point still works afterwards
    t = P.Solver(I.tiny_rcpsp(8, 1), num_wgs=1)
    assert t.solve_noalloc(P.MINIMIZE, time_limit=60) == P.OUT_OPTIMAL
