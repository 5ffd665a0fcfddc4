"""Programs of the PCCP front-end on the GPU against the oracle (the same
compiled models):
  - job shops: single-workgroup searches give the oracle's depth-first
    counters (every table, and dependency-driven); whole-GPU searches prove
    the oracle's optimum, which equals the disjunctive-graph brute force on
    the small ones;
  - random small programs enumerated: solution count and set hash."""
import random
import sys

import pytest

import oracle as O
from paper_2207_12116_amd import instances as I
from tests.models import jobshop_brute
from tests.test_lang import _random_program

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


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
@pytest.mark.parametrize("nj,nm,seed", [(3, 3, 0), (4, 3, 1), (5, 4, 2), (6, 4, 3)])
def test_jobshop_single_wg_parity(P, nj, nm, seed, dep):
    m = I.jobshop(nj, nm, seed)
    ref = O.solve(m, node_limit=200000)
    say("jobshop 1wg", nj, nm, seed, dep, ref["nodes"])
    s = P.Solver(m, num_wgs=1, dep=dep)
    out = s.solve(node_limit=200000, time_limit=60)
    st = s.stats()
    assert (st["nodes"], st["fails"], st["solutions"], st["best"], st["max_depth"]) == \
        (ref["nodes"], ref["fails"], ref["solutions"], ref["best"], ref["max_depth"])
    if ref["outcome"] == O.OUT_OPTIMAL:
        assert out == P.OUT_OPTIMAL


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
@pytest.mark.parametrize("nj,nm,seed", [(4, 3, 0), (6, 4, 1), (7, 4, 2)])
def test_jobshop_whole_gpu_optimum(P, nj, nm, seed, dep):
    m = I.jobshop(nj, nm, seed)
    ref = O.solve(m, node_limit=2000000)
    s = P.Solver(m, dep=dep)
    out = s.solve(time_limit=60)
    obj, vals = s.best()
    say("jobshop whole", nj, nm, seed, dep, P.OUTCOME_NAMES[out], obj, ref["best"])
    if ref["outcome"] == O.OUT_OPTIMAL:
        assert out == P.OUT_OPTIMAL and obj == ref["best"]
    if nj * nm <= 12:
        assert obj == jobshop_brute(m.meta["jobs"])


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
def test_random_programs_enumerated(P, dep):
    for seed in range(20):
        p, own, _ = _random_program(random.Random(seed))
        model = p.compile()
        ref = O.solve(model, sol_cap=0)
        s = P.Solver(model, num_wgs=1, dep=dep)
        assert s.solve(time_limit=30) == P.OUT_ALL
        st = s.stats()
        assert (st["nodes"], st["fails"], st["solutions"], st["sol_hash"]) == \
            (ref["nodes"], ref["fails"], ref["solutions"], ref["sol_hash"]), seed
