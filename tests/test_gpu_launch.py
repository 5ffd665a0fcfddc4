"""Launch forms of the search: hipGraph replay vs plain launches, and the
autotuner.  A graph is replayed several times with eager work and
synchronisation in between; every replay must equal the plain launch."""
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
    return (st["nodes"], st["fails"], st["solutions"], st["sol_hash"], st["best"])


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
def test_graph_replays_match_plain_launch(P, dep):
    model = I.tiny_csp(1, dom=12)
    ref = O.solve(model)
    plain = P.Solver(model, num_wgs=1, launch=1, dep=dep)
    assert plain.solve(time_limit=60) == P.OUT_ALL
    want = counts(plain)
    assert want[:4] == (ref["nodes"], ref["fails"], ref["solutions"], ref["sol_hash"])
    g = P.Solver(model, num_wgs=1, launch=0, dep=dep)
    other = P.Solver(I.rcpsp(30, 1))
    for rep in range(4):
        print("graph replay", rep, file=sys.stderr, flush=True)
        assert g.solve(time_limit=60) == P.OUT_ALL
        assert counts(g) == want
        other.propagate()        # eager work between replays
    # multi-workgroup graph: ENUMERATE counts are schedule-free
    gm = P.Solver(I.tiny_csp(2, dom=14), launch=0, dep=dep)
    refm = O.solve(I.tiny_csp(2, dom=14))
    for rep in range(3):
        assert gm.solve(time_limit=60) == P.OUT_ALL
        st = gm.stats()
        assert (st["nodes"], st["solutions"], st["sol_hash"]) == \
            (refm["nodes"], refm["solutions"], refm["sol_hash"])


def test_graph_minimize_batch_replays(P):
    models = [I.tiny_rcpsp(n, s) for n, s in [(8, 0), (10, 1), (9, 2), (12, 3)]]
    refs = [O.solve(m)["best"] for m in models]
    solvers = [P.Solver(m) for m in models]
    cfg = P.Config(launch=0)
    for rep in range(3):
        outs = P.batch_solve(solvers, P.MINIMIZE, config=cfg, time_limit=60)
        assert outs == [P.OUT_OPTIMAL] * 4
        assert [s.best()[0] for s in solvers] == refs


def test_autotune_picks_a_working_config(P, tmp_path):
    from paper_2207_12116_amd import autotune
    models = [I.rcpsp(30, s) for s in range(4)]
    cfg, rep = autotune.tune(models, budget_s=0.15, cache_path=str(tmp_path / "at.json"),
                             wg_sizes=(128, 256))
    assert not rep["cached"] and len(rep["candidates"]) >= 4
    assert cfg.wg_size in (128, 256)
    cfg2, rep2 = autotune.tune(models, budget_s=0.15, cache_path=str(tmp_path / "at.json"),
                               wg_sizes=(128, 256))
    assert rep2["cached"] and cfg2.wg_size == cfg.wg_size
    # the tuned configuration still finds the oracle's optimum
    small = [I.tiny_rcpsp(10, 1)]
    s = P.Solver(small[0], config=cfg)
    assert s.solve(time_limit=60) == P.OUT_OPTIMAL
    assert s.best()[0] == O.solve(small[0])["best"]


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
def test_instance_node_budget_abandons_only_the_hard_instance(P, dep):
    """A batch with a per-instance node budget: the instance that exhausts it
    is abandoned (LIMIT) while the small ones are still proven, with the
    oracle's optima; the abandoned instance stopped near its budget."""
    easy = [I.rcpsp_model(*I.rcpsp_data(n, s)[:4]) for n, s in [(8, 0), (10, 2), (9, 1)]]
    hard = I.rcpsp(30, 0)
    refs = [O.solve(m, node_limit=400000) for m in easy]
    solvers = [P.Solver(m) for m in easy + [hard]]
    budget = 2_000_000
    outs = P.batch_solve(solvers, P.MINIMIZE, config=P.Config(dep=dep), time_limit=60,
                         inst_node_limit=budget)
    say("budget outcomes", outs)
    for s, o, r, m in zip(solvers, outs, refs, easy):
        assert o == P.OUT_OPTIMAL
        assert s.best()[0] == r["best"]
        ok, ms = O.check_schedule(m.meta, s.best()[1])
        assert ok and ms == s.best()[0]
    st = solvers[-1].stats()
    assert outs[-1] == P.OUT_LIMIT and st["ttpo_ms"] < 0
    assert budget <= st["nodes"] <= budget + 512 * st["grid"]


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
def test_host_cancel_word_stops_search(P, dep):
    """A search with a 30 s limit on an instance no search proves in that
    time: another host thread sets the pinned cancel word after 0.5 s, and
    the search returns CANCELLED well before its limit, with sound
    counters."""
    import threading
    import time
    import torch
    cancel = torch.zeros(1, dtype=torch.int32).pin_memory()
    s = P.Solver(I.rcpsp(30, 0), dep=dep)

    def setter():
        time.sleep(0.5)
        cancel[0] = 1

    th = threading.Thread(target=setter)
    th.start()
    t0 = time.time()
    out = s.solve(time_limit=30.0, cancel=cancel)
    el = time.time() - t0
    th.join()
    st = s.stats()
    say("cancel", dep, P.OUTCOME_NAMES[out], round(el, 3), st["nodes"])
    assert out == P.OUT_CANCELLED and st["outcome"] == P.OUT_CANCELLED
    assert 0.4 < el < 10.0
    assert st["nodes"] > 0 and st["ttpo_ms"] < 0
    # the word cleared, the same solver searches again to its limit
    cancel[0] = 0
    assert s.solve(time_limit=0.3, cancel=cancel) == P.OUT_LIMIT
