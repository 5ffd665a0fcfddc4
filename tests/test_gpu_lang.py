"""Programs of the PCCP front-end on the GPU against the oracle (the same
compiled models):
  - job shops: single-workgroup searches give the oracle's depth-first
    counters (every table, and dependency-driven); whole-GPU searches prove
    the oracle's optimum, which equals the disjunctive-graph brute force on
    the small ones;
  - random small programs enumerated: solution count and set hash;
  - the same with general guarded commands ({guards} => x <- f, §3 guarded
    normal form) on the library's guarded-command kind: random guarded
    programs, job shops whose disjunctions are guarded commands, and fixed
    points of random sub-boxes, element by element."""
import random
import sys

import numpy as np

import pytest

import oracle as O
from paper_2207_12116_amd import instances as I
from tests.models import jobshop_brute, random_subbox
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


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
def test_random_guarded_programs_enumerated(P, dep):
    """Guarded programs (when, ask_row, iff_row, disj_rows, views) run on
    the guarded-command kind: one workgroup reproduces the oracle's
    enumeration tree; 64 workgroups find the same solution set."""
    for seed in range(40):
        p, own, _ = _random_program(random.Random(seed + 1000), guarded=True)
        model = p.compile()
        assert model.ncmd > 0
        ref = O.solve(model, sol_cap=0)
        s = P.Solver(model, num_wgs=1, dep=dep)
        assert s.solve(time_limit=30) == P.OUT_ALL
        st = s.stats()
        assert (st["nodes"], st["fails"], st["solutions"], st["sol_hash"]) == \
            (ref["nodes"], ref["fails"], ref["solutions"], ref["sol_hash"]), seed
        m = P.Solver(model, num_wgs=64, dep=dep)
        assert m.solve(time_limit=30) == P.OUT_ALL
        sm = m.stats()
        assert (sm["nodes"], sm["solutions"], sm["sol_hash"]) == \
            (ref["nodes"], ref["solutions"], ref["sol_hash"]), seed


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
@pytest.mark.parametrize("nj,nm,seed", [(3, 3, 0), (4, 3, 1), (5, 4, 2)])
def test_guarded_jobshop_single_wg_parity(P, nj, nm, seed, dep):
    m = I.jobshop(nj, nm, seed, guarded=True)
    assert m.ncmd > 0
    ref = O.solve(m, node_limit=200000)
    say("guarded jobshop 1wg", nj, nm, seed, dep, ref["nodes"])
    s = P.Solver(m, num_wgs=1, dep=dep)
    out = s.solve(node_limit=200000, time_limit=60)
    st = s.stats()
    assert (st["nodes"], st["fails"], st["solutions"], st["best"], st["max_depth"]) == \
        (ref["nodes"], ref["fails"], ref["solutions"], ref["best"], ref["max_depth"])
    if ref["outcome"] == O.OUT_OPTIMAL:
        assert out == P.OUT_OPTIMAL
        if nj * nm <= 12:
            assert st["best"] == jobshop_brute(m.meta["jobs"])


@pytest.mark.parametrize("dep", [2, 1], ids=["tables", "dep"])
def test_guarded_jobshop_whole_gpu_optimum(P, dep):
    m = I.jobshop(6, 4, 1, guarded=True)
    ref = O.solve(m, node_limit=2000000)
    s = P.Solver(m, dep=dep)
    out = s.solve(time_limit=60)
    obj, vals = s.best()
    say("guarded jobshop whole", dep, P.OUTCOME_NAMES[out], obj, ref["best"])
    if ref["outcome"] == O.OUT_OPTIMAL:
        assert out == P.OUT_OPTIMAL and obj == ref["best"]


@pytest.mark.parametrize("wg", [64, 256, 1024])
def test_guarded_fixpoints_match_oracle(P, wg):
    """Fixed points of random sub-boxes of guarded models, every table every
    sweep and incrementally from fixed points, against the oracle."""
    import torch
    rng = random.Random(77 + wg)
    models = [I.jobshop(5, 4, 2, guarded=True)]
    for seed in range(6):
        p, own, _ = _random_program(random.Random(seed + 3000), guarded=True)
        models.append(p.compile())
    for model in models:
        om = O.OracleModel(model)
        boxes = [random_subbox(model, rng, frac=0.3) for _ in range(64)]
        dev = lambda a: torch.tensor(np.asarray(a), dtype=torch.int32, device="cuda")
        lbs, ubs = dev(np.stack([b[0] for b in boxes])), dev(np.stack([b[1] for b in boxes]))
        olb, oub = torch.empty_like(lbs), torch.empty_like(ubs)
        stt = torch.zeros(len(boxes), dtype=torch.int32, device="cuda")
        s = P.Solver(model, wg_size=wg)
        s.propagate_batch(lbs, ubs, olb, oub, stt)
        torch.cuda.synchronize()
        glb, gub, gst = olb.cpu().numpy(), oub.cpu().numpy(), stt.cpu().numpy()
        parents, dec = [], []
        for k, (lb0, ub0) in enumerate(boxes):
            st, lb, ub, _ = O.propagate(om, lb0, ub0)
            assert int(gst[k]) == st, (model.ncmd, k)
            if st == O.FIXPOINT:
                assert np.array_equal(glb[k], lb) and np.array_equal(gub[k], ub), (model.ncmd, k)
                free = [v for v in range(model.nvars) if lb[v] < ub[v]]
                if free:
                    x = rng.choice(free)
                    mid = rng.randint(int(lb[x]), int(ub[x]) - 1)
                    parents.append((lb, ub))
                    dec.append((x, int(lb[x]), mid) if rng.random() < 0.5 else (x, mid + 1, int(ub[x])))
        if not parents:
            continue
        # incremental: fixed point + one decision
        pl, pu = dev(np.stack([p_[0] for p_ in parents])), dev(np.stack([p_[1] for p_ in parents]))
        il, iu = torch.empty_like(pl), torch.empty_like(pu)
        ist = torch.zeros(len(parents), dtype=torch.int32, device="cuda")
        s.propagate_batch_incr(pl, pu, dev([d[0] for d in dec]), dev([d[1] for d in dec]),
                               dev([d[2] for d in dec]), il, iu, ist)
        torch.cuda.synchronize()
        gl, gu, gs = il.cpu().numpy(), iu.cpu().numpy(), ist.cpu().numpy()
        for k, ((lb, ub), (x, lo, hi)) in enumerate(zip(parents, dec)):
            jl, ju = lb.copy(), ub.copy()
            jl[x], ju[x] = max(jl[x], lo), min(ju[x], hi)
            st, rl, ru, _ = O.propagate(om, jl, ju)
            assert int(gs[k]) == st, (model.ncmd, k)
            if st == O.FIXPOINT:
                assert np.array_equal(gl[k], rl) and np.array_equal(gu[k], ru), (model.ncmd, k)
