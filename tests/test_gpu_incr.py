"""Dependency-driven fixed points compared store by store with the oracle.

pccp_propagate_batch_incr starts from a fixed point and one decision, and
runs only the propagators that read a bound the decision (and then each
sweep) tightened.  Chaotic iteration (§3, Theorem 2) says this reaches the
least fixed point of the joined box; the oracle computes that fixed point by
running every propagator until nothing changes.  Parents are fixed points of
the oracle's own: the root and nodes reached by random splits of decision
variables; decisions range over every variable kind (start times, overlap
Booleans, the makespan) and include ones that change nothing, ones that
empty a domain, and an out-of-range variable.
"""
import random
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


def _parents(om, model, rng, count, depth):
    """Fixed points of the oracle: the root and the nodes reached by up to
    `depth` random splits (x <= mid or x >= mid + 1) of decision variables,
    each split propagated; a split that fails is dropped."""
    st, lb0, ub0, _ = O.propagate(om)
    assert st == O.FIXPOINT
    out = [(lb0, ub0)]
    while len(out) < count:
        lb, ub = lb0, ub0
        for _ in range(rng.randint(1, depth)):
            free = [x for x in model.decision if lb[x] < ub[x]]
            if not free:
                break
            x = rng.choice(free)
            mid = rng.randint(int(lb[x]), int(ub[x]) - 1)
            clb, cub = lb.copy(), ub.copy()
            if rng.random() < 0.5:
                cub[x] = mid
            else:
                clb[x] = mid + 1
            r = O.propagate(om, clb, cub)
            if r[0] == O.FIXPOINT:
                lb, ub = r[1], r[2]
        out.append((lb, ub))
    return out


def _decision(model, lb, ub, rng):
    """(var, lo, hi): a split of a random variable, or a join that changes
    nothing, or one that empties the domain."""
    r = rng.random()
    x = rng.randrange(model.nvars)
    if r < 0.1:
        return x, int(lb[x]), int(ub[x])                 # no change
    if r < 0.15:
        return x, int(ub[x]) + 1, int(ub[x]) + 1         # empty
    free = [v for v in range(model.nvars) if lb[v] < ub[v]]
    if not free:
        return x, int(lb[x]), int(ub[x])
    if r < 0.7:
        x = rng.choice([v for v in model.decision if lb[v] < ub[v]] or free)
    else:
        x = rng.choice(free)
    mid = rng.randint(int(lb[x]), int(ub[x]) - 1)
    if rng.random() < 0.5:
        return x, int(lb[x]), mid
    return x, mid + 1, int(ub[x])


INCR_MODELS = [("csp3", lambda: I.tiny_csp(3), 40, 3), ("rcpsp30s0", lambda: I.rcpsp(30, 0), 48, 6),
               ("rcpsp30s7", lambda: I.rcpsp(30, 7), 48, 6), ("rcpsp60", lambda: I.rcpsp(60, 1), 24, 6),
               ("rcpsp120", lambda: I.rcpsp(120, 0), 12, 8),
               ("jobshop", lambda: I.jobshop(6, 6, 2), 32, 6)]


@pytest.mark.parametrize("name,mk,npar,depth", INCR_MODELS, ids=[m[0] for m in INCR_MODELS])
@pytest.mark.parametrize("wg", [64, 256, 1024])
def test_incremental_fixpoints_match_oracle(P, name, mk, npar, depth, wg):
    import torch
    model = mk()
    om = O.OracleModel(model)
    rng = random.Random(sum(map(ord, name)) * 7 + wg)
    parents = _parents(om, model, rng, npar, depth)
    boxes, dec = [], []
    for i, (lb, ub) in enumerate(parents):
        for j in range(3):
            boxes.append((lb, ub))
            if i == 0 and j == 2:
                x = int(model.decision[0])
                dec.append((x, int(ub[x]) + 1, int(ub[x]) + 1))      # empties s_0
            else:
                dec.append(_decision(model, lb, ub, rng))
    # an out-of-range variable: the box comes back unchanged with status -1
    boxes.append(parents[0])
    dec.append((model.nvars, 0, 0))
    nb = len(boxes)
    say("incremental", name, wg, nb, "boxes")
    dev = lambda a: torch.tensor(np.asarray(a), dtype=torch.int32, device="cuda")
    lbs = dev(np.stack([b[0] for b in boxes]))
    ubs = dev(np.stack([b[1] for b in boxes]))
    dv, dlo, dhi = dev([d[0] for d in dec]), dev([d[1] for d in dec]), dev([d[2] for d in dec])
    olb, oub = torch.empty_like(lbs), torch.empty_like(ubs)
    stt = torch.full((nb,), 7, dtype=torch.int32, device="cuda")
    sw = torch.zeros(nb, dtype=torch.int32, device="cuda")
    s = P.Solver(model, wg_size=wg)
    s.propagate_batch_incr(lbs, ubs, dv, dlo, dhi, olb, oub, stt, sw)
    # the same joined boxes through the every-table loop
    jl, ju = lbs.clone(), ubs.clone()
    for k, (x, lo, hi) in enumerate(dec[:-1]):
        jl[k, x] = max(int(jl[k, x]), lo)
        ju[k, x] = min(int(ju[k, x]), hi)
    flb, fub = torch.empty_like(lbs), torch.empty_like(ubs)
    fst = torch.zeros(nb, dtype=torch.int32, device="cuda")
    fsw = torch.zeros(nb, dtype=torch.int32, device="cuda")
    s.propagate_batch(jl[:-1].contiguous(), ju[:-1].contiguous(), flb[:-1], fub[:-1], fst, fsw)
    torch.cuda.synchronize()
    glb, gub, gst = olb.cpu().numpy(), oub.cpu().numpy(), stt.cpu().numpy()
    jl, ju = jl.cpu().numpy(), ju.cpu().numpy()
    nfail = nsame = 0
    for k in range(nb - 1):
        st, lb, ub, _ = O.propagate(om, jl[k], ju[k])
        assert int(gst[k]) == st, (name, k, dec[k])
        assert int(fst.cpu().numpy()[k]) == st
        if st == O.FIXPOINT:
            assert np.array_equal(glb[k], lb), (name, k, dec[k])
            assert np.array_equal(gub[k], ub), (name, k, dec[k])
            nsame += np.array_equal(lb, boxes[k][0]) and np.array_equal(ub, boxes[k][1])
        else:
            nfail += 1
    assert gst[-1] == -1
    assert np.array_equal(glb[-1], boxes[-1][0]) and np.array_equal(gub[-1], boxes[-1][1])
    # the incremental loop never runs more sweeps than the every-table loop
    # needs plus one (its first sweep may find nothing to do)
    sweeps = sw.cpu().numpy()[:-1]
    say("incremental", name, wg, "failed", nfail, "unchanged", nsame,
        "sweeps incr/full", int(sweeps.sum()), int(fsw.cpu().numpy().sum()))
    assert nfail > 0 and nfail < nb - 1


@pytest.mark.parametrize("wg", [256, 512])
def test_incremental_chain_follows_search_path(P, wg):
    """A chain of incremental calls down one path of decisions (each output
    the next input) ends at the oracle's fixed point of the whole path."""
    import torch
    model = I.rcpsp(30, 4)
    om = O.OracleModel(model)
    st, lb, ub, _ = O.propagate(om)
    s = P.Solver(model, wg_size=wg)
    cur_l = torch.tensor(lb[None, :], dtype=torch.int32, device="cuda")
    cur_u = torch.tensor(ub[None, :], dtype=torch.int32, device="cuda")
    rl, ru = lb.copy(), ub.copy()
    for step, x in enumerate(model.decision[:12]):
        # left branch of first-fail's value rule: x = lb(x)
        v = int(rl[x])
        dv = torch.tensor([x], dtype=torch.int32, device="cuda")
        lo = torch.tensor([v], dtype=torch.int32, device="cuda")
        hi = torch.tensor([v], dtype=torch.int32, device="cuda")
        nl, nu = torch.empty_like(cur_l), torch.empty_like(cur_u)
        stt = torch.zeros(1, dtype=torch.int32, device="cuda")
        s.propagate_batch_incr(cur_l, cur_u, dv, lo, hi, nl, nu, stt)
        torch.cuda.synchronize()
        jl, ju = rl.copy(), ru.copy()
        jl[x], ju[x] = max(jl[x], v), min(ju[x], v)
        ref = O.propagate(om, jl, ju)
        assert int(stt.item()) == ref[0], step
        if ref[0] != O.FIXPOINT:
            break
        assert np.array_equal(nl.cpu().numpy()[0], ref[1]) and np.array_equal(nu.cpu().numpy()[0], ref[2])
        cur_l, cur_u, rl, ru = nl, nu, ref[1], ref[2]
