"""Float interval stores on the GPU against the oracle (oracle/fprop.c),
bit for bit: the tells are monotone, so the least fixed point is unique
(§3 Theorem 2) and the concurrent sweeps must reach the oracle's store
exactly, rounding included.  Root boxes and random sub-boxes of the tiny CSP
over the reals and of sparse random systems up to 4000 variables, several
workgroup sizes; boxes that fail; canonical zeros; invalid models refused."""
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


def _subboxes(model, rng, count, frac=0.3):
    out = [(model.lb.copy(), model.ub.copy())]
    for _ in range(count - 1):
        lb, ub = model.lb.copy(), model.ub.copy()
        for v in range(model.nvars):
            if rng.random() < frac:
                a = np.float32(rng.uniform(float(lb[v]), float(ub[v])))
                b = np.float32(rng.uniform(float(lb[v]), float(ub[v])))
                lo, hi = min(a, b), max(a, b)
                r = rng.random()
                if r < 0.4:
                    lb[v], ub[v] = lo, hi
                elif r < 0.7:
                    lb[v] = lo
                else:
                    ub[v] = hi
        out.append((lb, ub))
    return out


def _run(P, model, boxes, wg):
    import torch
    dev = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")
    lbs = dev(np.stack([b[0] for b in boxes]))
    ubs = dev(np.stack([b[1] for b in boxes]))
    olb, oub = torch.empty_like(lbs), torch.empty_like(ubs)
    st = torch.full((len(boxes),), 7, dtype=torch.int32, device="cuda")
    sw = torch.zeros(len(boxes), dtype=torch.int32, device="cuda")
    s = P.FSolver(model, wg_size=wg)
    s.propagate_batch(lbs, ubs, olb, oub, st, sw)
    torch.cuda.synchronize()
    return st.cpu().numpy(), olb.cpu().numpy(), oub.cpu().numpy(), sw.cpu().numpy()


FMODELS = [("csp%d" % s, lambda s=s: I.float_csp(s)) for s in (0, 1, 2, 3)] + \
          [("net100", lambda: I.float_network(100, 1)), ("net1000", lambda: I.float_network(1000, 2)),
           ("net4000", lambda: I.float_network(4000, 3, rows_per_var=1)),
           # rows of 2..12 terms: rows longer than the kernel's register rows,
           # and wavefronts whose rows differ in length
           ("net300k12", lambda: I.float_network(300, 4, kmax=12)),
           # a store of 120 KB: most of a workgroup's LDS
           ("net15000", lambda: I.float_network(15000, 5, rows_per_var=1))]


@pytest.mark.parametrize("name,mk", FMODELS, ids=[m[0] for m in FMODELS])
@pytest.mark.parametrize("wg", [64, 256, 1024])
def test_float_fixpoints_bit_exact(P, name, mk, wg):
    model = mk()
    om = O.OracleFModel(model)
    rng = random.Random(sum(map(ord, name)) + wg)
    nbox = 64 if model.nvars <= 1000 else 8
    boxes = _subboxes(model, rng, nbox)
    say("float fixpoints", name, wg, nbox)
    gst, glb, gub, gsw = _run(P, model, boxes, wg)
    nfail = 0
    for k, (lb0, ub0) in enumerate(boxes):
        st, lb, ub, _ = O.fpropagate(om, lb0, ub0)
        assert int(gst[k]) == st, (name, k)
        if st == O.FIXPOINT:
            assert np.array_equal(glb[k].view(np.uint32), lb.view(np.uint32)), (name, k)
            assert np.array_equal(gub[k].view(np.uint32), ub.view(np.uint32)), (name, k)
        else:
            nfail += 1
    assert (gsw >= 1).all()
    say("float fixpoints", name, wg, "failed", nfail, "of", nbox)


# Bounds, coefficients and right-hand sides from subnormals to 3.4e38: the
# products and sums overflow to -inf, underflow to subnormals and cancel to
# signed zeros, and the quotients leave the float range.  Small systems
# (rows of 1..10 terms, every code path of the row kernel in mixed
# wavefronts) and wide ones (hundreds of rows of each length, so whole
# wavefronts share a length).  The oracle runs first: every case here takes
# it at most a few sweeps.
FEXT = [("ext%d" % s, lambda s=s: I.float_extreme(s), 64, 0.3) for s in range(4)] + \
       [("ext_wide3_%d" % s, lambda s=s: I.float_extreme(s, n=1000, nrows=500, kmax=3), 16, 0.05)
        for s in (4, 5)] + \
       [("ext_wide4_%d" % s, lambda s=s: I.float_extreme(s, n=600, nrows=400, kmax=4), 16, 0.05)
        for s in (4, 5)]


@pytest.mark.parametrize("name,mk,nbox,frac", FEXT, ids=[m[0] for m in FEXT])
def test_float_extreme_magnitudes_bit_exact(P, name, mk, nbox, frac):
    model = mk()
    om = O.OracleFModel(model)
    boxes = _subboxes(model, random.Random(sum(map(ord, name))), nbox, frac)
    refs = [O.fpropagate(om, lb0, ub0) for lb0, ub0 in boxes]
    assert max(r[3] for r in refs) <= 20, name
    say("float extreme", name, model.nvars, model.nrows, nbox)
    gst, glb, gub, _ = _run(P, model, boxes, 256)
    nfix = 0
    for k, (st, lb, ub, _) in enumerate(refs):
        assert int(gst[k]) == st, (name, k)
        if st == O.FIXPOINT:
            nfix += 1
            assert np.array_equal(glb[k].view(np.uint32), lb.view(np.uint32)), (name, k)
            assert np.array_equal(gub[k].view(np.uint32), ub.view(np.uint32)), (name, k)
    say("float extreme", name, "fixed points", nfix, "of", nbox)


def test_float_failure_and_zeros(P):
    # no real solution: x + y <= 1, x >= 0.75, y >= 0.5
    m = I._fmodel([0.0, 0.0], [10.0, 10.0],
                  [([1.0, 1.0], [0, 1], 1.0), ([-1.0], [0], -0.75), ([-1.0], [1], -0.5)], {})
    st, lb, ub, _ = _run(P, m, [(m.lb, m.ub)], 64)
    assert st[0] == 1
    # zero bounds come back canonical: -0 below, +0 above
    m = I._fmodel([0.0, -1.0], [1.0, 0.0], [([1.0, 1.0], [0, 1], 0.0),
                                            ([-1.0, -1.0], [0, 1], 0.0)], {})
    box = (np.float32([0.0, -0.0]), np.float32([-0.0, 0.0]))
    st, lb, ub, _ = _run(P, m, [box], 64)
    ref = O.fpropagate(m, *box)
    assert st[0] == ref[0] == 0
    assert np.array_equal(lb[0].view(np.uint32), ref[1].view(np.uint32))
    assert np.array_equal(ub[0].view(np.uint32), ref[2].view(np.uint32))
    assert np.signbit(lb[0][0]) and not np.signbit(ub[0][0])


def test_float_models_refused(P):
    bad = [I._fmodel([0.0], [np.inf], [([1.0], [0], 1.0)], {}),          # infinite bound
           I._fmodel([0.0], [1.0], [([0.0], [0], 1.0)], {}),             # zero coefficient
           I._fmodel([0.0, 0.0], [1.0, 1.0], [([1.0, 1.0], [0, 0], 1.0)], {})]   # repeated
    for m in bad:
        with pytest.raises(P.PccpError) as e:
            P.FSolver(m)
        assert e.value.code == P.E_MODEL
