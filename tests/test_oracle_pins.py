"""Pins of the oracle's propagators against things other than itself:
hand-worked fixed points (tests/golden), Python's floor division, and brute
force over all points of tiny boxes."""
import itertools
import json
import os
import random

import numpy as np
import pytest

import oracle as O
from tests.models import make_model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- rounding
@pytest.mark.parametrize("a", list(range(-13, 14)))
@pytest.mark.parametrize("b", [-5, -4, -3, -2, -1, 1, 2, 3, 4, 5, 7])
def test_floor_ceil_div_match_python(a, b):
    # Python's // is floor division by definition; ceil(a/b) = -((-a)//b)
    assert O.floor_div(a, b) == a // b
    assert O.ceil_div(a, b) == -((-a) // b)


def test_floor_ceil_div_large():
    for a in (2**31 - 1, -(2**31), 2**40 + 3, -(2**40) - 7):
        for b in (1, 3, -7, 10):
            assert O.floor_div(a, b) == a // b
            assert O.ceil_div(a, b) == -((-a) // b)


# ---------------------------------------------------------------- golden
def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden("hand_fixpoints.json"), ids=lambda c: c["name"])
@pytest.mark.parametrize("sched", [O.SCHED_GS, O.SCHED_JACOBI, O.SCHED_REVERSE,
                                   O.SCHED_PERM, O.SCHED_SELECT])
def test_hand_fixpoints(case, sched):
    m = make_model(case["boxes"], case["rows"], case["reif"])
    st, lb, ub, _ = O.propagate(m, sched=sched, seed=7)
    if case["expect"] == "failed":
        assert st == O.FAILED
    else:
        assert st == O.FIXPOINT
        assert lb.tolist() == case["lb"]
        assert ub.tolist() == case["ub"]


# ------------------------------------------------- single linear row = hull
def _points(boxes):
    return itertools.product(*[range(lo, hi + 1) for lo, hi in boxes])


def test_single_row_fixpoint_is_hull_of_solutions():
    """For one row sum a_t x_t <= c, bound propagation is exact on bounds:
    the fixed point is the per-variable hull of the satisfying points, and
    it fails iff there is none.  Checked by enumeration on 3000 random
    rows of 1-3 variables over sub-boxes of [-6, 6]."""
    rng = random.Random(12345)
    nfail = 0
    for _ in range(3000):
        k = rng.randint(1, 3)
        boxes = []
        for _ in range(k):
            lo = rng.randint(-6, 6)
            boxes.append((lo, rng.randint(lo, 6)))
        coefs = [rng.choice([-4, -3, -2, -1, 1, 2, 3, 4]) for _ in range(k)]
        c = rng.randint(-20, 20)
        m = make_model(boxes, [(coefs, list(range(k)), c)])
        sols = [p for p in _points(boxes) if sum(a * x for a, x in zip(coefs, p)) <= c]
        st, lb, ub, _ = O.propagate(m)
        if not sols:
            nfail += 1
            assert st == O.FAILED, (boxes, coefs, c)
            continue
        assert st == O.FIXPOINT, (boxes, coefs, c)
        for v in range(k):
            vals = [p[v] for p in sols]
            assert lb[v] == min(vals) and ub[v] == max(vals), (boxes, coefs, c, v)
    assert nfail > 50  # the sample exercises failure too


# ------------------------------------------------- reified overlap, brute force
def _intervals(lo, hi):
    return [(a, b) for a in range(lo, hi + 1) for b in range(a, hi + 1)]


def test_reified_overlap_sound_and_decides_b():
    """b <=> (si <= sj and sj < si + d) over every sub-box of
    [0,6]^2 x {[0,0],[1,1],[0,1]}, d = 1..4:
      (i) soundness: no satisfying point of the box is removed, and failure
          only when there is no satisfying point;
      (ii) once si and sj are fixed, b is decided by the truth table."""
    for d in range(1, 5):
        for bi in _intervals(0, 6):
            for bj in _intervals(0, 6):
                for bb in [(0, 0), (1, 1), (0, 1)]:
                    boxes = [bb, bi, bj]
                    m = make_model(boxes, [], [(0, 1, 2, d)])
                    sols = [p for p in _points(boxes)
                            if (p[0] >= 1) == (p[1] <= p[2] < p[1] + d)]
                    st, lb, ub, _ = O.propagate(m)
                    if st == O.FAILED:
                        assert not sols, (boxes, d)
                        continue
                    for p in sols:
                        assert all(lb[v] <= p[v] <= ub[v] for v in range(3)), (boxes, d, p)
                    if bi[0] == bi[1] and bj[0] == bj[1]:
                        truth = int(bi[0] <= bj[0] < bi[0] + d)
                        if bb[0] <= truth <= bb[1]:
                            assert st == O.FIXPOINT and lb[0] == ub[0] == truth
                        else:
                            assert st == O.FAILED


def test_reified_overlap_fixed_b_hull_on_s():
    """With b fixed, the s-bounds after propagation contain the hull of the
    satisfying points (soundness), and when b = 1 the bounds equal the hull
    of psi (si <= sj <= si + d - 1 is a conjunction of two linear rows whose
    bound propagation reaches the hull for two variables)."""
    for d in range(1, 5):
        for bi in _intervals(0, 6):
            for bj in _intervals(0, 6):
                boxes = [(1, 1), bi, bj]
                m = make_model(boxes, [], [(0, 1, 2, d)])
                sols = [p for p in _points(boxes) if p[1] <= p[2] < p[1] + d]
                st, lb, ub, _ = O.propagate(m)
                if not sols:
                    assert st == O.FAILED
                    continue
                assert st == O.FIXPOINT
                for v in (1, 2):
                    vals = [p[v] for p in sols]
                    assert (lb[v], ub[v]) == (min(vals), max(vals)), (bi, bj, d)


# ------------------------------------------------- resource sum reading
def test_resource_sum_matches_corrected_lsum_reading():
    """The resource rows of §2 read with the term's own contribution taken
    out of lsum: for 0/1 variables with positive demands r_i and capacity c,
    the fixed point of one row fails iff sum r_i*lb(b_i) > c, and otherwise
    sets ub(b_i) = 0 exactly for the unfixed b_i with r_i + lsum > c."""
    rng = random.Random(99)
    for _ in range(2000):
        k = rng.randint(1, 8)
        r = [rng.randint(1, 10) for _ in range(k)]
        c = rng.randint(0, 25)
        boxes = [rng.choice([(0, 0), (1, 1), (0, 1), (0, 1)]) for _ in range(k)]
        m = make_model(boxes, [(r, list(range(k)), c)])
        st, lb, ub, _ = O.propagate(m)
        lsum = sum(ri * b[0] for ri, b in zip(r, boxes))
        if lsum > c:
            assert st == O.FAILED
            continue
        assert st == O.FIXPOINT
        for i in range(k):
            expect_ub = boxes[i][1]
            if boxes[i] == (0, 1) and r[i] + lsum > c:
                expect_ub = 0
            assert (lb[i], ub[i]) == (boxes[i][0], expect_ub)


# ------------------------------------- reified overlap with b = 0: exact hull
def _b0_cases():
    """Every sub-box of [0,6]^2 for (si, sj) with b = [0, 0], d = 1..4, in
    which interval entailment decides a disjunct of not psi = (si > sj) or
    (sj >= si + d): si <= sj or sj < si + d entailed (then the other
    disjunct, one difference constraint, must hold), or either disjunct
    entailed true (then nothing may be pruned).  On these boxes the
    constraint reduces to at most one linear row over two variables, whose
    bound propagation reaches the hull of its solutions exactly."""
    for d in range(1, 5):
        for bi in _intervals(0, 6):
            for bj in _intervals(0, 6):
                e1 = bi[1] <= bj[0]
                e2 = bj[1] <= bi[0] + d - 1
                n1 = bi[0] > bj[1]
                n2 = bj[0] >= bi[1] + d
                if e1 or e2 or n1 or n2:
                    yield d, bi, bj


def _b0_violations(prop):
    """Boxes of _b0_cases on which `prop(boxes, d) -> (failed, lb, ub)`
    differs from the hull of the points with b = 0 (FAILED iff none)."""
    bad, n = [], 0
    for d, bi, bj in _b0_cases():
        n += 1
        boxes = [(0, 0), bi, bj]
        sols = [p for p in _points(boxes) if not (p[1] <= p[2] < p[1] + d)]
        failed, lb, ub = prop(boxes, d)
        if not sols:
            if not failed:
                bad.append((d, bi, bj))
            continue
        hull = [(min(p[v] for p in sols), max(p[v] for p in sols)) for v in range(3)]
        if failed or [(int(lb[v]), int(ub[v])) for v in range(3)] != hull:
            bad.append((d, bi, bj))
    return bad, n


def _oracle_prop(boxes, d):
    st, lb, ub, _ = O.propagate(make_model(boxes, [], [(0, 1, 2, d)]))
    return st == O.FAILED, lb, ub


def _restated_prop(mutation=None):
    """The ten guarded commands of the reified item restated independently
    of the oracle, with one command dropped or weakened on request; used
    only to show that the b = 0 pin detects such a mistake."""
    def prop(boxes, d):
        lb = [b[0] for b in boxes]
        ub = [b[1] for b in boxes]
        B, I, J = 0, 1, 2
        cmds = {
            0: lambda e1, e2: (e1 and e2) and ("lb", B, 1),
            1: lambda e1, e2: (lb[I] > ub[J] or lb[J] >= ub[I] + d) and ("ub", B, 0),
            2: lambda e1, e2: lb[B] >= 1 and ("ub", I, ub[J]),
            3: lambda e1, e2: lb[B] >= 1 and ("lb", J, lb[I]),
            4: lambda e1, e2: lb[B] >= 1 and ("ub", J, ub[I] + d - 1),
            5: lambda e1, e2: lb[B] >= 1 and ("lb", I, lb[J] - d + 1),
            6: lambda e1, e2: (ub[B] <= 0 and e1) and ("lb", J, lb[I] + d),
            7: lambda e1, e2: (ub[B] <= 0 and e1) and ("ub", I, ub[J] - d),
            8: lambda e1, e2: (ub[B] <= 0 and e2) and ("ub", J, ub[I] - 1),
            9: lambda e1, e2: (ub[B] <= 0 and e2) and ("lb", I, lb[J] + 1),
        }
        if mutation == "drop7":
            del cmds[7]
        elif mutation == "drop8":
            del cmds[8]
        elif mutation == "drop9":
            del cmds[9]
        elif mutation == "dropG5":
            del cmds[8], cmds[9]
        elif mutation == "weaken8":
            cmds[8] = lambda e1, e2: (ub[B] <= 0 and e2) and ("ub", J, ub[I])
        elif mutation == "weaken7":
            cmds[7] = lambda e1, e2: (ub[B] <= 0 and e1) and ("ub", I, ub[J] - d + 1)
        changed = True
        while changed:
            changed = False
            for k in sorted(cmds):
                e1 = ub[I] <= lb[J]
                e2 = ub[J] <= lb[I] + d - 1
                t = cmds[k](e1, e2)
                if not t:
                    continue
                side, x, v = t
                if side == "lb" and v > lb[x]:
                    lb[x], changed = v, True
                elif side == "ub" and v < ub[x]:
                    ub[x], changed = v, True
                if lb[x] > ub[x]:
                    return True, lb, ub
        return False, lb, ub
    return prop


def test_reified_b_false_fixpoint_is_hull():
    """b = 0 with a disjunct of not psi decided by entailment: the s-bounds
    of the oracle's fixed point equal the hull of the points satisfying
    not psi, or the store fails iff there are none (commands 6-9, the two
    halves of each disjunct's difference constraint)."""
    bad, n = _b0_violations(_oracle_prop)
    assert n > 1000
    assert not bad, bad[:10]


@pytest.mark.parametrize("mutation", ["drop7", "drop8", "drop9", "dropG5", "weaken8", "weaken7"])
def test_reified_b_false_pin_detects_mistakes(mutation):
    """The pin above is strong enough to catch a dropped or weakened b = 0
    tell: the correct restatement passes it and each mutant fails it."""
    assert not _b0_violations(_restated_prop())[0]
    assert _b0_violations(_restated_prop(mutation))[0]


# ------------------------------------------------ the network's branching
def test_mlp_choice_hand_scores():
    """orc_mlp_choice against scores worked out by hand.  Parameters: hidden
    unit 0 reads the width feature f2 = (ub - lb) / H with weight 1, unit 1
    reads -f0 (never positive, so ReLU zeroes it) with output weight 100,
    unit 2 reads f0 = (lb - lo) / H with weight 1; output weights 1, 100, 1;
    every bias 0.  Four variables over [0, 10] (H = 10), no constraints:
      x0 = [10, 10]  fixed: skipped (its score f0 = 1 would win otherwise)
      x1 = [0, 4]    score 0.4
      x2 = [0, 6]    score 0.6
      x3 = [0, 6]    score 0.6  (tie with x2: the earlier position wins)
    so the choice is position 2 (first-fail would pick x1, position 1).
    With x2 and x3 fixed too, x1 is the only candidate; with every
    variable fixed the choice is -1."""
    p = np.zeros(O.NPARAM)
    nf, nh = O.NFEAT, O.NHID
    W1 = lambda k, f: k * nf + f
    b1, w2, b2 = nh * nf, nh * nf + nh, nh * nf + 2 * nh
    p[W1(0, 2)] = 1.0
    p[W1(1, 0)] = -1.0
    p[W1(2, 0)] = 1.0
    p[w2 + 0], p[w2 + 1], p[w2 + 2] = 1.0, 100.0, 1.0
    assert b1 + nh == w2 and b2 == O.NPARAM - 1
    m = make_model([(0, 10)] * 4, [], [])
    assert O.mlp_choice(m, p, [10, 0, 0, 0], [10, 4, 6, 6]) == 2
    assert O.mlp_choice(m, p, [10, 0, 3, 6], [10, 4, 3, 6]) == 1
    assert O.mlp_choice(m, p, [10, 4, 3, 6], [10, 4, 3, 6]) == -1
    # a larger lower bound raises f0 (unit 2): x3 = [1, 7] scores 0.6 + 0.1
    assert O.mlp_choice(m, p, [10, 0, 0, 1], [10, 4, 6, 7]) == 3
    # the output bias shifts every score alike and changes no choice
    p[b2] = -5.0
    assert O.mlp_choice(m, p, [10, 0, 0, 0], [10, 4, 6, 6]) == 2
