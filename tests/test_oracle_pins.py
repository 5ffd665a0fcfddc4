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
