"""Entailment of a propagator, the condition under which the search may leave
it out of every sweep below a node (item lists).  The reading: a propagator
is entailed in a box when none of its tells can tighten that box or any
tighter non-empty box.  Dropping such propagators leaves every least fixed
point unchanged (§3 Theorem 2: the fixed point is the least box closed under
the propagators, and an entailed one is closed on every box that follows).

For each kind the condition the search uses is restated here and checked
against the oracle by brute force: whenever it holds on a small random box,
the oracle's propagation of that single propagator changes no non-empty
sub-box at all.  The conditions are also checked to be reachable (they hold
on a good share of the boxes drawn), so the check is not vacuous."""
import itertools
import random

import numpy as np
import pytest

import oracle as O
from tests.models import make_model


def _intervals(lo, hi):
    return [(a, b) for a in range(lo, hi + 1) for b in range(a, hi + 1)]


def _closed_on_all_subboxes(model, box):
    for sub in itertools.product(*[_intervals(a, b) for a, b in box]):
        lb = np.array([s[0] for s in sub], dtype=np.int32)
        ub = np.array([s[1] for s in sub], dtype=np.int32)
        st, l2, u2, _ = O.propagate(model, lb, ub)
        if st != O.FIXPOINT or not (np.array_equal(l2, lb) and np.array_equal(u2, ub)):
            return False, sub
    return True, None


def _random_box(rng, nvar, lo, hi, boolean=()):
    box = []
    for v in range(nvar):
        if v in boolean:
            box.append(rng.choice([(0, 0), (1, 1), (0, 1)]))
        else:
            a, b = sorted((rng.randint(lo, hi), rng.randint(lo, hi)))
            box.append((a, b))
    return box


def diff_entailed(box, c):
    (lx, ux), (ly, uy) = box
    return ux - ly <= c


def reif_entailed(box, d):
    (lb_, ub_), (li, ui), (lj, uj) = box
    return (lb_ >= 1 and ui <= lj and uj <= li + d - 1) or \
           (ub_ <= 0 and (li > uj or lj >= ui + d))


def row_entailed(box, a, c):
    return sum(max(k * l, k * u) for k, (l, u) in zip(a, box)) <= c


@pytest.mark.parametrize("seed", range(4))
def test_difference_row_entailment(seed):
    rng = random.Random(seed)
    hits = 0
    for _ in range(60):
        c = rng.randint(-3, 3)
        box = _random_box(rng, 2, 0, 5)
        if not diff_entailed(box, c):
            continue
        hits += 1
        model = make_model([(0, 5), (0, 5)], [([1, -1], [0, 1], c)])
        ok, sub = _closed_on_all_subboxes(model, box)
        assert ok, (box, c, sub)
    assert hits >= 5


@pytest.mark.parametrize("seed", range(4))
def test_reified_overlap_entailment(seed):
    rng = random.Random(100 + seed)
    hits = 0
    for _ in range(150):
        d = rng.randint(1, 3)
        box = _random_box(rng, 3, 0, 5, boolean=(0,))
        if not reif_entailed(box, d):
            continue
        hits += 1
        model = make_model([(0, 1), (0, 5), (0, 5)], [], [(0, 1, 2, d)])
        ok, sub = _closed_on_all_subboxes(model, box)
        assert ok, (box, d, sub)
    assert hits >= 5


def test_reified_overlap_not_entailed_is_live():
    """A box just outside the condition can still be tightened by some
    sub-box (the condition is not needlessly strong for these cases)."""
    model = make_model([(0, 1), (0, 5), (0, 5)], [], [(0, 1, 2, 2)])
    # b = 1, si <= sj entailed but sj < si + d not: sub-boxes get tightened
    box = [(1, 1), (0, 1), (1, 4)]
    assert not reif_entailed(box, 2)
    assert not _closed_on_all_subboxes(model, box)[0]
    # b open and nothing decided
    box = [(0, 1), (0, 3), (0, 3)]
    assert not reif_entailed(box, 2)
    assert not _closed_on_all_subboxes(model, box)[0]


@pytest.mark.parametrize("seed", range(4))
def test_linear_row_entailment(seed):
    rng = random.Random(200 + seed)
    hits = 0
    for _ in range(80):
        n = rng.randint(2, 3)
        a = [rng.choice([-3, -2, -1, 1, 2, 3]) for _ in range(n)]
        c = rng.randint(-4, 8)
        boolean = tuple(v for v in range(n) if rng.random() < 0.4)
        box = _random_box(rng, n, 0, 3, boolean=boolean)
        if not row_entailed(box, a, c):
            continue
        hits += 1
        boxes = [(0, 1) if v in boolean else (0, 3) for v in range(n)]
        model = make_model(boxes, [(a, list(range(n)), c)])
        ok, sub = _closed_on_all_subboxes(model, box)
        assert ok, (box, a, c, sub)
    assert hits >= 5
