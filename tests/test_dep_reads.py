"""Which bounds each propagator reads — the reading behind dependency-driven
propagation: a propagator has to run again only after a bound it reads was
tightened.  Pinned on the oracle's propagators: the tells of one Jacobi
sweep over a single propagator depend only on the bounds it is said to
read.  With s and s2 equal on those bounds, and s2 arbitrary (within the
initial box) on the others, one sweep from s2 must give s2 joined with what
one sweep from s gives when every other bound of s is the initial one:

  difference row x - y <= c : lb(x), ub(y)
  linear row sum a x <= c   : lb(x) for a > 0, ub(x) for a < 0
  Boolean row (0/1, a > 0)  : lb of every term
  reified overlap           : both bounds of b, si, sj (its whole scope)
"""
import random

import numpy as np
import pytest

import oracle as O
from paper_2207_12116_amd.instances import _Builder, MODE_ENUMERATE

H = 12


def _model(add):
    b = _Builder()
    add(b)
    return b.finish([], -1, MODE_ENUMERATE, {})


def _random_box(rng, lo, hi, n):
    lb = np.empty(n, np.int32)
    ub = np.empty(n, np.int32)
    for i in range(n):
        a, c = sorted((rng.randint(lo[i], hi[i]), rng.randint(lo[i], hi[i])))
        lb[i], ub[i] = a, c
    return lb, ub


def _check(model, reads_lb, reads_ub, rng, trials=400):
    """reads_lb[i] / reads_ub[i]: the propagator reads lb / ub of variable i."""
    lo, hi = model.lb.copy(), model.ub.copy()
    n = model.nvars
    for _ in range(trials):
        lb, ub = _random_box(rng, lo, hi, n)
        lb2, ub2 = _random_box(rng, lo, hi, n)
        # s2 agrees with s on the bounds read
        lb2 = np.where(reads_lb, lb, lb2).astype(np.int32)
        ub2 = np.where(reads_ub, ub, ub2).astype(np.int32)
        if np.any(lb2 > ub2):
            continue
        # s with every bound it does not read at the initial box
        lbl = np.where(reads_lb, lb, lo).astype(np.int32)
        ubl = np.where(reads_ub, ub, hi).astype(np.int32)
        _, ol, ou = O.jacobi_step(model, lbl, ubl)
        _, o2l, o2u = O.jacobi_step(model, lb2, ub2)
        assert np.array_equal(o2l, np.maximum(lb2, ol)), (lb2, ub2, lbl, ubl)
        assert np.array_equal(o2u, np.minimum(ub2, ou)), (lb2, ub2, lbl, ubl)


@pytest.mark.parametrize("c", [-5, -1, 0, 3])
def test_difference_row_reads_lb_x_ub_y(c):
    m = _model(lambda b: (b.add_vars(2, 0, H), b.add_row([1, -1], [0, 1], c)))
    _check(m, np.array([True, False]), np.array([False, True]), random.Random(c))


def test_difference_row_read_set_is_not_smaller():
    """The pin above has teeth: leaving out lb(x) (or ub(y)) from the read
    set makes the check fail."""
    m = _model(lambda b: (b.add_vars(2, 0, H), b.add_row([1, -1], [0, 1], -2)))
    for rl, ru in (([False, False], [False, True]), ([True, False], [False, False])):
        with pytest.raises(AssertionError):
            _check(m, np.array(rl), np.array(ru), random.Random(1))


@pytest.mark.parametrize("seed", range(6))
def test_linear_row_reads_by_coefficient_sign(seed):
    rng = random.Random(seed)
    k = rng.randint(2, 4)
    coefs = [rng.choice([-3, -2, -1, 1, 2, 3]) for _ in range(k)]
    rhs = rng.randint(-H, 2 * H)
    m = _model(lambda b: (b.add_vars(k, -H // 2, H), b.add_row(coefs, list(range(k)), rhs)))
    pos = np.array([a > 0 for a in coefs])
    _check(m, pos, ~pos, rng)


@pytest.mark.parametrize("seed", range(4))
def test_boolean_row_reads_lower_bounds(seed):
    rng = random.Random(100 + seed)
    k = rng.randint(3, 6)
    coefs = [rng.randint(1, 5) for _ in range(k)]
    rhs = rng.randint(1, sum(coefs))
    m = _model(lambda b: (b.add_vars(k, 0, 1), b.add_row(coefs, list(range(k)), rhs)))
    _check(m, np.ones(k, bool), np.zeros(k, bool), rng)


@pytest.mark.parametrize("d", [1, 2, 4])
def test_reified_overlap_reads_its_scope_only(d):
    """The item reads every bound of b, si and sj, and nothing else: a
    fourth variable outside its scope may take any value."""
    def add(b):
        b.add_vars(2, 0, H)
        b.add_vars(1, 0, 1)
        b.add_vars(1, 0, H)          # not in the item's scope
        b.add_reif(2, 0, 1, d)
    m = _model(add)
    _check(m, np.array([True, True, True, False]), np.array([True, True, True, False]),
           random.Random(d))
