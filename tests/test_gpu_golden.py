"""HIP solver against the hand-worked values of tests/golden directly (no
oracle in between): every fixed point worked out by hand from the
compilation rules of §2 and every hand-solved search of §1-§2 (solution
sets of a small CSP, optima of tiny RCPSPs), in each propagation mode."""
import json
import os
import sys

import numpy as np
import pytest

from paper_2207_12116_amd import instances as I
from tests.models import make_model

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cases(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)["cases"]


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_12116_amd import pccp
    pccp.lib()
    return pccp


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("case", _cases("hand_fixpoints.json"), ids=lambda c: c["name"])
def test_hand_fixpoints_on_gpu(P, case):
    say("hand fixpoint", case["name"])
    m = make_model(case["boxes"], case["rows"], case["reif"])
    st, lb, ub = P.Solver(m).propagate()
    if case["expect"] == "failed":
        assert st == P.FAILED
    else:
        assert st == P.FIXPOINT
        assert np.asarray(lb).tolist() == case["lb"]
        assert np.asarray(ub).tolist() == case["ub"]


MODES = pytest.mark.parametrize("mode", [dict(live=2), dict(live=1), dict(dep=1)],
                                ids=["tables", "lists", "dep"])


@MODES
@pytest.mark.parametrize("wgs", [1, 0], ids=["one_wg", "whole_gpu"])
@pytest.mark.parametrize("case", _cases("hand_searches.json"), ids=lambda c: c["name"])
def test_hand_searches_on_gpu(P, case, mode, wgs):
    say("hand search", case["name"], mode, wgs)
    extra = dict(num_wgs=1) if wgs == 1 else {}
    if case["mode"] == "enumerate":
        m = make_model(case["boxes"], case["rows"], case["reif"])
        s = P.Solver(m, sol_cap=100, **extra, **mode)
        assert s.solve(time_limit=30) == P.OUT_ALL
        sols = sorted(map(list, np.asarray(s.solutions()).tolist()))
        assert sols == case["solutions"]
        assert s.stats()["solutions"] == len(case["solutions"])
    else:
        d = case["rcpsp"]
        m = I.rcpsp_model(d["durations"], [tuple(e) for e in d["edges"]],
                          d["demands"], d["capacities"])
        s = P.Solver(m, **extra, **mode)
        assert s.solve(time_limit=30) == P.OUT_OPTIMAL
        obj, vals = s.best()
        assert obj == case["optimum"]
        dur = d["durations"]
        start = np.asarray(vals)[:len(dur)]
        # the schedule itself: precedences and capacities hold at every time
        for i, j in d["edges"]:
            assert start[i] + dur[i] <= start[j]
        for t in range(obj):
            run = [i for i in range(len(dur)) if start[i] <= t < start[i] + dur[i]]
            for dem, cap in zip(d["demands"], d["capacities"]):
                assert sum(dem[i] for i in run) <= cap
        assert max(start[i] + dur[i] for i in range(len(dur))) == obj
