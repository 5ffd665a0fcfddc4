"""The boundary calls added around the search, through the C-ABI on the GPU:
  - a solver built from a model file (written by the generator module, read
    by pccp_model_load_file) gives the oracle's fixed point and search;
  - pccp_get_solution_hash equals the oracle's solution-set hash;
  - the lattice-join counter lies between one join per node and the most
    tells the executed propagators can make;
  - the LDS peak measurement returns rates in a plausible range for the
    device's compute units and clock."""
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


def test_solver_from_model_file(P, tmp_path):
    for model in (I.rcpsp(30, 4), I.tiny_rcpsp(7, 2)):
        path = str(tmp_path / "m.pccp")
        I.save_model(model, path)
        h = P.ModelHandle.from_file(path)
        s = P.Solver(model, handle=h)
        st, lb, ub = s.propagate()
        ref = O.propagate(I.load_model(path))
        assert st == ref[0] and np.array_equal(lb, ref[1]) and np.array_equal(ub, ref[2])
    r = O.solve(model)
    s1 = P.Solver(model, handle=h, num_wgs=1)
    assert s1.solve(time_limit=60) == P.OUT_OPTIMAL
    st = s1.stats()
    assert (st["nodes"], st["fails"], st["best"]) == (r["nodes"], r["fails"], r["best"])


@pytest.mark.parametrize("seed", [1, 4])
def test_solution_hash_matches_oracle(P, seed):
    model = I.tiny_csp(seed, dom=11)
    ref = O.solve(model)
    s = P.Solver(model)
    assert s.solve(time_limit=60) == P.OUT_ALL
    assert s.solution_hash() == s.stats()["sol_hash"] == ref["sol_hash"]
    assert s.solution_count() == ref["solutions"]


def test_solution_hash_before_search_is_refused(P):
    s = P.Solver(I.tiny_csp(0, dom=8))
    with pytest.raises(P.PccpError) as e:
        s.solution_hash()
    assert e.value.code == P.E_STATE


def _upper(st):
    # every join is one of a propagator's tells: at most 2 per difference
    # row, 6 per reified item, one per term of the other rows, per execution
    return 2 * st["prop_linear2"] + 6 * st["prop_reified"] + st["prop_terms"]


@pytest.mark.parametrize("kw", [dict(occupancy=1), dict(occupancy=2), dict(live=1), dict(dep=1)],
                         ids=["hiocc", "normal", "lists", "dep"])
def test_join_counter(P, kw):
    """Single-workgroup node-limited prefix (the oracle's tree): the joins
    the sweeps issued lie between one per node on average (every decision
    of the RCPSP sets off tells) and the most the executed propagators can
    issue.  The exact count depends on which lane sees which update first,
    so only these bounds are fixed."""
    model = I.rcpsp(30, 2)
    s = P.Solver(model, num_wgs=1, **kw)
    assert s.solve(node_limit=1500, time_limit=60) == P.OUT_LIMIT
    st = s.stats()
    say("joins per node", kw, st["atomics"] / st["nodes"])
    assert st["nodes"] == 1500
    assert st["nodes"] < st["atomics"] <= _upper(st)


def test_lds_peaks_plausible(P):
    import torch
    pk = P.lds_peaks()
    say("lds peaks", pk)
    props = torch.cuda.get_device_properties(0)
    assert pk["num_cus"] == props.multi_processor_count
    # between 1/16 and 4x of 128 bytes per clock per CU at 1-3 GHz
    lo = pk["num_cus"] * 128 * 1.0e9 / 16 / 1e9
    hi = pk["num_cus"] * 128 * 3.0e9 * 4 / 1e9
    assert lo < pk["read_GBs"] < hi
    assert 0 < pk["atomic_Gops"] and 0 < pk["atomic_ret_Gops"]
    assert pk["atomic_Gops"] < pk["read_GBs"]        # at most one 4-byte lane op per byte read
