"""The seeded instance generators: determinism, shapes and the stated
distributions."""
import numpy as np
import pytest

from paper_2207_12116_amd import instances as I


def test_splitmix64_deterministic_and_uniform():
    a = I.SplitMix64(42)
    b = I.SplitMix64(42)
    xs = [a.next_u64() for _ in range(100)]
    assert xs == [b.next_u64() for _ in range(100)]
    assert len(set(xs)) == 100 and all(0 <= x < 2**64 for x in xs)
    r = I.SplitMix64(7)
    counts = np.bincount([r.below(6) for _ in range(60000)], minlength=6)
    assert counts.min() > 9400 and counts.max() < 10600


def test_tiny_csp_shape():
    for seed in range(20):
        m = I.tiny_csp(seed)
        assert m.nvars == 8 and m.nrows == 13 and m.nreif == 0
        assert np.all(m.lb == 0) and np.all(m.ub == 20)
        precs = m.meta["precedences"]
        assert len({(u, v) for u, v, _ in precs}) == 12
        assert all(1 <= d <= 5 for _, _, d in precs)
        assert all(1 <= a <= 4 for a in m.meta["weights"])
        assert m.meta["cap"] * 10 == 6 * 20 * sum(m.meta["weights"])
        # the precedence graph is acyclic (a topological order exists)
        order = list(range(8))
        succ = {v: [w for u, w, _ in precs if u == v] for v in range(8)}
        seen, onstack = set(), set()

        def dfs(v):
            onstack.add(v)
            for w in succ[v]:
                assert w not in onstack
                if w not in seen:
                    dfs(w)
            onstack.discard(v)
            seen.add(v)
        for v in order:
            if v not in seen:
                dfs(v)
        assert I.tiny_csp(seed).content_hash() == m.content_hash()


@pytest.mark.parametrize("n", [30, 60, 90, 120])
def test_rcpsp_shape(n):
    m = I.rcpsp(n, 3)
    meta = m.meta
    assert m.nvars == n + n * n + 1
    assert m.nreif == n * n
    assert meta["horizon"] == sum(meta["durations"])
    assert all(1 <= d <= 10 for d in meta["durations"])
    outdeg = np.bincount([i for i, _ in meta["edges"]], minlength=n)
    assert all(1 <= outdeg[i] <= 3 for i in range(n - 1)) and outdeg[n - 1] == 0
    assert all(i < j for i, j in meta["edges"])
    dem = np.asarray(meta["demands"])
    assert dem.shape == (4, n) and dem.min() >= 0 and dem.max() <= 10
    assert meta["capacities"] == [10] * 4
    assert m.objective == n + n * n and list(m.decision) == list(range(n))
    nprec = len(meta["edges"])
    nres_rows = int(np.sum(dem.sum(axis=1) > 0)) * n
    assert m.nrows == nprec + n + nres_rows
    assert m.nterms == 2 * (nprec + n) + int(np.count_nonzero(dem)) * n


def test_rcpsp_demand_density():
    dem = np.concatenate([np.asarray(I.rcpsp(60, s).meta["demands"]).ravel()
                          for s in range(20)])
    frac_zero = np.mean(dem == 0)
    assert 0.45 < frac_zero < 0.55
    nz = dem[dem > 0]
    assert nz.min() == 1 and nz.max() == 10


def test_float_extreme_models_valid_and_seeded():
    """float_extreme: deterministic per seed; finite bounds with lb <= ub,
    finite nonzero coefficients, distinct variables per row, finite
    right-hand sides; magnitudes reach both ends of the float32 range."""
    a, b = I.float_extreme(3), I.float_extreme(3)
    assert np.array_equal(a.coef, b.coef) and np.array_equal(a.rhs, b.rhs)
    assert not np.array_equal(I.float_extreme(4).lb, a.lb)
    for s in range(4):
        m = I.float_extreme(s)
        assert np.isfinite(m.lb).all() and np.isfinite(m.ub).all() and (m.lb <= m.ub).all()
        assert np.isfinite(m.coef).all() and (m.coef != 0).all() and np.isfinite(m.rhs).all()
        for r in range(m.nrows):
            xs = m.var[m.row_ptr[r]:m.row_ptr[r + 1]]
            assert len(set(xs.tolist())) == len(xs) >= 1
        mags = np.abs(np.concatenate([m.coef, m.lb, m.ub]))
        assert mags.max() > 1e38 and mags[mags > 0].min() < 1e-38
