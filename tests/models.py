"""Small hand-written models for tests (data only)."""
import numpy as np

from paper_2207_12116_amd.instances import Model, MODE_ENUMERATE, MODE_MINIMIZE


def make_model(boxes, rows=(), reif=(), decision=None, objective=-1, mode=None):
    """boxes: [(lb, ub)]; rows: [(coefs, vars, rhs)]; reif: [(b, si, sj, d)]."""
    lb = np.array([b[0] for b in boxes], dtype=np.int32)
    ub = np.array([b[1] for b in boxes], dtype=np.int32)
    ptr, coef, var, rhs = [0], [], [], []
    for (a, x, c) in rows:
        coef.extend(a)
        var.extend(x)
        rhs.append(c)
        ptr.append(len(coef))
    reif = np.asarray(list(reif), dtype=np.int32).reshape(-1, 4)
    if decision is None:
        decision = list(range(len(boxes)))
    if mode is None:
        mode = MODE_MINIMIZE if objective >= 0 else MODE_ENUMERATE
    i32 = lambda v: np.asarray(v, dtype=np.int32)
    return Model(lb, ub, i32(ptr), i32(coef), i32(var), i32(rhs), reif,
                 i32(decision), int(objective), int(mode), {})


def random_subbox(model, rng, frac=0.3, tight=0.5):
    """Shrink a random subset of the variables' initial intervals (data only)."""
    lb, ub = model.lb.copy(), model.ub.copy()
    for v in range(model.nvars):
        if rng.random() < frac and lb[v] < ub[v]:
            a = rng.randint(int(lb[v]), int(ub[v]))
            b = rng.randint(int(lb[v]), int(ub[v]))
            a, b = min(a, b), max(a, b)
            if rng.random() < tight:
                lb[v], ub[v] = a, b
            elif rng.random() < 0.5:
                lb[v] = a
            else:
                ub[v] = b
    return lb, ub


def jobshop_brute(jobs):
    """Minimum makespan of a job shop by enumeration of every machine's
    operation order (the disjunctive graph): for each combination of orders,
    the earliest schedule is the longest path through the job and machine
    arcs; a combination with a cycle is infeasible.  Independent of any
    constraint model."""
    import itertools
    ops = [(j, k) for j, job in enumerate(jobs) for k in range(len(job))]
    dur = {(j, k): jobs[j][k][1] for j, k in ops}
    on = {}
    for j, k in ops:
        on.setdefault(jobs[j][k][0], []).append((j, k))
    machines = sorted(on)
    best = None
    for orders in itertools.product(*[itertools.permutations(on[m]) for m in machines]):
        succ = {o: [] for o in ops}
        indeg = {o: 0 for o in ops}
        for j, job in enumerate(jobs):
            for k in range(len(job) - 1):
                succ[(j, k)].append((j, k + 1))
                indeg[(j, k + 1)] += 1
        for order in orders:
            for a, b in zip(order, order[1:]):
                succ[a].append(b)
                indeg[b] += 1
        start = {o: 0 for o in ops}
        ready = [o for o in ops if indeg[o] == 0]
        seen = 0
        while ready:
            o = ready.pop()
            seen += 1
            for q in succ[o]:
                start[q] = max(start[q], start[o] + dur[o])
                indeg[q] -= 1
                if indeg[q] == 0:
                    ready.append(q)
        if seen < len(ops):
            continue            # a cycle: these orders admit no schedule
        ms = max(start[o] + dur[o] for o in ops)
        best = ms if best is None else min(best, ms)
    return best
