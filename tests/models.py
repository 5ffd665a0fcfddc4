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
