"""Pins of the oracle's learned-branching reference (FP64): the gradient
against central finite differences, closed-form special cases of the loss,
hand-computed features, and the expert label against a direct re-derivation
from propagate calls."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2207_12116_amd import instances as I
from tests.models import make_model


def _data(seed, nnodes=12, maxc=7):
    rng = np.random.default_rng(seed)
    counts = rng.integers(2, maxc + 1, size=nnodes)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    x = rng.normal(size=(off[-1], O.NFEAT))
    label = np.array([rng.integers(0, c) for c in counts], dtype=np.int32)
    return x, off, label


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(100 + seed)
    p = rng.normal(size=O.NPARAM) * 0.4
    x, off, lab = _data(seed)
    rng2 = np.random.default_rng(200 + seed)
    soft = rng2.random(off[-1])
    for i in range(len(off) - 1):
        soft[off[i]:off[i + 1]] /= soft[off[i]:off[i + 1]].sum()
    for tgt in (O.one_hot(off, lab), soft):
        _check_fd(p, x, off, tgt, rng)


def _check_fd(p, x, off, lab, rng):
    loss, g = O.mlp_loss_grad(p, x, off, lab)
    eps = 1e-6
    idx = rng.choice(O.NPARAM, size=80, replace=False).tolist() + [O.NPARAM - 1, 0, 384, 448]
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (O.mlp_loss_grad(pp, x, off, lab)[0] - O.mlp_loss_grad(pm, x, off, lab)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_loss_special_cases():
    x, off, lab = _data(7)
    counts = np.diff(off)
    # all weights zero: every score equals b2, the softmax is uniform
    p = np.zeros(O.NPARAM)
    p[-1] = 3.0
    loss, g = O.mlp_loss_grad(p, x, off, O.one_hot(off, lab))
    assert loss == pytest.approx(np.mean(np.log(counts)), rel=1e-12)
    assert g[-1] == pytest.approx(0.0, abs=1e-12)      # shifting all scores changes nothing
    # one hidden unit with a linear (positive) response: score = w * (b1 + x0)
    p = np.zeros(O.NPARAM)
    p[0] = 1.0                 # W1[0][0]
    p[384] = 100.0             # b1[0] keeps z > 0
    p[448] = 2.0               # w2[0]
    s = O.mlp_forward(p, x)
    assert np.allclose(s, 2.0 * (100.0 + x[:, 0]), rtol=1e-12)


def test_features_by_hand():
    # x0 in [0, 10] now [2, 6]; x1 in [0, 20] now [5, 20]; rows x0 - x1 <= -3
    # (slack (c + ub(x1) - lb(x0)) / H = (-3 + 20 - 2) / 10 = 1.5 -> capped at 1)
    # and x0 - x2 <= 1 with x2 in [0, 4] -> (1 + 4 - 2) / 10 = 0.3; reified
    # item b0 <=> (x0 <= x1 < x0 + 4) with b0 = [1, 1]; b0 appears in the row
    # 6 b0 + 3 b1 <= 10 (w(b0) = 6/10).
    boxes = [(0, 10), (0, 20), (0, 4), (0, 1), (0, 1)]
    model = make_model(boxes, [([1, -1], [0, 1], -3), ([1, -1], [0, 2], 1),
                               ([6, 3], [3, 4], 10)], [(3, 0, 1, 4)], decision=[0, 1])
    lb = np.array([2, 5, 0, 1, 0], dtype=np.int32)
    ub = np.array([6, 20, 4, 1, 1], dtype=np.int32)
    f = O.features(model, lb, ub)
    # degrees: x0: 2 rows + 1 item = 3; x1: 1 row + 1 item = 2; max = 3
    assert f[0].tolist() == pytest.approx([0.2, 0.6, 0.4, 1.0, 0.3, 4 * 0.6 / 10 + 1.0])
    assert f[1].tolist() == pytest.approx([0.25, 1.0, 0.75, 2 / 3, 1.0, 0.0])


def test_trace_labels_are_the_strong_branching_argmax():
    model = I.tiny_rcpsp(7, 4)
    tr = O.trace(model, node_limit=40)
    assert len(tr["label"]) >= 3
    # replay: the recorded nodes are those of the first-fail DFS; re-derive
    # the first node's label from its features' candidates by propagation
    st, lb, ub, _ = O.propagate(model)
    cands = tr["cand"][tr["off"][0]:tr["off"][1]]
    w0 = int(np.sum(ub.astype(np.int64) - lb))
    scores = []
    for q in cands:
        x = int(model.decision[q])
        sc = 0.0
        for side in range(2):
            l2, u2 = lb.copy(), ub.copy()
            if side == 0:
                u2[x] = lb[x]
            else:
                l2[x] = lb[x] + 1
            s2, l3, u3, _ = O.propagate(model, l2, u2)
            sc += 1e6 if s2 == O.FAILED else math.log(1 + w0 - int(np.sum(u3.astype(np.int64) - l3)))
        scores.append(sc)
    assert tr["label"][0] == int(np.argmax(scores))
    f = O.features(model, lb, ub)
    assert np.allclose(tr["feat"][:len(cands)], f[cands], atol=1e-6)
    for i in range(len(tr["label"])):
        assert 0 <= tr["label"][i] < tr["off"][i + 1] - tr["off"][i]


def test_adam_closed_forms():
    """Adam (the optimiser of the training kernels) from m = v = 0: the bias
    corrections make the first step move every parameter by exactly
    lr * g / (|g| + eps), and so does every step of a constant gradient;
    a zero gradient leaves the parameter; a restatement without the bias
    corrections (a planted mistake) moves the first step by about
    lr * 0.1 / sqrt(0.001) = 3.16 lr instead."""
    rng = np.random.default_rng(7)
    n, lr, eps = 200, 3e-3, 1e-8
    p0 = rng.normal(size=n)
    g = rng.normal(size=n) * np.exp(rng.uniform(-8, 2, size=n))
    g[:5] = 0.0
    p1, m, v = O.adam_step(p0, g, np.zeros(n), np.zeros(n), lr, 1)
    want = p0 - lr * g / (np.abs(g) + eps)
    assert np.allclose(p1, want, rtol=0, atol=1e-15)
    assert np.array_equal(p1[:5], p0[:5])
    p, mm, vv = p1, m, v
    for t in range(2, 6):
        q, mm, vv = O.adam_step(p, g, mm, vv, lr, t)
        assert np.allclose(p - q, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-16)
        p = q
    # the planted mistake: no bias correction
    planted = p0 - lr * (0.1 * g) / (np.sqrt(0.001 * g * g) + eps)
    assert not np.allclose(planted[5:], p1[5:], rtol=0, atol=1e-4)
