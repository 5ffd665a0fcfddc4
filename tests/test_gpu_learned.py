"""Learned branching on the GPU against the FP64 CPU oracle:
  - the in-kernel features equal the oracle's (FP32 vs FP64);
  - the training kernels' loss and gradient equal the oracle's FP64 loss and
    gradient at the same parameters;
  - training on oracle traces lowers the loss and beats chance at picking the
    expert's candidate;
  - BF16 inference picks the same candidate as the FP64 CPU network with the
    same (bf16-rounded) weights except on near-ties;
  - searches branching on the trained network reach the oracle's optimum
    (every optimum exact), and the network's gain over first-fail on held-out
    instances the oracle can prove is measured."""
import os
import random
import sys

import numpy as np
import pytest

import oracle as O
from paper_2207_12116_amd import instances as I
from tests.models import random_subbox

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


def bf16_round(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


@pytest.fixture(scope="module")
def small_traces():
    trs = [O.trace(I.rcpsp(30, s), node_limit=60) for s in range(10000, 10008)]
    feat, off, lab, sc = [], [0], [], []
    for tr in trs:
        feat.append(tr["feat"])
        sc.append(tr["score"])
        off.extend((tr["off"][1:] + off[-1]).tolist())
        lab.append(tr["label"])
    out = {"feat": np.concatenate(feat), "off": np.asarray(off, np.int32),
           "label": np.concatenate(lab).astype(np.int32), "score": np.concatenate(sc)}
    from paper_2207_12116_amd import learn
    out["target"] = learn.targets(out, tau=1.0)
    return out


@pytest.mark.parametrize("name,mk", [("rcpsp30", lambda: I.rcpsp(30, 3)),
                                      ("rcpsp60", lambda: I.rcpsp(60, 4)),
                                      ("rcpsp12", lambda: I.rcpsp_model(*I.rcpsp_data(12, 1)[:4])),
                                      ("csp", lambda: I.tiny_csp(2))])
def test_features_match_oracle(P, name, mk):
    import torch
    model = mk()
    rng = random.Random(7)
    st, lb0, ub0, _ = O.propagate(model)
    boxes = []
    for _ in range(40):
        lb, ub = random_subbox(model, rng, frac=0.1)
        s2, l2, u2, _ = O.propagate(model, np.maximum(lb, lb0), np.minimum(ub, ub0))
        if s2 == O.FIXPOINT:
            boxes.append((l2, u2))
    boxes.append((lb0, ub0))
    lbs = torch.tensor(np.stack([b[0] for b in boxes]), dtype=torch.int32, device="cuda")
    ubs = torch.tensor(np.stack([b[1] for b in boxes]), dtype=torch.int32, device="cuda")
    nd = len(model.decision)
    out = torch.zeros((len(boxes), nd, 6), dtype=torch.float32, device="cuda")
    s = P.Solver(model)
    s.node_features(lbs, ubs, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for k, (lb, ub) in enumerate(boxes):
        ref = O.features(model, lb, ub)
        assert np.allclose(got[k], ref, rtol=2e-6, atol=2e-6), (name, k)


def test_gradient_matches_oracle(P, small_traces):
    import torch
    tr = small_traces
    mlp = P.MLP(seed=3)
    p = mlp.params().astype(np.float64)
    feat = torch.tensor(tr["feat"], device="cuda")
    off = torch.tensor(tr["off"], device="cuda")
    maxc = int(np.max(np.diff(tr["off"])))
    for tgt in (O.one_hot(tr["off"], tr["label"]), tr["target"].astype(np.float64)):
        t = torch.tensor(tgt.astype(np.float32), device="cuda")
        loss = mlp.train_step(feat, off, t, maxc, 0.0)
        g = mlp.grads().astype(np.float64)
        ref_loss, ref_g = O.mlp_loss_grad(p, tr["feat"].astype(np.float64), tr["off"],
                                          tgt.astype(np.float32).astype(np.float64))
        say("loss", loss, ref_loss, "grad norm", np.linalg.norm(ref_g))
        assert abs(loss - ref_loss) <= 1e-5 * max(1.0, abs(ref_loss))
        assert np.linalg.norm(g - ref_g) <= 1e-4 * np.linalg.norm(ref_g)
        assert np.allclose(g, ref_g, rtol=1e-3, atol=1e-6 * np.abs(ref_g).max())
    # parameters unchanged by a step with lr = 0
    assert np.array_equal(mlp.params(), p.astype(np.float32))


def test_training_lowers_loss_and_beats_chance(P, small_traces):
    from paper_2207_12116_amd import learn
    mlp, info = learn.train(small_traces, steps=300, lr=3e-3, seed=1, val_frac=0.0)
    h = info["history"]
    say("history", h[0], h[-1], "top1", info["train_top1"])
    assert h[-1]["train_loss"] < 0.8 * h[0]["train_loss"]
    chance = np.mean(1.0 / np.diff(small_traces["off"]))
    assert info["train_top1"] > 2 * chance
    # the host loss at the trained parameters agrees with the device
    p = mlp.params().astype(np.float64)
    ref_loss, _ = O.mlp_loss_grad(p, small_traces["feat"].astype(np.float64),
                                  small_traces["off"], small_traces["target"].astype(np.float64))
    dt = learn.DeviceTraces(small_traces)
    assert abs(learn.loss_of(mlp, dt) - ref_loss) <= 1e-5 * max(1.0, ref_loss)


def test_bf16_scores_and_argmax(P, small_traces):
    import torch
    from paper_2207_12116_amd import learn
    mlp, _ = learn.train(small_traces, steps=100, lr=3e-3, seed=2, val_frac=0.0)
    p = mlp.params()
    pb = bf16_round(p).astype(np.float64)
    feat = torch.tensor(small_traces["feat"], device="cuda")
    sc = torch.empty(feat.shape[0], dtype=torch.float32, device="cuda")
    mlp.scores(feat, sc, bf16=True)
    torch.cuda.synchronize()
    got = sc.cpu().numpy().astype(np.float64)
    ref = O.mlp_forward(pb, small_traces["feat"].astype(np.float64))
    assert np.allclose(got, ref, rtol=1e-4, atol=1e-4)
    off = small_traces["off"]
    mism = near = 0
    for i in range(len(off) - 1):
        a, b = off[i], off[i + 1]
        r = ref[a:b]
        if np.argmax(got[a:b]) != np.argmax(r):
            mism += 1
            top2 = np.sort(r)[-2:]
            near += (top2[1] - top2[0]) < 1e-3
    say("argmax mismatches", mism, "near ties", near, "of", len(off) - 1)
    assert mism == near


def _gain_instances():
    # held out: 10-14 tasks (training used 30 and 60 tasks)
    return [(n, s) for n in (10, 12, 14) for s in range(5)]


def _provable(n, s):
    m = I.rcpsp_model(*I.rcpsp_data(n, s)[:4])
    r = O.solve(m, node_limit=300000)
    return m, r


def test_learned_search_optimum_and_gain(P):
    from paper_2207_12116_amd import learn
    if not os.path.exists(learn.DEFAULT_WEIGHTS):
        pytest.fail(f"trained weights missing: {learn.DEFAULT_WEIGHTS}")
    mlp = learn.network()
    rows = []
    for n, s in _gain_instances():
        m, r = _provable(n, s)
        if r["outcome"] != O.OUT_OPTIMAL:
            continue                         # only optima the oracle proves
        ff = P.Solver(m, num_wgs=1)
        assert ff.solve(time_limit=60, node_limit=2_000_000) == P.OUT_OPTIMAL
        ln = P.Solver(m, num_wgs=1)
        learn.attach(ln, mlp)
        out = ln.solve(time_limit=60, node_limit=2_000_000)
        assert out == P.OUT_OPTIMAL, (n, s)
        assert ff.best()[0] == r["best"] and ln.best()[0] == r["best"], (n, s)
        ok, ms = O.check_schedule(m.meta, ln.best()[1])
        assert ok and ms == r["best"]
        rows.append((n, s, r["best"], ff.stats()["nodes"], ln.stats()["nodes"]))
        say("gain", rows[-1])
    assert len(rows) >= 8
    ff_tot = sum(x[3] for x in rows)
    ln_tot = sum(x[4] for x in rows)
    say("total nodes first-fail", ff_tot, "learned", ln_tot, "ratio", ff_tot / max(1, ln_tot))
    # the trained network must not lose to first-fail overall
    assert ln_tot < ff_tot
