"""Training driver of the learned branching rule.

Reads search traces from an .npz file (features [C, 6] float32, node
offsets [N+1] int32, the expert's score of every candidate [C] and its
label [N] int32: the candidate the expert prefers at each recorded node)
and trains the network with the library's own kernels
(pccp_mlp_train_step: forward, per-node cross-entropy against a target
distribution, backward, Adam), full batch on the GPU.  The target of a
node is the softmax of its candidates' expert scores at temperature tau
(tau = 0: one-hot on the label).  The trained parameters are written as JSON
(513 floats plus provenance) and attached to solvers with
`attach(solver, mlp)`.

    python -m paper_2207_12116_amd.learn --traces traces.npz --out weights.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import pccp

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "mlp_rcpsp.json")


def load_traces(path) -> dict:
    with np.load(path, allow_pickle=False) as z:
        out = {k: z[k] for k in ("feat", "off", "label")}
        out["score"] = z["score"] if "score" in z.files else None
        out["spec"] = str(z["spec"]) if "spec" in z.files else ""
    return out


def targets(tr, tau=1.0) -> np.ndarray:
    """Per-candidate target distribution: softmax of the expert scores at
    temperature tau within each node, or one-hot on the label (tau = 0)."""
    off, lab = np.asarray(tr["off"]), np.asarray(tr["label"])
    t = np.zeros(int(off[-1]), dtype=np.float64)
    if tau <= 0 or tr.get("score") is None:
        t[off[:-1] + lab] = 1.0
        return t.astype(np.float32)
    sc = np.asarray(tr["score"], dtype=np.float64)
    for i in range(len(lab)):
        x = sc[off[i]:off[i + 1]]
        e = np.exp((x - x.max()) / tau)
        t[off[i]:off[i + 1]] = e / e.sum()
    return t.astype(np.float32)


def split(tr, val_frac=0.1):
    """Hold out the last val_frac of the nodes (contiguous, so whole instances
    mostly stay on one side)."""
    n = len(tr["label"])
    k = int(round(n * (1 - val_frac)))
    off = tr["off"]
    a = {"feat": tr["feat"][:off[k]], "off": off[:k + 1].copy(), "label": tr["label"][:k],
         "target": tr["target"][:off[k]]}
    b = {"feat": tr["feat"][off[k]:], "off": (off[k:] - off[k]).astype(np.int32),
         "label": tr["label"][k:], "target": tr["target"][off[k]:]}
    return a, b


class DeviceTraces:
    """Traces resident in device memory (torch tensors)."""

    def __init__(self, tr):
        import torch
        self.feat = torch.tensor(np.ascontiguousarray(tr["feat"], dtype=np.float32), device="cuda")
        self.off = torch.tensor(np.ascontiguousarray(tr["off"], dtype=np.int32), device="cuda")
        self.target = torch.tensor(np.ascontiguousarray(tr["target"], dtype=np.float32),
                                   device="cuda")
        self.max_cand = int(np.max(np.diff(tr["off"]))) if len(tr["label"]) else 1
        self.off_host = np.asarray(tr["off"])
        self.label_host = np.asarray(tr["label"])


def loss_of(mlp: pccp.MLP, dt: DeviceTraces) -> float:
    """Loss at the current parameters (a step with lr = 0 updates nothing)."""
    return mlp.train_step(dt.feat, dt.off, dt.target, dt.max_cand, 0.0)


def top1(mlp: pccp.MLP, dt: DeviceTraces, bf16=True) -> float:
    """Fraction of nodes where the best-scored candidate is the label."""
    import torch
    scores = torch.empty(dt.feat.shape[0], dtype=torch.float32, device="cuda")
    mlp.scores(dt.feat, scores, bf16=bf16)
    torch.cuda.synchronize()
    s = scores.cpu().numpy()
    off, lab = dt.off_host, dt.label_host
    hit = 0
    for i in range(len(lab)):
        hit += int(np.argmax(s[off[i]:off[i + 1]]) == lab[i])
    return hit / max(1, len(lab))


def train(tr, steps=400, lr=3e-3, seed=0, val_frac=0.1, tau=1.0, log=None):
    """Full-batch Adam on the training part; returns (mlp, info)."""
    tr = dict(tr)
    if "target" not in tr:
        tr["target"] = targets(tr, tau)
    a, b = split(tr, val_frac)
    dta, dtb = DeviceTraces(a), DeviceTraces(b)
    mlp = pccp.MLP(seed=seed)
    hist = []
    t0 = time.perf_counter()
    for k in range(steps):
        loss = mlp.train_step(dta.feat, dta.off, dta.target, dta.max_cand, lr)
        if k % 50 == 0 or k == steps - 1:
            rec = {"step": k, "train_loss": loss}
            if len(b["label"]):
                rec["val_loss"] = loss_of(mlp, dtb)
            hist.append(rec)
            if log:
                log(f"step {k}: {rec}")
    info = {"steps": steps, "lr": lr, "seed": seed, "tau": tau,
            "seconds": time.perf_counter() - t0,
            "train_nodes": int(len(a["label"])), "val_nodes": int(len(b["label"])),
            "train_top1": top1(mlp, dta), "val_top1": top1(mlp, dtb) if len(b["label"]) else None,
            "history": hist}
    return mlp, info


def save(path, params, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"params": [float(x) for x in params], "meta": meta}, f, indent=0)


def load_params(path=DEFAULT_WEIGHTS) -> np.ndarray:
    with open(path) as f:
        p = np.asarray(json.load(f)["params"], dtype=np.float32)
    assert p.shape == (pccp.NPARAM,)
    return p


def network(path=DEFAULT_WEIGHTS, seed=0) -> pccp.MLP:
    """An MLP on the current device holding the saved parameters."""
    mlp = pccp.MLP(seed=seed)
    mlp.set_params(load_params(path))
    return mlp


def attach(solver: pccp.Solver, mlp: pccp.MLP):
    """Make `solver` branch on the network's scores (the network must outlive
    the searches)."""
    solver.set_branching(pccp.BRANCH_MLP, mlp.weights_ptr())
    solver._mlp = mlp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--traces", required=True)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tau", type=float, default=1.0)
    args = ap.parse_args()
    tr = load_traces(args.traces)
    mlp, info = train(tr, args.steps, args.lr, args.seed, tau=args.tau,
                      log=lambda *a: print(*a, file=sys.stderr, flush=True))
    save(args.out, mlp.params(), {"traces": tr["spec"], **info})
    print(json.dumps({k: v for k, v in info.items() if k != "history"}))


if __name__ == "__main__":
    main()
