"""Write expert-labelled search traces of the oracle to an .npz file.

TEST INFRASTRUCTURE / DATA PREPARATION: calls only the oracle and the
data-only instance generators.  Each spec "n:first-last:nodes" traces the
RCPSP instances of n tasks with seeds first..last for at most `nodes` search
nodes each (first-fail depth-first search with branch-and-bound; each
recorded node carries its candidates' features, their expert scores and the
expert's label).

    python -m oracle.make_traces --out traces.npz --spec 30:10000-10299:200 \\
        --spec 60:20000-20099:60 --workers 8
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _one(job):
    import oracle as O
    from paper_2207_12116_amd import instances as I
    n, seed, nodes = job
    tr = O.trace(I.rcpsp(n, seed), node_limit=nodes)
    return n, seed, tr


def parse_spec(spec):
    n, seeds, nodes = spec.split(":")
    a, b = seeds.split("-")
    return [(int(n), s, int(nodes)) for s in range(int(a), int(b) + 1)]


def make_traces(jobs, workers=8):
    feats, scores, offs, labels, inst = [], [], [0], [], []
    with Pool(workers) as pool:
        for n, seed, tr in pool.imap(_one, jobs):
            base = offs[-1]
            feats.append(tr["feat"])
            scores.append(tr["score"])
            offs.extend((tr["off"][1:] + base).tolist())
            labels.append(tr["label"])
            inst.extend([(n, seed)] * len(tr["label"]))
    feat = np.concatenate(feats) if feats else np.zeros((0, 6), np.float32)
    score = np.concatenate(scores) if scores else np.zeros(0)
    return dict(feat=feat.astype(np.float32), score=score.astype(np.float64),
                off=np.asarray(offs, dtype=np.int32),
                label=np.concatenate(labels).astype(np.int32) if labels else np.zeros(0, np.int32),
                inst=np.asarray(inst, dtype=np.int32).reshape(-1, 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--spec", action="append", required=True)
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    jobs = [j for s in args.spec for j in parse_spec(s)]
    tr = make_traces(jobs, args.workers)
    np.savez_compressed(args.out, **tr, spec=json.dumps(args.spec))
    print(f"{len(tr['label'])} nodes, {tr['feat'].shape[0]} candidates -> {args.out}")


if __name__ == "__main__":
    main()
