"""Scan generator seeds for instances the oracle proves within a node budget.

TEST INFRASTRUCTURE ONLY (it calls the oracle).  The learned-branching
evaluation set of the 120-task configuration is defined as the held-out
seeds from 90000 upward that the oracle proves within its budget; this
script runs that filter and prints one JSON object: the seeds tried, the
budget, the seeds proven (with optima) and the count.

    python -m oracle.scan_provable --n 120 --first 90000 --count 24 \
        --nodes 100000 --threads 6
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=120)
    ap.add_argument("--first", type=int, default=90000)
    ap.add_argument("--count", type=int, default=24)
    ap.add_argument("--nodes", type=int, default=100000)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    import oracle as O
    from paper_2207_12116_amd import instances as I
    seeds = list(range(a.first, a.first + a.count))
    models = [I.rcpsp(a.n, s) for s in seeds]
    r = O.solve_timed(models, a.threads, node_limit=a.nodes)
    proven = [(s, b) for s, o, b in zip(seeds, r["outcome"], r["best"])
              if o in (O.OUT_OPTIMAL, O.OUT_UNSAT)]
    print(json.dumps({"tasks": a.n, "seeds": f"{seeds[0]}-{seeds[-1]}", "node_budget": a.nodes,
                      "threads": a.threads, "proven": len(proven),
                      "proven_seeds": [s for s, _ in proven],
                      "optima": [b for _, b in proven],
                      "with_incumbent": sum(b is not None for b in r["best"]),
                      "best": r["best"], "wall_s": round(r["wall_s"], 1),
                      "nodes_per_s_per_thread": round(float(r["nodes"].sum() / r["secs"].sum()), 1)}))


if __name__ == "__main__":
    main()
