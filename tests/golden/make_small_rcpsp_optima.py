"""Write small_rcpsp_optima.json: proven optimal makespans of the held-out
small RCPSP instances (12, 14 and 16 tasks, seeds 6-11), computed by the CPU
oracle's depth-first branch-and-bound (first-fail, falling back to input
order when first-fail needs more than the node budget).  Calls only the
oracle and the seeded instance generator.

    python tests/golden/make_small_rcpsp_optima.py
"""
import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2207_12116_amd import instances as I  # noqa: E402

BUDGET = 30_000_000
INSTANCES = [(n, s) for n in (12, 14, 16) for s in range(6, 12)]


def prove(arg):
    n, s = arg
    m = I.rcpsp_model(*I.rcpsp_data(n, s)[:4])
    for br, name in ((O.FIRST_FAIL, "first-fail"), (O.INPUT_ORDER, "input-order")):
        r = O.solve(m, branching=br, node_limit=BUDGET)
        if r["outcome"] == O.OUT_OPTIMAL:
            return {"tasks": n, "seed": s, "optimum": int(r["best"]), "branching": name,
                    "oracle_nodes": int(r["nodes"])}
    raise RuntimeError(f"instance {(n, s)} not proven within {BUDGET} nodes")


def main():
    with Pool(min(8, os.cpu_count() or 1)) as p:
        rows = p.map(prove, INSTANCES)
    out = {"about": "Proven optimal makespans of the held-out small RCPSP instances "
                    "(instances.rcpsp_data(n, seed), the literal decomposition plus the "
                    "makespan rows), by the CPU oracle's exhaustive branch-and-bound; "
                    "written by make_small_rcpsp_optima.py, which calls only the oracle.",
           "node_budget": BUDGET, "cases": rows}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                           "small_rcpsp_optima.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
