#!/usr/bin/env python3
"""Benchmark: search nodes/s and time-to-proven-optimum on one MI355X.

Workload (one "step"): the synthetic project-scheduling family with 30 tasks
and 4 resources (capacity 10, durations 1..10, demands 0 or 1..10 at density
0.5, precedence out-degree 1..3), `--batch` instances (seeds 0..batch-1),
minimise the makespan by branch-and-bound with first-fail branching.  One
step is one persistent launch that searches every instance of the batch
(the batched form), bounded by `--step-time` seconds of device time; the
whole hot path runs in it (recomputation, propagation sweeps, fixed-point and
failure detection, branching, depth-first control, the subtree queue).

Printed: ONE JSON line on stdout with the contract fields plus
  roofline      the search kernel's algorithmic LDS traffic (propagator
                executions x bytes each) over its HIP-event duration,
                against the LDS peak (256 CUs x 128 B/clk x 2.4 GHz)
  cpu_baseline  the CPU oracle on one core on a bounded sample
  plain         the same search on one instance alone (whole GPU)
  ttpo          time to proven optimum of the instances proven in a step
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("search nodes/sec + time-to-proven-optimum; plain vs batched vs learned, "
          "1 MI355X")
LDS_PEAK_GBS = 256 * 128 * 2.4  # GB/s: CUs x bytes/clk/CU x GHz
# algorithmic LDS bytes per propagator execution (int32 bounds):
# difference row: lb/ub of both variables; reified overlap: lb/ub of si, sj,
# b; linear-row term: the bound entering the sum and the bound it tightens
BYTES_DIFF, BYTES_REIF, BYTES_TERM = 16, 24, 8


# HBM traffic of the search kernel from rocprofv3 counter runs (FETCH_SIZE and
# WRITE_SIZE in separate passes), per search node, for one kernel source and
# launch shape.  FETCH_SIZE is scaled by 2.0 and WRITE_SIZE by 1.0: what a
# 2 GiB device copy (`--copy-calibration`) reads back as 1 GiB fetched and
# 2 GiB written.  A run whose kernel source or shape differs reports null.
PROFILED_TRAFFIC = [
    {"kernel_sha256": "f93944629382ade5083d7819b38a25671f393a8fe98934eecca7174463bdd410",
     "block": 256, "desc_lds": 0, "root_lds": 1, "live": 0,
     "fetch_bytes_per_node": 4.858, "write_bytes_per_node": 1.394,
     "profile": "profiles/search_kernel_rcpsp30_traffic.md"},
]
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def kernel_sha256():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2207_12116_amd", "csrc")
    for f in ("pccp_kernels.hip", "pccp_types.h"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(st, nodes_per_launch):
    sha = kernel_sha256()
    for e in PROFILED_TRAFFIC:
        if (e["kernel_sha256"], e["block"], e["desc_lds"], e["root_lds"], e["live"]) == \
                (sha, st["block"], st["desc_lds"], st["root_lds"], st["live"]):
            return round((e["fetch_bytes_per_node"] + e["write_bytes_per_node"]) * nodes_per_launch)
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(st):
    return (st["prop_linear2"] * BYTES_DIFF + st["prop_reified"] * BYTES_REIF
            + st["prop_terms"] * BYTES_TERM)


def cpu_baseline(n, seed, nodes):
    import oracle as O
    from paper_2207_12116_amd import instances as I
    model = I.rcpsp(n, seed)
    t0 = time.perf_counter()
    r = O.solve(model, node_limit=nodes)
    dt = time.perf_counter() - t0
    return {"value": r["nodes"] / dt, "unit": "nodes/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential oracle DFS on the {n}-task instance seed {seed}, "
                      f"first {r['nodes']} nodes ({dt:.1f} s)"}


def ttpo_suite(n, seeds, limit, cfg, weights):
    """Time to proven optimum of the same instances in three forms:
    plain (one launch per instance, whole GPU), batched (one launch for all)
    and learned (batched, branching on the trained network).  Instance times
    are device-clock times from launch start to proof (the limit if not
    proven); `total_s` is the time to prove the whole set: the sum of the
    plain launches, the duration of the batched launch."""
    from paper_2207_12116_amd import instances as I, learn, pccp
    models = [I.rcpsp(n, s) for s in seeds]
    solved = (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT)

    def summary(times, proven, total, best):
        g = [max(t, 1e-4) for t in times]
        return {"proven": proven, "instances": len(times), "total_s": round(total, 4),
                "sum_s": round(sum(times), 4),
                "geomean_ms": round(1e3 * math.exp(sum(math.log(x) for x in g) / len(g)), 3),
                "best": best}

    times, proven, best = [], 0, []
    for m in models:
        s = pccp.Solver(m, config=cfg)
        out = s.solve(pccp.MINIMIZE, time_limit=limit)
        st = s.stats()
        ok = out in solved
        proven += ok
        times.append(st["ttpo_ms"] / 1e3 if ok else limit)
        best.append(st["best"])
    res = {"tasks": n, "seeds": f"{seeds[0]}-{seeds[-1]}", "limit_s": limit,
           "plain": summary(times, proven, sum(times), best)}
    for form in ("batched", "learned"):
        solvers = [pccp.Solver(m, config=cfg) for m in models]
        mlp = None
        if form == "learned":
            if not os.path.exists(weights):
                res[form] = None
                continue
            mlp = learn.network(weights)
            for s in solvers:
                learn.attach(s, mlp)
        outs = pccp.batch_solve(solvers, pccp.MINIMIZE, config=cfg, time_limit=limit)
        sts = [s.stats() for s in solvers]
        t = [x["ttpo_ms"] / 1e3 if o in solved else limit for o, x in zip(outs, sts)]
        pr = sum(o in solved for o in outs)
        total = max(t) if pr == len(t) else limit
        res[form] = summary(t, pr, total, [x["best"] for x in sts])
    return res


def copy_calibration(gib=2):
    """One device-to-device copy of `gib` GiB (larger than the last-level
    cache) through an elementwise kernel: the FETCH_SIZE / WRITE_SIZE that
    rocprofv3 reports for it calibrate the counters' unit and overheads."""
    import torch
    n = gib * (1 << 30) // 4
    src = torch.empty(n, dtype=torch.int32, device="cuda")
    src.fill_(7)
    dst = torch.empty_like(src)
    flush = torch.empty(512 * (1 << 20) // 4, dtype=torch.int32, device="cuda")
    flush.fill_(1)                      # evict src from the last-level cache
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "read_bytes": n * 4, "write_bytes": n * 4}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--step-time", type=float, default=3.0)
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-nodes", type=int, default=150000)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--desc-lds", type=int, default=0, choices=(0, 1, 2),
                    help="with --wg: descriptors 0 chosen by the library, 1 LDS, 2 global")
    ap.add_argument("--root-lds", type=int, default=0, choices=(0, 1, 2),
                    help="with --wg: subtree-root store 0 chosen, 1 LDS, 2 global")
    ap.add_argument("--live", type=int, default=0, choices=(0, 1, 2),
                    help="with --wg: item lists 0 chosen, 1 on, 2 off")
    ap.add_argument("--max-depth", type=int, default=0,
                    help="decision-stack capacity per workgroup (0 = library default)")
    ap.add_argument("--no-ttpo", action="store_true")
    ap.add_argument("--ttpo-n", type=int, default=18)
    ap.add_argument("--ttpo-seeds", type=int, default=16)
    ap.add_argument("--ttpo-limit", type=float, default=2.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a 2 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        copy_calibration()
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the search runs on one MI355X and this "
              "build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2207_12116_amd import instances as I, pccp

    seeds = list(range(args.batch))
    log(f"building {args.batch} instances of {args.n} tasks")
    models = [I.rcpsp(args.n, s) for s in seeds]
    tuned = None
    if args.wg == 0 and not args.no_autotune:
        from paper_2207_12116_amd import autotune
        cfg, rep = autotune.tune(models, pccp.MINIMIZE, budget_s=0.4, cache_path=None, log=log)
        tuned = {"wg_size": cfg.wg_size, "desc_lds": cfg.desc_lds, "root_lds": cfg.root_lds,
                 "live": cfg.live, "candidates": len(rep["candidates"])}
        log(f"autotuned: {tuned}")
    else:
        cfg = pccp.Config(wg_size=args.wg, desc_lds=args.desc_lds, root_lds=args.root_lds,
                          live=args.live, max_depth=args.max_depth)
    solvers = [pccp.Solver(m, config=cfg) for m in models]

    def step():
        outs = pccp.batch_solve(solvers, pccp.MINIMIZE, config=cfg, time_limit=args.step_time)
        sts = [s.stats() for s in solvers]
        return outs, sts

    for w in range(args.warmup):
        outs, sts = step()
        log(f"warmup {w}: nodes {sum(s['nodes'] for s in sts)}")
    torch.cuda.synchronize()
    tot_nodes = tot_bytes = tot_kernel_ms = 0
    tot_props = 0
    last = None
    t0 = time.perf_counter()
    for k in range(args.steps):
        outs, sts = step()
        nodes = sum(s["nodes"] for s in sts)
        tot_nodes += nodes
        tot_bytes += sum(algorithmic_bytes(s) for s in sts)
        tot_props += sum(s["prop_linear2"] + s["prop_reified"] + s["prop_linear"] for s in sts)
        tot_kernel_ms += sts[0]["kernel_ms"]
        last = (outs, sts)
        log(f"step {k}: nodes {nodes} kernel {sts[0]['kernel_ms']:.1f} ms "
            f"proven {sum(o in (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT) for o in outs)}/{len(outs)}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = tot_nodes / wall
    outs, sts = last
    proven = [s["ttpo_ms"] for o, s in zip(outs, sts) if o in (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT)]
    ttpo = {"proven": len(proven), "instances": len(outs), "limit_s": args.step_time,
            "median_ms": statistics.median(proven) if proven else None,
            "geomean_ms": math.exp(sum(math.log(max(p, 1e-3)) for p in proven) / len(proven))
            if proven else None,
            "total_s_with_limit": (sum(proven) / 1e3 + (len(outs) - len(proven)) * args.step_time),
            "best": [s["best"] for s in sts]}
    kernel_s = tot_kernel_ms / 1e3
    achieved = tot_bytes / kernel_s / 1e9 if kernel_s > 0 else 0.0
    roofline = {"bound": "lds", "achieved": round(achieved, 1), "peak": LDS_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / LDS_PEAK_GBS, 4),
                "traffic": profiled_traffic(sts[0], tot_nodes / args.steps),
                "kernel": "search_kernel", "kernel_ms_avg": round(tot_kernel_ms / args.steps, 3),
                "bytes_per_launch": tot_bytes // args.steps,
                "nodes_per_launch": tot_nodes // args.steps}

    plain = None
    if not args.no_plain:
        s = pccp.Solver(models[0], config=cfg)
        tp = time.perf_counter()
        out = s.solve(pccp.MINIMIZE, time_limit=args.step_time)
        dtp = time.perf_counter() - tp
        st = s.stats()
        plain = {"nodes_per_s": st["nodes"] / dtp, "instance_seed": 0,
                 "outcome": pccp.OUTCOME_NAMES[out], "best": st["best"],
                 "grid": st["grid"], "time_s": round(dtp, 3)}
        log(f"plain: {plain}")

    ttpo_cmp = None
    if not args.no_ttpo:
        from paper_2207_12116_amd import learn
        log(f"time to proven optimum: {args.ttpo_seeds} instances of {args.ttpo_n} tasks")
        ttpo_cmp = ttpo_suite(args.ttpo_n, list(range(args.ttpo_seeds)), args.ttpo_limit, cfg,
                              learn.DEFAULT_WEIGHTS)
        log(f"ttpo: {json.dumps({k: v for k, v in ttpo_cmp.items()})}")

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle, 1 core)")
        cpu = cpu_baseline(args.n, 0, args.cpu_nodes)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "nodes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"rcpsp_{args.n}tasks_4res_batch{args.batch}",
                   "tasks": args.n, "resources": 4, "capacity": 10,
                   "instances": args.batch, "seeds": f"0-{args.batch - 1}",
                   "form": "batched", "branching": "first-fail",
                   "step_time_limit_s": args.step_time,
                   "grid": sts[0]["grid"], "block": sts[0]["block"],
                   "desc_lds": sts[0]["desc_lds"], "root_lds": sts[0]["root_lds"],
                   "live": sts[0]["live"],
                   "autotuned": tuned, "launch": "hipGraph"},
        "propagations_per_s": round(tot_props / wall, 1),
        "roofline": roofline, "cpu_baseline": cpu, "plain": plain, "ttpo": ttpo,
        "ttpo_forms": ttpo_cmp,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
