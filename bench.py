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
    {"kernel_sha256": K, "block": blk, "desc_lds": dl, "root_lds": rl, "live": 0, "occupancy": oc,
     "dep": dep, "fetch_bytes_per_node": f, "write_bytes_per_node": w,
     "profile": "profiles/search_kernel_rcpsp30_traffic.md"}
    for K in ["b443c51ee41959df42d43192414e7c1dc54d61a554b1ba44484a4e7269b5b9fa"]
    for blk, dl, rl, oc, dep, f, w in [(128, 0, 0, 1, 1, 6.21, 301.0)]
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
        if (e["kernel_sha256"], e["block"], e["desc_lds"], e["root_lds"], e["live"],
                e["occupancy"], e["dep"]) == (sha, st["block"], st["desc_lds"], st["root_lds"],
                                              st["live"], st["occupancy"], st["dep"]):
            return round((e["fetch_bytes_per_node"] + e["write_bytes_per_node"]) * nodes_per_launch)
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(st):
    return (st["prop_linear2"] * BYTES_DIFF + st["prop_reified"] * BYTES_REIF
            + st["prop_terms"] * BYTES_TERM)


def _oracle_worker(args):
    n, seed, nodes = args
    import oracle as O
    from paper_2207_12116_amd import instances as I
    model = I.rcpsp(n, seed)
    t0 = time.perf_counter()
    r = O.solve(model, node_limit=nodes)
    return r["nodes"], time.perf_counter() - t0


def cpu_baseline(n, nodes, procs):
    """The oracle's sequential DFS on `procs` instances at once (one process
    each, seeds 0..procs-1), `nodes` nodes each: total nodes / wall time."""
    import multiprocessing as mp
    one_nodes, one_s = _oracle_worker((n, 0, nodes))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_worker, [(n, s, nodes) for s in range(procs)])
    wall = time.perf_counter() - t0
    tot = sum(r[0] for r in res)
    return {"value": tot / wall, "unit": "nodes/s", "cores": procs, "kind": "oracle",
            "sample": f"sequential oracle DFS, {procs} processes on the {n}-task instances "
                      f"seeds 0-{procs - 1}, first {nodes} nodes each ({wall:.1f} s wall)",
            "single_core": {"value": one_nodes / one_s, "cores": 1,
                            "sample": f"seed 0, first {one_nodes} nodes ({one_s:.1f} s)"}}


def single_instance_leg(n, seed, limit, cfg):
    """One large instance searched by the whole GPU (plain form): node and
    propagation rates and the LDS fraction."""
    from paper_2207_12116_amd import instances as I, pccp
    s = pccp.Solver(I.rcpsp(n, seed), config=cfg)
    t0 = time.perf_counter()
    out = s.solve(pccp.MINIMIZE, time_limit=limit)
    dt = time.perf_counter() - t0
    st = s.stats()
    kern = st["kernel_ms"] / 1e3
    props = st["prop_linear2"] + st["prop_reified"] + st["prop_linear"]
    ach = algorithmic_bytes(st) / kern / 1e9
    return {"tasks": n, "seed": seed, "nodes_per_s": round(st["nodes"] / dt, 1),
            "propagations_per_s": round(props / dt, 1), "outcome": pccp.OUTCOME_NAMES[out],
            "lds_achieved_GBs": round(ach, 1), "lds_frac": round(ach / LDS_PEAK_GBS, 4),
            "grid": st["grid"], "block": st["block"], "time_s": round(dt, 3)}


def jobshop_leg(models, limit, cfg):
    """Job shops compiled by the PCCP front-end (disjunctions on reified
    differences), searched in one persistent launch."""
    from paper_2207_12116_amd import pccp
    solvers = [pccp.Solver(m, config=cfg) for m in models]
    t0 = time.perf_counter()
    outs = pccp.batch_solve(solvers, pccp.MINIMIZE, config=cfg, time_limit=limit)
    dt = time.perf_counter() - t0
    sts = [s.stats() for s in solvers]
    nodes = sum(x["nodes"] for x in sts)
    return {"instances": len(models), "jobs": 10, "machines": 10,
            "nodes_per_s": round(nodes / dt, 1),
            "proven": sum(o in (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT) for o in outs),
            "best": [x["best"] for x in sts], "grid": sts[0]["grid"], "block": sts[0]["block"],
            "time_s": round(dt, 3)}


def mixed_batch_leg(count, limit, cfg):
    """`count` instances of 30, 60 and 90 tasks (by seed mod 3) in one
    persistent launch."""
    from paper_2207_12116_amd import instances as I, pccp
    models = [I.rcpsp(I.batch_sizes(s), s) for s in range(count)]
    solvers = [pccp.Solver(m, config=cfg) for m in models]
    t0 = time.perf_counter()
    outs = pccp.batch_solve(solvers, pccp.MINIMIZE, config=cfg, time_limit=limit)
    dt = time.perf_counter() - t0
    sts = [s.stats() for s in solvers]
    nodes = sum(x["nodes"] for x in sts)
    props = sum(x["prop_linear2"] + x["prop_reified"] + x["prop_linear"] for x in sts)
    proven = sum(o in (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT) for o in outs)
    return {"instances": count, "sizes": "30/60/90 by seed mod 3", "nodes_per_s": round(nodes / dt, 1),
            "propagations_per_s": round(props / dt, 1), "proven": proven,
            "with_incumbent": sum(x["best"] is not None for x in sts),
            "grid": sts[0]["grid"], "block": sts[0]["block"], "time_s": round(dt, 3)}


def ttpo_suite(n, seeds, budget, cfg, weights):
    """Time to proven optimum of the same instances in three forms, each
    instance allowed `budget` search nodes (then abandoned, outcome LIMIT).
    plain: one whole-GPU launch per instance.  batched: one launch for all
    instances.  learned: batched, branching on the trained network.
    Per-instance TTPO is device-clock time from its launch's start to proof.
    `total_s` is the device time to settle the whole set (sum of the plain
    launches; the batched launch), `wall_s` the host time of the calls;
    `plain_set_s` is the time until every instance the plain form proved is
    proven (null if one is not), counted from the start of the set."""
    from paper_2207_12116_amd import instances as I, learn, pccp
    models = [I.rcpsp(n, s) for s in seeds]
    solved = (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT)
    safety = 120.0

    def summary(ok, ttpo, total, wall, best, nodes, cover):
        return {"proven": int(sum(ok)), "instances": len(ok), "total_s": round(total, 4),
                "wall_s": round(wall, 4), "plain_set_s": None if cover is None else round(cover, 4),
                "nodes": int(nodes), "ttpo_ms": [None if t is None else round(t, 3) for t in ttpo],
                "best": best}

    ok, ttpo, best, kern, nodes = [], [], [], [], 0
    t0 = time.perf_counter()
    for m in models:
        s = pccp.Solver(m, config=cfg)
        out = s.solve(pccp.MINIMIZE, node_limit=budget, time_limit=safety)
        st = s.stats()
        ok.append(out in solved)
        ttpo.append(st["ttpo_ms"] if ok[-1] else None)
        best.append(st["best"])
        kern.append(st["kernel_ms"] / 1e3)
        nodes += st["nodes"]
    wall = time.perf_counter() - t0
    # plain set: launches run one after another, so instance i is settled at
    # the sum of the launches before it plus its own time to proof
    starts = [sum(kern[:i]) for i in range(len(kern))]
    cover = max((starts[i] + ttpo[i] / 1e3 for i in range(len(ok)) if ok[i]), default=0.0)
    res = {"tasks": n, "seeds": f"{seeds[0]}-{seeds[-1]}", "node_budget": budget,
           "plain": summary(ok, ttpo, sum(kern), wall, best, nodes, cover)}
    plain_ok = ok
    for form in ("batched", "learned"):
        solvers = [pccp.Solver(m, config=cfg) for m in models]
        if form == "learned":
            if not os.path.exists(weights):
                res[form] = None
                continue
            mlp = learn.network(weights)
            for s in solvers:
                learn.attach(s, mlp)
        t0 = time.perf_counter()
        outs = pccp.batch_solve(solvers, pccp.MINIMIZE, config=cfg, time_limit=safety,
                                inst_node_limit=budget)
        wall = time.perf_counter() - t0
        sts = [s.stats() for s in solvers]
        fok = [o in solved for o in outs]
        ft = [x["ttpo_ms"] if o else None for o, x in zip(fok, sts)]
        cov = None
        if all(f for f, p in zip(fok, plain_ok) if p):
            cov = max((t / 1e3 for t, p in zip(ft, plain_ok) if p), default=0.0)
        res[form] = summary(fok, ft, sts[0]["kernel_ms"] / 1e3, wall, [x["best"] for x in sts],
                            sum(x["nodes"] for x in sts), cov)
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
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes for the CPU baseline (0 = min(16, cores))")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the 120-task and 256-instance legs")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--desc-lds", type=int, default=0, choices=(0, 1, 2),
                    help="with --wg: descriptors 0 chosen by the library, 1 LDS, 2 global")
    ap.add_argument("--root-lds", type=int, default=0, choices=(0, 1, 2),
                    help="with --wg: subtree-root store 0 chosen, 1 LDS, 2 global")
    ap.add_argument("--live", type=int, default=0, choices=(0, 1, 2),
                    help="with --wg: item lists 0 chosen, 1 on, 2 off")
    ap.add_argument("--occupancy", type=int, default=0, choices=(0, 1, 2),
                    help="with --wg: search kernel build 0 chosen, 1 high, 2 normal")
    ap.add_argument("--dep", type=int, default=0, choices=(0, 1, 2),
                    help="with --wg: dependency-driven propagation 0/2 off, 1 on")
    ap.add_argument("--max-depth", type=int, default=0,
                    help="decision-stack capacity per workgroup (0 = library default)")
    ap.add_argument("--no-ttpo", action="store_true")
    ap.add_argument("--ttpo-n", type=int, default=18)
    ap.add_argument("--ttpo-seeds", type=int, default=16)
    ap.add_argument("--ttpo-budget", type=int, default=30_000_000,
                    help="search nodes each instance may use in the TTPO comparison")
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
                 "prop": rep["prop"], "occupancy": cfg.occupancy,
                 "candidates": len(rep["candidates"])}
        log(f"autotuned: {tuned}")
    else:
        cfg = pccp.Config(wg_size=args.wg, desc_lds=args.desc_lds, root_lds=args.root_lds,
                          live=args.live, max_depth=args.max_depth, occupancy=args.occupancy,
                          dep=args.dep)
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
        from paper_2207_12116_amd import autotune
        # tuned on whole short runs: proofs of these instances take
        # milliseconds to seconds, so the start-up counts
        tcfg, _ = autotune.tune([I.rcpsp(args.ttpo_n, s) for s in range(args.ttpo_seeds)],
                                pccp.MINIMIZE, budget_s=0.2, cache_path=None,
                                wg_sizes=(128, 256), log=log, steady=False)
        ttpo_cmp = ttpo_suite(args.ttpo_n, list(range(args.ttpo_seeds)), args.ttpo_budget, tcfg,
                              learn.DEFAULT_WEIGHTS)
        ttpo_cmp["config"] = {"wg_size": tcfg.wg_size, "desc_lds": tcfg.desc_lds,
                              "root_lds": tcfg.root_lds, "occupancy": tcfg.occupancy,
                              "dep": tcfg.dep}
        log(f"ttpo: {json.dumps({k: v for k, v in ttpo_cmp.items()})}")

    legs = None
    if not args.no_legs:
        from paper_2207_12116_amd import autotune
        log("120-task instance, whole GPU")
        c3m = [I.rcpsp(120, 0)]
        # deeper stacks than the default for the larger instances: the
        # faster modes reach depths past 1024 within the time limit (the
        # stack beyond its deepest 256 levels lives in HBM, so depth costs
        # no LDS)
        c3cfg, c3rep = autotune.tune(c3m, pccp.MINIMIZE, budget_s=0.3, cache_path=None,
                                     wg_sizes=(256, 512, 1024), max_depth=4096, log=log)
        legs = {"c3_120tasks": single_instance_leg(120, 0, 2.0, c3cfg)}
        legs["c3_120tasks"]["config"] = {"wg_size": c3cfg.wg_size, "prop": c3rep["prop"],
                                         "max_depth": c3cfg.max_depth}
        log(f"c3: {legs['c3_120tasks']}")
        log("256 mixed instances, one launch")
        c4m = [I.rcpsp(I.batch_sizes(s), s) for s in range(0, 256, 16)]
        c4cfg, c4rep = autotune.tune(c4m, pccp.MINIMIZE, budget_s=0.3, cache_path=None,
                                     wg_sizes=(256, 512, 1024), max_depth=4096, log=log)
        legs["c4_mixed256"] = mixed_batch_leg(256, 3.0, c4cfg)
        log("job shops 10x10 from the PCCP front-end, 16 in one launch")
        jsm = [I.jobshop(10, 10, s) for s in range(16)]
        jscfg, jsrep = autotune.tune(jsm, pccp.MINIMIZE, budget_s=0.3, cache_path=None,
                                     wg_sizes=(128, 256), max_depth=4096, log=log)
        legs["jobshop_10x10_batch16"] = jobshop_leg(jsm, 3.0, jscfg)
        legs["jobshop_10x10_batch16"]["config"] = {"wg_size": jscfg.wg_size, "prop": jsrep["prop"],
                                                   "occupancy": jscfg.occupancy}
        log(f"jobshop: {legs['jobshop_10x10_batch16']}")
        legs["c4_mixed256"]["config"] = {"wg_size": c4cfg.wg_size, "desc_lds": c4cfg.desc_lds,
                                         "root_lds": c4cfg.root_lds, "prop": c4rep["prop"],
                                         "max_depth": c4cfg.max_depth}
        log(f"c4: {legs['c4_mixed256']}")

    cpu = None
    if not args.no_cpu:
        procs = args.cpu_procs or min(16, os.cpu_count() or 1)
        log(f"cpu baseline (oracle, {procs} processes)")
        cpu = cpu_baseline(args.n, args.cpu_nodes, procs)

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
                   "live": sts[0]["live"], "occupancy": sts[0]["occupancy"],
                   "dep": sts[0]["dep"], "max_depth_reached": max(s["max_depth"] for s in sts),
                   "autotuned": tuned, "launch": "hipGraph"},
        "propagations_per_s": round(tot_props / wall, 1),
        "roofline": roofline, "cpu_baseline": cpu, "plain": plain, "ttpo": ttpo,
        "ttpo_forms": ttpo_cmp, "legs": legs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
