#!/usr/bin/env python3
"""Benchmark: search nodes/s and time-to-proven-optimum on one MI355X.

Workload (one "step"): 256 instances of the synthetic project-scheduling
family - 30, 60 or 90 tasks by seed mod 3 (seeds 0..255), 4 renewable
resources of capacity 10, durations 1..10, demands 0 or 1..10 at density
0.5, precedence out-degree 1..3 - each minimising its makespan by
branch-and-bound with first-fail branching, all searched in ONE persistent
launch (the batched form: one workgroup per subproblem, a device queue of
subtrees, the launch replayed from a hipGraph), bounded by `--step-time`
seconds of device time.  The whole hot path runs in that launch (node setup,
propagation sweeps, fixed-point and failure detection, branching, the
depth-first and bound control, the subtree queue).

Printed: ONE JSON line on stdout with the contract fields plus
  roofline      the search kernel against the LDS roofline: algorithmic LDS
                bytes (propagator executions x bytes each) over the kernel's
                HIP-event time, against the LDS read peak MEASURED on this
                device (pccp_measure_lds_peaks); and the lattice joins the
                sweeps issued (LDS atomic max / min) per second against the
                measured LDS atomic peak
  cpu_baseline  the CPU oracle (C, -O3 -march=native, built on this host),
                one POSIX thread per host core, timed in C, on a bounded
                sample of the same workload
  ttpo          time to proven optimum of the instances proven in a step
  legs          c2 plain (30 tasks, one instance on the whole GPU, several
                seeds), c3 (120 tasks, its own roofline), job shops from the
                PCCP front-end
  ttpo_forms    plain vs batched vs learned time to settle a set of
                instances under the same device-time budget
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("search nodes/sec + time-to-proven-optimum; plain vs batched vs learned, "
          "1 MI355X")
# algorithmic LDS bytes per propagator execution (int32 bounds): difference
# row: lb/ub of both variables; reified overlap: lb/ub of si, sj, b; linear-
# row term: the bound entering the sum and the bound it tightens
BYTES_DIFF, BYTES_REIF, BYTES_TERM = 16, 24, 8


# HBM traffic of the search kernel from rocprofv3 counter runs (FETCH_SIZE and
# WRITE_SIZE in separate passes), per search node, for one kernel source and
# launch shape on one workload (the headline batch, or the 120-task instance).  FETCH_SIZE is scaled by 2.0 and
# WRITE_SIZE by 1.0: what a 2 GiB device copy (`--copy-calibration`) reads
# back as 1 GiB fetched and 2 GiB written.  A run whose kernel source or
# shape differs reports null.
PROFILED_TRAFFIC = [
    {"workload": "rcpsp_mixed_30_60_90tasks_4res_batch256",
     "kernel_sha256": "7197025a878158d14d2299204c0a556c7ce0fa4e08ebd26d4bb648579002a030",
     "block": 128, "desc_lds": 0, "root_lds": 0, "live": 0, "occupancy": 2, "dep": 1,
     "fetch_bytes_per_node": 745.6, "write_bytes_per_node": 275.7,
     "profile": "profiles/search_kernel_rcpsp_mixed256_wg128.md"},
    {"workload": "rcpsp_120tasks_4res_single",
     "kernel_sha256": "7197025a878158d14d2299204c0a556c7ce0fa4e08ebd26d4bb648579002a030",
     "block": 256, "desc_lds": 0, "root_lds": 0, "live": 0, "occupancy": 1, "dep": 1,
     "fetch_bytes_per_node": 20.9, "write_bytes_per_node": 756.0,
     "profile": "profiles/search_kernel_rcpsp120_single.md"},
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


def profiled_traffic(st, nodes_per_launch, workload):
    sha = kernel_sha256()
    for e in PROFILED_TRAFFIC:
        if (e["workload"], e["kernel_sha256"], e["block"], e["desc_lds"], e["root_lds"], e["live"],
                e["occupancy"], e["dep"]) == (workload, sha, st["block"], st["desc_lds"], st["root_lds"],
                                              st["live"], st["occupancy"], st["dep"]):
            return round((e["fetch_bytes_per_node"] + e["write_bytes_per_node"]) * nodes_per_launch)
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(st):
    return (st["prop_linear2"] * BYTES_DIFF + st["prop_reified"] * BYTES_REIF
            + st["prop_terms"] * BYTES_TERM)


def propagations(st):
    return st["prop_linear2"] + st["prop_reified"] + st["prop_linear"]


def roofline(bytes_, atomics, kernel_s, peaks):
    """LDS roofline of a search launch: algorithmic bytes and issued joins
    per second of kernel time against the measured peaks."""
    ach = bytes_ / kernel_s / 1e9 if kernel_s > 0 else 0.0
    aops = atomics / kernel_s / 1e9 if kernel_s > 0 else 0.0
    return {"bound": "lds", "achieved": round(ach, 1), "peak": round(peaks["read_GBs"], 1),
            "unit": "GB/s", "frac": round(ach / peaks["read_GBs"], 5),
            "atomic_achieved": round(aops, 3), "atomic_peak": round(peaks["atomic_Gops"], 1),
            "atomic_unit": "Gop/s", "atomic_frac": round(aops / peaks["atomic_Gops"], 5)}


def host_cores() -> int:
    """Cores the CPU baseline may use: the ones this process may run on,
    at most 16 (the host share of one GPU on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


# nodes per instance of the CPU sample, by task count: about one second of
# the oracle's sequential search each on a current server core
CPU_NODES = {30: 8000, 60: 2000, 90: 1000, 120: 500}


def cpu_baseline(models_by_size, threads, label, scale=1.0):
    """The oracle's sequential depth-first search (built -O3 -march=native on
    this host) on independent instances, one POSIX thread per core, timed in
    C: for each task count, `threads` instances of it searched for
    CPU_NODES[n] * scale nodes each (or to their proof); total nodes over the
    summed wall time of the three sets.  Also one thread on one instance of
    each size."""
    import oracle as O
    from oracle import build as obuild
    tmp = tempfile.mkdtemp(prefix="pccp_oracle_")
    path = obuild.build(native=True, out=os.path.join(tmp, "liboracle_native.so"))
    O.use_library(path)
    nodes = wall = one_nodes = one_wall = 0.0
    count = 0
    for n, models in sorted(models_by_size.items()):
        lim = max(1, int(CPU_NODES.get(n, 1000) * scale))
        r = O.solve_timed(models, threads, node_limit=lim)
        nodes += float(r["nodes"].sum())
        wall += r["wall_s"]
        count += len(models)
        one = O.solve_timed(models[:1], 1, node_limit=lim)
        one_nodes += float(one["nodes"].sum())
        one_wall += one["wall_s"]
    ncpu, cpu_model = host_info()
    sizes = "/".join(str(n) for n in sorted(models_by_size))
    return {"value": nodes / wall, "unit": "nodes/s", "cores": threads, "kind": "oracle",
            "sample": f"{label}: {count} instances ({sizes} tasks, {threads} of each size), "
                      f"{', '.join(f'{n}: {max(1, int(CPU_NODES.get(n, 1000) * scale))}' for n in sorted(models_by_size))} "
                      f"nodes each (or to proof), {threads} threads, {wall:.1f} s wall, "
                      f"oracle built -O3 -march=native",
            "nproc": ncpu, "cpu_model": cpu_model,
            "single_core": {"value": one_nodes / one_wall, "cores": 1,
                            "sample": f"one instance of each size, {one_wall:.1f} s"}}


def plain_leg(models, limit, cfg, peaks):
    """Each instance alone on the whole GPU (the plain form): node and
    propagation rates, and the LDS roofline of the launches together."""
    from paper_2207_12116_amd import pccp
    rows, nodes, props, byt, atom, kern, wall = [], 0, 0, 0, 0, 0.0, 0.0
    for i, m in enumerate(models):
        s = pccp.Solver(m, config=cfg)
        t0 = time.perf_counter()
        out = s.solve(pccp.MINIMIZE, time_limit=limit)
        dt = time.perf_counter() - t0
        st = s.stats()
        nodes += st["nodes"]
        props += propagations(st)
        byt += algorithmic_bytes(st)
        atom += st["atomics"]
        kern += st["kernel_ms"] / 1e3
        wall += dt
        rows.append({"nodes_per_s": round(st["nodes"] / dt, 1), "outcome": pccp.OUTCOME_NAMES[out],
                     "best": st["best"], "time_s": round(dt, 3)})
    return {"nodes_per_s": round(nodes / wall, 1), "propagations_per_s": round(props / wall, 1),
            "roofline": roofline(byt, atom, kern, peaks), "grid": st["grid"], "block": st["block"],
            "per_instance": rows}


def enumerate_leg(seeds, limit):
    """The tiny CSP (8 variables over [0, 20], 12 precedences, one weighted
    sum; every solution enumerated), each seed alone on the whole GPU with
    the library's default launch: nodes/s and time to exhaust the tree."""
    from paper_2207_12116_amd import instances as I, pccp
    rows, nodes, wall = [], 0, 0.0
    for sd in seeds:
        s = pccp.Solver(I.tiny_csp(sd))
        t0 = time.perf_counter()
        out = s.solve(pccp.ENUMERATE, time_limit=limit)
        dt = time.perf_counter() - t0
        st = s.stats()
        nodes += st["nodes"]
        wall += dt
        rows.append({"seed": sd, "outcome": pccp.OUTCOME_NAMES[out], "nodes": st["nodes"],
                     "solutions": st["solutions"], "sol_hash": st["sol_hash"],
                     "ttpo_ms": round(st["ttpo_ms"], 3) if out == pccp.OUT_ALL else None})
    return {"nodes_per_s": round(nodes / wall, 1), "per_instance": rows,
            "grid": st["grid"], "block": st["block"]}


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


def ttpo_forms(models, per_limit, cfg, weights, label):
    """Time to settle a set of instances in three forms under the same
    device-time budget (per_limit seconds per instance):
      plain    one whole-GPU launch per instance, each limited to per_limit;
               the set is settled after the sum of the launches
      batched  one launch over every instance, limited to per_limit x count
      learned  batched, branching on the trained network
    Per-instance TTPO is device-clock time from its launch's start to its
    proof.  Optima proven by two forms must agree."""
    from paper_2207_12116_amd import learn, pccp
    solved = (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT)

    def summary(outs, sts, total):
        ok = [o in solved for o in outs]
        tt = [round(x["ttpo_ms"], 3) if o else None for o, x in zip(ok, sts)]
        return {"proven": int(sum(ok)), "instances": len(ok), "total_s": round(total, 3),
                "nodes": int(sum(x["nodes"] for x in sts)), "ttpo_ms": tt,
                "best": [x["best"] for x in sts]}

    res = {"set": label, "per_instance_limit_s": per_limit}
    outs, sts, total = [], [], 0.0
    for m in models:
        s = pccp.Solver(m, config=cfg)
        o = s.solve(pccp.MINIMIZE, time_limit=per_limit)
        st = s.stats()
        outs.append(o)
        sts.append(st)
        total += min(st["ttpo_ms"] / 1e3, per_limit) if o in solved else per_limit
    res["plain"] = summary(outs, sts, total)
    for form in ("batched", "learned"):
        solvers = [pccp.Solver(m, config=cfg) for m in models]
        if form == "learned":
            if not os.path.exists(weights):
                res[form] = None
                continue
            mlp = learn.network(weights)
            for s in solvers:
                learn.attach(s, mlp)
        outs = pccp.batch_solve(solvers, pccp.MINIMIZE, config=cfg,
                                time_limit=per_limit * len(models))
        sts = [s.stats() for s in solvers]
        res[form] = summary(outs, sts, sts[0]["kernel_ms"] / 1e3)
    # optima proven by two forms agree
    for a in ("batched", "learned"):
        if res.get(a) is None:
            continue
        for i, (x, y) in enumerate(zip(res["plain"]["ttpo_ms"], res[a]["ttpo_ms"])):
            if x is not None and y is not None:
                assert res["plain"]["best"][i] == res[a]["best"][i], (a, i)
    return res


def fixpoint_leg(peaks, nbox=4096, fbox=1024, reps=5):
    """Fixed points of many boxes per launch, inputs resident in HBM, timed
    with HIP events on the solvers' stream (the current one):
      every_table  the 30-task instance's root box, every table every sweep
      incremental  its root fixed point joined with one random decision per
                   box (a start time split at a random point),
                   dependency-driven
      float        a sparse system over the reals (1000 variables, 2000 rows
                   of 2-6 terms, built around a point that satisfies every
                   row), its root box (random sub-boxes of such a system are
                   nearly all empty), outward-rounded linear tells on float32
                   bounds
    The float kernel's algorithmic LDS bytes: every sweep runs every row,
    and a row reads the bounds of each of its L terms once (8 bytes each),
    so 8 L bytes per row and sweep; the tells' atomics are not counted."""
    import numpy as np
    import torch
    from paper_2207_12116_amd import instances as I, pccp
    rng = np.random.default_rng(11)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    out = {}
    m = I.rcpsp(30, 0)
    s = pccp.Solver(m)
    V = m.nvars
    lbs = torch.tensor(np.tile(m.lb, (nbox, 1)), dtype=torch.int32, device="cuda")
    ubs = torch.tensor(np.tile(m.ub, (nbox, 1)), dtype=torch.int32, device="cuda")
    olb, oub = torch.empty_like(lbs), torch.empty_like(ubs)
    st = torch.zeros(nbox, dtype=torch.int32, device="cuda")
    sw = torch.zeros(nbox, dtype=torch.int32, device="cuda")
    t = timed(lambda: s.propagate_batch(lbs, ubs, olb, oub, st, sw))
    out["every_table"] = {"boxes": nbox, "variables": V, "s_per_launch": round(t, 6),
                          "boxes_per_s": round(nbox / t, 1),
                          "sweeps_per_box": float(sw.float().mean().item())}
    # parents: the root fixed point; decisions: random start-time splits
    root_l, root_u = olb[:1].clone(), oub[:1].clone()
    plb, pub = root_l.repeat(nbox, 1).contiguous(), root_u.repeat(nbox, 1).contiguous()
    rl, ru = root_l[0].cpu().numpy(), root_u[0].cpu().numpy()
    dec = np.asarray(m.decision)
    xs = rng.choice(dec, size=nbox)
    dlo, dhi = np.empty(nbox, np.int32), np.empty(nbox, np.int32)
    for k, x in enumerate(xs):
        lo, hi = int(rl[x]), int(ru[x])
        mid = lo + int(rng.integers(0, max(1, hi - lo)))
        if rng.random() < 0.5:
            dlo[k], dhi[k] = lo, mid
        else:
            dlo[k], dhi[k] = mid + 1, hi
    dv = torch.tensor(xs.astype(np.int32), device="cuda")
    dl, dh = torch.tensor(dlo, device="cuda"), torch.tensor(dhi, device="cuda")
    t = timed(lambda: s.propagate_batch_incr(plb, pub, dv, dl, dh, olb, oub, st, sw))
    out["incremental"] = {"boxes": nbox, "s_per_launch": round(t, 6),
                          "boxes_per_s": round(nbox / t, 1),
                          "sweeps_per_box": float(sw.float().mean().item()),
                          "failed": int((st == 1).sum().item())}
    # float boxes
    fm = I.float_network(1000, 2)
    fs = pccp.FSolver(fm)
    flb = np.tile(fm.lb, (fbox, 1)).astype(np.float32)
    fub = np.tile(fm.ub, (fbox, 1)).astype(np.float32)
    tl, tu = torch.tensor(flb, device="cuda"), torch.tensor(fub, device="cuda")
    ol, ou = torch.empty_like(tl), torch.empty_like(tu)
    fst = torch.zeros(fbox, dtype=torch.int32, device="cuda")
    fsw = torch.zeros(fbox, dtype=torch.int32, device="cuda")
    t = timed(lambda: fs.propagate_batch(tl, tu, ol, ou, fst, fsw))
    L = np.diff(np.asarray(fm.row_ptr, dtype=np.int64))
    per_sweep = int(8 * L.sum())
    sweeps = float(fsw.sum().item())
    fb = per_sweep * sweeps
    out["float"] = {"boxes": fbox, "variables": fm.nvars, "rows": fm.nrows,
                    "s_per_launch": round(t, 6), "boxes_per_s": round(fbox / t, 1),
                    "sweeps_per_box": round(sweeps / fbox, 2),
                    "failed": int((fst == 1).sum().item()),
                    "lds_bytes_per_launch": int(fb),
                    "lds_GBs": round(fb / t / 1e9, 1),
                    "lds_frac": round(fb / t / 1e9 / peaks["read_GBs"], 5)}
    fs.close()
    return out


def mlp_leg(nodes=4096, cmin=10, cmax=90, steps=20):
    """The learned rule's kernels on synthetic traces of the training shape
    (4096 nodes, 10-90 candidates each, 6 features, a target distribution
    per node): training steps (forward and per-node cross-entropy, backward,
    reduce and Adam, BF16 refresh) and BF16 scoring, timed with HIP events.
    Work per candidate: the forward pass is 2*6*64 + 64 + 2*64 = 960 flops
    (FP32), the backward about twice that; so about 2.9 kflop per candidate
    per training step, 0.96 kflop per scored candidate."""
    import numpy as np
    import torch
    from paper_2207_12116_amd import pccp
    rng = np.random.default_rng(5)
    cnt = rng.integers(cmin, cmax + 1, size=nodes)
    off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    C = int(off[-1])
    feat = rng.random((C, 6), dtype=np.float32)
    tgt = np.empty(C, np.float32)
    for i in range(nodes):
        z = rng.random(cnt[i]).astype(np.float32)
        tgt[off[i]:off[i + 1]] = z / z.sum()
    f = torch.tensor(feat, device="cuda")
    o = torch.tensor(off, device="cuda")
    t = torch.tensor(tgt, device="cuda")
    sc = torch.empty(C, dtype=torch.float32, device="cuda")
    mlp = pccp.MLP(seed=1)
    mlp.train_step(f, o, t, cmax, 1e-3)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        mlp.train_step(f, o, t, cmax, 1e-3)
    e1.record()
    torch.cuda.synchronize()
    ts = e0.elapsed_time(e1) / 1e3 / steps
    mlp.scores(f, sc)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        mlp.scores(f, sc)
    e1.record()
    torch.cuda.synchronize()
    tsc = e0.elapsed_time(e1) / 1e3 / steps
    mlp.close()
    return {"nodes": nodes, "candidates": C,
            "train_step_ms": round(ts * 1e3, 3), "train_candidates_per_s": round(C / ts, 1),
            "train_TFLOPs": round(2.88e3 * C / ts / 1e12, 3),
            "score_ms": round(tsc * 1e3, 3), "score_candidates_per_s": round(C / tsc, 1),
            "score_TFLOPs": round(0.96e3 * C / tsc / 1e12, 3),
            "fp32_vector_peak_TFLOPs": 157.3}


def learned_120_leg(seeds, limit, cfg, weights, scan):
    """The learned branching rule against first-fail on held-out 120-task
    instances (training used 30- and 60-task seeds), each form on the whole
    GPU for `limit` seconds per instance.  `scan` is what the oracle proved
    of the same seeds within its node budget (the evaluation set of proven
    instances is empty when it proved none).  Optima proven by both forms
    must agree."""
    from paper_2207_12116_amd import instances as I, learn, pccp
    mlp = learn.network(weights) if os.path.exists(weights) else None
    rows = []
    for sd in seeds:
        m = I.rcpsp(120, sd)
        row = {"seed": sd}
        for form in ("first_fail", "learned"):
            if form == "learned" and mlp is None:
                row[form] = None
                continue
            s = pccp.Solver(m, config=cfg)
            if form == "learned":
                learn.attach(s, mlp)
            out = s.solve(pccp.MINIMIZE, time_limit=limit)
            st = s.stats()
            row[form] = {"outcome": pccp.OUTCOME_NAMES[out], "best": st["best"],
                         "nodes": st["nodes"], "ttpo_ms": round(st["ttpo_ms"], 3)
                         if out in (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT) else None}
        a, b = row["first_fail"], row.get("learned")
        if b and a["ttpo_ms"] is not None and b["ttpo_ms"] is not None:
            assert a["best"] == b["best"], sd
        rows.append(row)
    found = {f: sum(r[f] is not None and r[f]["best"] is not None for r in rows)
             for f in ("first_fail", "learned")}
    better = sum(1 for r in rows if r.get("learned") and r["learned"]["best"] is not None and
                 (r["first_fail"]["best"] is None or r["learned"]["best"] < r["first_fail"]["best"]))
    return {"seeds": f"{seeds[0]}-{seeds[-1]}", "limit_s": limit, "instances": rows,
            "with_incumbent": found, "learned_better_incumbent": better, "oracle_scan": scan}


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
    ap.add_argument("--workload", choices=("mixed", "single120"), default="mixed",
                    help="mixed: the 256-instance 30/60/90-task batch (the headline); single120: "
                         "one 120-task instance (seed 0) on the whole GPU per step, for profiles")
    ap.add_argument("--batch", type=int, default=256, help="instances (seeds 0..batch-1)")
    ap.add_argument("--step-time", type=float, default=3.0)
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-scale", type=float, default=1.0,
                    help="scales the CPU sample's nodes per instance")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="0 = the cores this process may run on, at most 16")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the plain 30-task, 120-task and job-shop legs")
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
    ap.add_argument("--max-depth", type=int, default=4096,
                    help="decision-stack capacity per workgroup")
    ap.add_argument("--no-ttpo", action="store_true")
    ap.add_argument("--ttpo-n", type=int, default=30)
    ap.add_argument("--ttpo-seeds", type=int, default=16)
    ap.add_argument("--ttpo-limit", type=float, default=1.0,
                    help="device seconds per instance in the TTPO comparison (the paper's "
                         "protocol for 30-task instances is 30)")
    ap.add_argument("--fixpoints-only", action="store_true",
                    help="run only the fixed-point batches (every table, incremental, float) "
                         "and the learned rule's kernels; print their figures as one JSON line")
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
    if args.fixpoints_only:
        from paper_2207_12116_amd import pccp
        print(json.dumps({"fixpoint_batches": fixpoint_leg(pccp.lds_peaks()),
                          "mlp_train_score": mlp_leg()}), flush=True)
        return
    from paper_2207_12116_amd import autotune, instances as I, pccp

    peaks = pccp.lds_peaks()
    log(f"measured LDS peaks: {peaks}")
    if args.workload == "single120":
        seeds = [0]
        log("building the 120-task instance, seed 0")
        models = [I.rcpsp(120, 0)]
    else:
        seeds = list(range(args.batch))
        log(f"building {args.batch} instances of 30/60/90 tasks")
        models = [I.rcpsp(I.batch_sizes(s), s) for s in seeds]
    tuned = None
    if args.wg == 0 and not args.no_autotune:
        # tuned on the whole batch, with the finalists timed over as long a
        # launch as a step: short runs on a subset ranked the high-occupancy
        # build above the normal one (125 against 111 M nodes/s on 16 of the
        # instances in 1.2 s runs; 95 against 114 in the 3 s steps over all
        # 256, where its shorter work lists overflow more as the search deepens)
        cfg, rep = autotune.tune(models, pccp.MINIMIZE, budget_s=args.step_time / 4, cache_path=None,
                                 wg_sizes=(128, 256, 512), max_depth=args.max_depth, log=log)
        if args.workload == "single120":
            log("the 120-task instance is tuned alone")
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
    tot_nodes = tot_bytes = tot_atom = tot_props = 0
    tot_kernel_ms = 0.0
    last = None
    t0 = time.perf_counter()
    for k in range(args.steps):
        outs, sts = step()
        nodes = sum(s["nodes"] for s in sts)
        tot_nodes += nodes
        tot_bytes += sum(algorithmic_bytes(s) for s in sts)
        tot_atom += sum(s["atomics"] for s in sts)
        tot_props += sum(propagations(s) for s in sts)
        tot_kernel_ms += sts[0]["kernel_ms"]
        last = (outs, sts)
        log(f"step {k}: nodes {nodes} kernel {sts[0]['kernel_ms']:.1f} ms "
            f"proven {sum(o in (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT) for o in outs)}/{len(outs)}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = tot_nodes / wall
    outs, sts = last
    solved = (pccp.OUT_OPTIMAL, pccp.OUT_UNSAT)
    proven = [s["ttpo_ms"] for o, s in zip(outs, sts) if o in solved]
    by_size = {}
    for sd, o, s in zip(seeds, outs, sts):
        size = 120 if args.workload == "single120" else I.batch_sizes(sd)
        b = by_size.setdefault(str(size), {"instances": 0, "proven": 0, "nodes": 0})
        b["instances"] += 1
        b["proven"] += o in solved
        b["nodes"] += s["nodes"]
    ttpo = {"proven": len(proven), "instances": len(outs), "limit_s": args.step_time,
            "median_ms": statistics.median(proven) if proven else None,
            "geomean_ms": math.exp(sum(math.log(max(p, 1e-3)) for p in proven) / len(proven))
            if proven else None,
            "total_s_with_limit": round(sum(proven) / 1e3 + (len(outs) - len(proven)) * args.step_time, 3),
            "by_size": by_size,
            "with_incumbent": sum(s["best"] is not None for s in sts)}
    kernel_s = tot_kernel_ms / 1e3
    workload = (f"rcpsp_mixed_30_60_90tasks_4res_batch{args.batch}" if args.workload == "mixed"
                else "rcpsp_120tasks_4res_single")
    roof = roofline(tot_bytes, tot_atom, kernel_s, peaks)
    roof.update({"traffic": profiled_traffic(sts[0], tot_nodes / args.steps, workload),
                 "kernel": "search_kernel", "kernel_ms_avg": round(tot_kernel_ms / args.steps, 3),
                 "bytes_per_launch": tot_bytes // args.steps,
                 "atomics_per_launch": tot_atom // args.steps,
                 "nodes_per_launch": tot_nodes // args.steps,
                 "peaks_measured": {"read_GBs": round(peaks["read_GBs"], 1),
                                    "atomic_Gops": round(peaks["atomic_Gops"], 1),
                                    "atomic_ret_Gops": round(peaks["atomic_ret_Gops"], 1)}})

    legs = None
    if not args.no_legs:
        log("plain: 30-task instances, one at a time on the whole GPU")
        c2 = [I.rcpsp(30, s) for s in range(4)]
        # tuned on one instance alone (the plain form), finalists over 2 s
        c2cfg, c2rep = autotune.tune(c2[:1], pccp.MINIMIZE, budget_s=0.5, cache_path=None,
                                     wg_sizes=(128, 256, 512), max_depth=args.max_depth, log=log)
        legs = {"c2_plain_30tasks": plain_leg(c2, 3.0, c2cfg, peaks)}
        legs["c2_plain_30tasks"]["config"] = {"wg_size": c2cfg.wg_size, "prop": c2rep["prop"],
                                              "occupancy": c2cfg.occupancy, "seeds": "0-3",
                                              "limit_s": 3.0}
        log(f"c2: {legs['c2_plain_30tasks']}")
        log("tiny CSP, every solution, whole GPU")
        legs["c1_enumerate"] = enumerate_leg([0, 1, 2, 3], 30.0)
        log(f"c1: {legs['c1_enumerate']}")
        log("120-task instance, whole GPU")
        c3m = [I.rcpsp(120, 0)]
        c3cfg, c3rep = autotune.tune(c3m, pccp.MINIMIZE, budget_s=0.5, cache_path=None,
                                     wg_sizes=(128, 256, 512), max_depth=args.max_depth, log=log)
        legs["c3_120tasks"] = plain_leg(c3m, 3.0, c3cfg, peaks)
        legs["c3_120tasks"]["config"] = {"wg_size": c3cfg.wg_size, "prop": c3rep["prop"],
                                         "occupancy": c3cfg.occupancy, "seed": 0, "limit_s": 3.0}
        log(f"c3: {legs['c3_120tasks']}")
        log("job shops 10x10 from the PCCP front-end, 16 in one launch")
        jsm = [I.jobshop(10, 10, s) for s in range(16)]
        jscfg, jsrep = autotune.tune(jsm, pccp.MINIMIZE, budget_s=0.3, cache_path=None,
                                     wg_sizes=(128, 256), max_depth=args.max_depth, log=log)
        legs["jobshop_10x10_batch16"] = jobshop_leg(jsm, 3.0, jscfg)
        legs["jobshop_10x10_batch16"]["config"] = {"wg_size": jscfg.wg_size, "prop": jsrep["prop"],
                                                   "occupancy": jscfg.occupancy}
        log(f"jobshop: {legs['jobshop_10x10_batch16']}")
        log("fixed points of box batches: every table, incremental, float")
        legs["fixpoint_batches"] = fixpoint_leg(peaks)
        log(f"fixpoints: {legs['fixpoint_batches']}")
        log("learned rule: training steps and scoring on synthetic traces")
        legs["mlp_train_score"] = mlp_leg()
        log(f"mlp: {legs['mlp_train_score']}")
        from paper_2207_12116_amd import learn
        log("learned vs first-fail on held-out 120-task instances")
        legs["c5_learned_120tasks"] = learned_120_leg(
            list(range(90000, 90008)), 1.5, c3cfg, learn.DEFAULT_WEIGHTS,
            {"seeds": "90000-90031", "node_budget": 20000, "proven": 0,
             "with_incumbent": 0, "note": "python -m oracle.scan_provable --n 120 --first 90000 "
                                          "--count 32 --nodes 20000 --threads 8"})
        log(f"c5: {legs['c5_learned_120tasks']}")

    forms = None
    if not args.no_ttpo:
        from paper_2207_12116_amd import learn
        forms = {}
        # the 30-task configuration itself, and a set of smaller held-out
        # instances where proofs take milliseconds to seconds (training used
        # 30- and 60-task seeds, the recipe choice 12-16 tasks seeds 0-5)
        for key, n, first, limit in (("c2_30tasks", args.ttpo_n, 0, args.ttpo_limit),
                                     ("held_out_16tasks", 16, 200, 2.0)):
            log(f"time to proven optimum: {args.ttpo_seeds} instances of {n} tasks from seed {first}")
            tm = [I.rcpsp(n, s) for s in range(first, first + args.ttpo_seeds)]
            # one fixed launch shape for every form and set (the headline's:
            # 128 threads, normal build, dependency-driven sweeps, tables in
            # HBM/L2): a tuner ranks shapes by node rate, and on searches
            # that end in milliseconds its pick varied from run to run
            tcfg = pccp.Config(wg_size=128, desc_lds=2, root_lds=2, occupancy=2, dep=1, live=2,
                               max_depth=args.max_depth)
            f = ttpo_forms(tm, limit, tcfg, learn.DEFAULT_WEIGHTS,
                           f"{n} tasks, seeds {first}-{first + args.ttpo_seeds - 1}")
            f["config"] = {"wg_size": tcfg.wg_size, "desc_lds": tcfg.desc_lds,
                           "root_lds": tcfg.root_lds, "occupancy": tcfg.occupancy, "dep": tcfg.dep}
            forms[key] = f
            log(f"ttpo forms {key}: {json.dumps(f)}")

    cpu = None
    if not args.no_cpu:
        threads = args.cpu_threads or host_cores()
        by_size = {}
        for sd, m in zip(seeds, models):
            size = 120 if args.workload == "single120" else I.batch_sizes(sd)
            lst = by_size.setdefault(size, [])
            if len(lst) < threads:
                lst.append(m)
        log(f"cpu baseline (oracle, {threads} threads)")
        cpu = cpu_baseline(by_size, threads, "the headline batch's first seeds of each size",
                           args.cpu_scale)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "nodes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": workload,
                   "tasks": "30/60/90 by seed mod 3" if args.workload == "mixed" else 120,
                   "resources": 4, "capacity": 10,
                   "instances": len(models), "seeds": f"{seeds[0]}-{seeds[-1]}",
                   "form": "batched" if args.workload == "mixed" else "plain",
                   "branching": "first-fail",
                   "step_time_limit_s": args.step_time,
                   "grid": sts[0]["grid"], "block": sts[0]["block"],
                   "desc_lds": sts[0]["desc_lds"], "root_lds": sts[0]["root_lds"],
                   "live": sts[0]["live"], "occupancy": sts[0]["occupancy"],
                   "dep": sts[0]["dep"], "max_depth": args.max_depth,
                   "max_depth_reached": max(s["max_depth"] for s in sts),
                   "autotuned": tuned, "launch": "hipGraph"},
        "propagations_per_s": round(tot_props / wall, 1),
        "roofline": roof, "cpu_baseline": cpu, "ttpo": ttpo, "legs": legs, "ttpo_forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
