"""Autotuner for the batched search launch (a cache in front of the
library's pccp_autotune).

For a batch of models the library times a short search under each candidate
launch configuration - workgroup size x placement of the propagator tables (LDS or
HBM/L2) x placement of the subtree-root store (LDS or HBM) x propagation
mode (every propagator every sweep, or dependency-driven sweeps with a
trail; item lists of non-entailed propagators on request) x kernel build
(high occupancy or normal, for workgroups of up to 256 threads) - and keeps
the one with the highest node rate.  Results are cached per device and size
class (largest store, table sizes, mode) in a JSON file, so a later call with
the same shapes costs nothing.
"""
from __future__ import annotations

import json
import os

from . import pccp

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pccp_autotune.json")
WG_SIZES = (128, 256, 512, 1024)
PLACEMENTS = ((1, 1), (1, 2), (2, 1), (2, 2))   # (desc_lds, root_lds): 1 = LDS, 2 = HBM
# propagation modes: every table every sweep, dependency-driven, item lists
MODES = {"tables": {"live": 2, "dep": 2}, "dep": {"live": 2, "dep": 1},
         "lists": {"live": 1, "dep": 2}}
DEFAULT_MODES = ("tables", "dep")


def size_class(models, mode) -> str:
    nv = max(m.nvars for m in models)
    nr = max(m.nreif for m in models)
    nt = max(m.nterms for m in models)
    # buckets of 1/8 octave keep nearby sizes together
    b = lambda x: 0 if x <= 0 else int(round(8 * __import__("math").log2(x)))
    return f"v{b(nv)}_r{b(nr)}_t{b(nt)}_m{mode}_k{len(models)}"


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(models, mode=pccp.MINIMIZE, budget_s=0.4, cache_path=DEFAULT_CACHE, force=False,
         wg_sizes=WG_SIZES, placements=PLACEMENTS, modes=DEFAULT_MODES, log=None, finalists=3,
         max_depth=0, steady=True):
    """Return (Config, report) for searching `models` together in one launch.
    The measurement is the library's pccp_autotune: every candidate's
    steady-state rate is taken from runs of budget_s / 2 and budget_s of
    device time (with steady=False: the rate of the whole run of budget_s,
    start-up included, which is what short searches to a proof see); the
    `finalists` best are timed again with runs four times as long and the
    best of those is kept, rates within 2 % counting as ties.  `placements`
    other than all four are not supported by the library's candidate set."""
    assert set(placements) == set(PLACEMENTS), "the tuner tries every placement"
    key = (f"{_device_name()}|{size_class(models, mode)}|d{max_depth}|{'+'.join(modes)}"
           f"|{'steady' if steady else 'whole'}")
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        c = cache[key]
        return pccp.Config(**c["config"]), {"cached": True, **c}
    bits = {"tables": 1, "dep": 2, "lists": 4}
    opts = pccp.TuneOpts(budget_s=budget_s, whole_run=0 if steady else 1, finalists=finalists,
                         modes=sum(bits[m] for m in modes),
                         wg_sizes=sum(1 << (w.bit_length() - 7) for w in wg_sizes),
                         max_depth=max_depth)
    solvers = [pccp.Solver(m, max_depth=max_depth) for m in models]
    best, cands = pccp.autotune(solvers, mode, opts)
    results = []
    for c in cands:
        cf = c["config"]
        prop = "dep" if cf["dep"] == 1 else ("lists" if cf["live"] == 1 else "tables")
        x = {"wg_size": cf["wg_size"], "desc_lds": cf["desc_lds"], "root_lds": cf["root_lds"],
             "prop": prop, "occupancy": cf["occupancy"], "nodes_per_s": c["nodes_per_s"],
             "nodes_per_s_long": c["nodes_per_s_long"], "grid": c["grid"], "status": c["status"]}
        results.append(x)
        if log and c["status"] == pccp.OK:
            log(f"autotune wg={x['wg_size']} desc={x['desc_lds']} root={x['root_lds']} "
                f"prop={prop} occ={x['occupancy']}: {x['nodes_per_s'] / 1e6:.2f} M nodes/s "
                f"(grid {x['grid']})" + (f", long {x['nodes_per_s_long'] / 1e6:.2f}"
                                         if x["nodes_per_s_long"] else ""))
    prop = "dep" if best.dep == 1 else ("lists" if best.live == 1 else "tables")
    entry = {"config": {"wg_size": best.wg_size, "desc_lds": best.desc_lds,
                        "root_lds": best.root_lds, "occupancy": best.occupancy,
                        "max_depth": max_depth, **MODES[prop]},
             "prop": prop,
             "nodes_per_s": max(x["nodes_per_s"] for x in results if x["status"] == pccp.OK),
             "candidates": [x for x in results if x["status"] == pccp.OK]}
    if cache_path:
        cache[key] = entry
        _store(cache_path, cache)
    return pccp.Config(**entry["config"]), {"cached": False, **entry}
