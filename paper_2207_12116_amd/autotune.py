"""Autotuner for the batched search launch.

For a batch of models it times a short search under each candidate launch
configuration - workgroup size x placement of the propagator tables (LDS or
HBM/L2) x placement of the subtree-root store (LDS or HBM) x item lists of
non-entailed propagators (on or off) - and keeps the one with the highest
node rate.  Results are cached per device and size
class (largest store, table sizes, mode) in a JSON file, so a later call with
the same shapes costs nothing.
"""
from __future__ import annotations

import json
import os
import time

from . import pccp

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pccp_autotune.json")
WG_SIZES = (64, 128, 256, 512, 1024)
PLACEMENTS = ((1, 1), (1, 2), (2, 1), (2, 2))   # (desc_lds, root_lds): 1 = LDS, 2 = HBM
LIVES = (1, 2)                                    # item lists on, off


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
         wg_sizes=WG_SIZES, placements=PLACEMENTS, lives=LIVES, log=None):
    """Return (Config, report) for searching `models` together in one launch."""
    key = f"{_device_name()}|{size_class(models, mode)}"
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        c = cache[key]
        return pccp.Config(**c["config"]), {"cached": True, **c}
    solvers = None
    results = []
    for wg, (d, r), lv in ((w, p, l) for w in wg_sizes for p in placements for l in lives):
        cfg = pccp.Config(wg_size=wg, desc_lds=d, root_lds=r, live=lv)
        try:
            solvers = [pccp.Solver(m, config=cfg) for m in models]
            t0 = time.perf_counter()
            pccp.batch_solve(solvers, mode, config=cfg, time_limit=budget_s)
            dt = time.perf_counter() - t0
        except pccp.PccpError as e:
            if e.code in (pccp.E_LDS_CAPACITY,):
                continue
            raise
        st = [s.stats() for s in solvers]
        nodes = sum(x["nodes"] for x in st)
        rate = nodes / dt
        results.append({"wg_size": wg, "desc_lds": d, "root_lds": r, "live": lv,
                        "nodes_per_s": rate, "grid": st[0]["grid"],
                        "placed_desc_lds": st[0]["desc_lds"],
                        "placed_root_lds": st[0]["root_lds"]})
        if log:
            log(f"autotune wg={wg} desc={d} root={r} live={lv}: {rate / 1e6:.2f} M nodes/s "
                f"(grid {st[0]['grid']})")
    if not results:
        raise RuntimeError("autotune: no configuration fits")
    best = max(results, key=lambda x: x["nodes_per_s"])
    entry = {"config": {"wg_size": best["wg_size"], "desc_lds": best["desc_lds"],
                        "root_lds": best["root_lds"], "live": best["live"]},
             "nodes_per_s": best["nodes_per_s"], "candidates": results}
    if cache_path:
        cache[key] = entry
        _store(cache_path, cache)
    return pccp.Config(**entry["config"]), {"cached": False, **entry}
