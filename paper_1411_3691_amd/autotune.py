"""Schedule autotuner for batched jobs, with a JSON cache.

    from paper_1411_3691_amd import autotune
    sched = autotune.tune(plans, T, "tree", S, w_src, w_snk, cache="tune.json")
    batch = mhc.Batch(plans, T, "tree", sched)

A batch's schedule (``mhc_schedule``: kernel family, persistent workgroups
per compute unit, work items per tile) changes only its speed, never its
result beyond summation order.  ``tune`` times each candidate schedule on
the caller's own inputs (one graph capture and a few replays each) and
keeps the fastest; the choice is stored under a key made of the jobs'
shapes, so a later batch of the same shapes reads it back without timing.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import sys
import time

# The multi-row group kernels take their tiles from the plans, so only the
# persistent workgroups per compute unit remain to choose for them (0: as
# many as stay resident, the library's choice); "group" forces the
# one-row-per-lane kernels, whose items per tile are then tried too.
DEFAULT_GRID = {
    "kernel": ["auto"],
    "blocks_per_cu": [0, 1, 2],
    "items_per_tile": [0],
}


def shape_key(plans, T, method: str) -> str:
    """Key of a batch: method and, per job, (flavour blocks, M, source and
    sink term counts, slices)."""
    parts = [method]
    for p, t in zip(plans, T):
        parts.append(f"{tuple(p.snk.nf)}:{p.M}:{p.n_src}:{p.n_snk}:{int(t)}")
    return hashlib.sha1("|".join(parts).encode()).hexdigest()


def candidates(plans, grid: dict | None = None) -> list[dict]:
    """Candidate schedules; the one-matrix-per-lane family is offered only
    when every job can take it."""
    g = dict(DEFAULT_GRID)
    g.update(grid or {})
    lane_ok = all(len(set(p.snk.nf)) == 1 and p.snk.nf[0] <= 8 for p in plans)
    kernels = [k for k in g["kernel"] if k != "lane" or lane_ok]
    return [dict(kernel=k, blocks_per_cu=b, items_per_tile=i)
            for k, b, i in itertools.product(kernels, g["blocks_per_cu"],
                                             g["items_per_tile"])]


def load_cache(path: str | None) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data if isinstance(data, dict) else {}


def store_cache(path: str, key: str, entry: dict) -> None:
    data = load_cache(path)
    data[key] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached(plans, T, method: str, cache: str | None) -> dict | None:
    """The schedule stored in ``cache`` for this batch's shapes, or None (the
    library then chooses); never times anything."""
    hit = load_cache(cache).get(shape_key(plans, T, method))
    return dict(hit["schedule"]) if hit is not None else None


def tune(plans, T, method, S, w_src, w_snk, cache: str | None = None,
         grid: dict | None = None, reps: int = 3, verbose: bool = False) -> dict:
    """The fastest schedule for this batch (read from ``cache`` when the
    same shapes were tuned before).  Every candidate runs on the given
    device tensors; timing uses events on torch's current stream."""
    import torch

    from . import mhc

    key = shape_key(plans, T, method)
    hit = load_cache(cache).get(key)
    if hit is not None:
        return dict(hit["schedule"])
    C = [torch.empty(int(t), dtype=torch.complex128, device=plans[0].device) for t in T]
    results = []
    for sc in candidates(plans, grid):
        batch = mhc.Batch(plans, T, method, sc)
        batch.run(S, w_src, w_snk, C)          # captures the graph
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            batch.run(S, w_src, w_snk, C)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        results.append((ms, sc))
        if verbose:
            print(f"autotune {sc}: {ms:.3f} ms", file=sys.stderr, flush=True)
        del batch
    ms, best = min(results, key=lambda r: r[0])
    if cache:
        store_cache(cache, key, {"schedule": best, "ms": ms, "time": time.time(),
                                 "n_jobs": len(plans), "method": method})
    return dict(best)
