"""Benchmark: complex128 det-pairs/s of the update-tree contraction against
the plain batched LU on the same GPU.

    python bench.py [--steps K] [--warmup W] [--workload mid]

One step = one update-tree contraction of every (slice, source term, sink
term) pair of the workload (gather, dominator LU, column solves, sibling
ratios, weighted reduction: one call of mhc_contract).  Inputs (propagator,
weights, plan) are resident on the GPU before timing starts.  The plain
batched LU is timed the same way on the same inputs and reported beside it.

Prints one JSON line.  Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X: 256 CU x 2.4 GHz x 128 FP64 flop/clk
METRIC = "complex128 det-pairs/sec: update-tree vs plain batched LU, same GPU, 1e-11"


# Algorithmic flop counts (complex MAC = 8, complex multiply = 6, complex
# reciprocal = 6; pivot search and row exchanges are not counted).
def f_lu(n: int) -> int:
    return 8 * (n - 1) * n * (2 * n - 1) // 6 + 3 * n * (n - 1) + 12 * (n - 1)


def f_solve(n: int) -> int:
    return 8 * (n * n - n) + 6 * n + 6


def f_ratio(n: int) -> int:
    return 8 * n + 12 + 5


def tree_flops(T, n_snk, nf, st) -> float:
    n = nf[0]
    F = len(nf)
    per_sink = (st["n_dom"] * (F * f_lu(n) + 11) + st["n_groups"] * f_solve(n)
                + st["n_children"] * f_ratio(n))
    return float(T) * n_snk * per_sink


def plain_flops(T, n_src, n_snk, nf) -> float:
    n = nf[0]
    return float(T) * n_src * n_snk * (len(nf) * f_lu(n) + 11)


def cpu_baseline(w, target_s: float = 15.0):
    """The CPU oracle on a bounded sample of the same workload: slice 0,
    the first source terms x all sink terms, over worker processes."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle_pool
    n_workers = oracle_pool.workers()
    # calibrate on a small piece, then size the sample to ~target_s
    rows = max(1, min(len(w.src), 8))
    t0 = time.perf_counter()
    oracle_pool.correlator(w.S, w.src[:rows], w.snk, w.nf, w.w_src[:rows], w.w_snk, [0],
                           n_workers=1)
    dt = time.perf_counter() - t0
    per_pair = dt / (rows * len(w.snk))
    n_rows = int(min(len(w.src), max(rows, target_s * n_workers / (per_pair * len(w.snk)))))
    t0 = time.perf_counter()
    oracle_pool.correlator(w.S, w.src[:n_rows], w.snk, w.nf, w.w_src[:n_rows], w.w_snk, [0],
                           n_workers=n_workers)
    dt = time.perf_counter() - t0
    pairs = n_rows * len(w.snk)
    return {"value": pairs / dt, "unit": "det-pairs/s", "cores": n_workers, "kind": "oracle",
            "sample": f"slice 0, source terms 0..{n_rows - 1} x all {len(w.snk)} sink terms "
                      f"({pairs} pairs, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the contraction has no multi-GPU path "
              "in this library (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    from paper_1411_3691_amd import workloads as W
    w = W.workload(args.workload)
    # CPU leg first, before the process touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(w)

    import numpy as np
    import torch
    from paper_1411_3691_amd import mhc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    src = mhc.Terms(w.src, w.nf, w.M)
    snk = mhc.Terms(w.snk, w.nf, w.M)
    tree = mhc.Tree(src)
    t_tree = time.perf_counter() - t0
    plan = mhc.Plan(tree, snk)
    st = tree.stats()
    S = torch.from_numpy(w.S).to(dev)
    ws = torch.from_numpy(np.ascontiguousarray(w.w_src)).to(dev)
    wk = torch.from_numpy(np.ascontiguousarray(w.w_snk)).to(dev)
    C = torch.empty(w.T, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()

    def timed(method):
        for _ in range(args.warmup):
            mhc.contract_into(plan, S, ws, wk, C, method)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        t0 = time.perf_counter()
        for a, b in evs:
            a.record()
            mhc.contract_into(plan, S, ws, wk, C, method)
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = [a.elapsed_time(b) for a, b in evs]          # ms, on the launch stream
        return wall, per, C.cpu().numpy().copy()

    wall_tree, ev_tree, C_tree = timed("tree")
    wall_plain, ev_plain, C_plain = timed("plain")
    pairs = w.n_pairs
    ms_tree = wall_tree * 1e3 / args.steps
    ms_plain = wall_plain * 1e3 / args.steps
    ev_tree_ms = float(np.mean(ev_tree))
    ev_plain_ms = float(np.mean(ev_plain))
    fl_tree = tree_flops(w.T, len(w.snk), w.nf, st)
    fl_plain = plain_flops(w.T, len(w.src), len(w.snk), w.nf)
    ach = fl_tree / (ev_tree_ms * 1e-3) / 1e12
    rel = float(np.max(np.abs(C_tree - C_plain)) / max(1e-300, float(np.max(np.abs(C_plain)))))

    out = {
        "metric": METRIC,
        "value": pairs / (wall_tree / args.steps),
        "unit": "det-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_tree,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: T={w.T} slices, M={w.M}, flavour blocks "
                        f"{list(w.nf)}, {len(w.src)} x {len(w.snk)} single-substitution "
                        f"tree terms",
            "pairs_per_step": pairs,
            "method": "update tree (greedy R2 dominating set)",
        },
        "plain_lu": {"value": pairs / (wall_plain / args.steps), "ms_per_step": ms_plain,
                     "kernel_ms": ev_plain_ms,
                     "flops_per_step": fl_plain,
                     "tflops": fl_plain / (ev_plain_ms * 1e-3) / 1e12},
        "speedup_vs_plain": (wall_plain / wall_tree),
        "tree_vs_plain_max_rel_diff": rel,
        "tree": {**st, "rho": st["n_dom"] / st["n_terms"], "build_s": t_tree,
                 "kernel_ms": ev_tree_ms, "flops_per_step": fl_tree},
        "roofline": {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS, "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
