"""Benchmark: complex128 det-pairs/s of the update-tree contraction against
the plain batched LU on the same GPU.

    python bench.py [--steps K] [--warmup W] [--workload mid|large|batch|grad]

One step = one update-tree contraction of every (slice, source term, sink
term) pair of the workload (gather, dominator LU, column solves, sibling
ratios, weighted reduction: one call of mhc_contract).  Inputs (propagator,
weights, plan) are resident on the GPU before timing starts.  The plain
batched LU is timed the same way on the same inputs and reported beside it.

Without --workload the headline is the mid workload (K timed steps after W
warm-ups), and the line carries two more measured workloads as
sub-objects: ``large`` (the full large workload, its own step counts) and
``batch`` (one graph launch of the 256-job batch per step, with the
autotuner's cached schedule).  Each sub-object has its own roofline and CPU
baseline.  Progress goes to stderr, one line per leg.  With --workload the
line is that workload alone.

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
SETTLE_S = 0.3              # untimed work before the first timed method

# HBM bytes per launch of the update-tree kernel on the mid workload, from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of this script
# (--copy-probe), each scaled by the same counter's reading for a 256 MiB
# device copy (fetch x 1.99975, write x 1.0).  Valid only for the kernel
# and launch-configuration sources they were measured on (SHA-256 below);
# null otherwise.
TRAFFIC = {
    "workload": "mid",
    "bytes": 7897.6 * 1.99975 * 1024 + 5312.0 * 1024,
    "sources": {
        "paper_1411_3691_amd/csrc/contract_kernels.hip":
            "9fbec0acae9e4cc410113541fe0e7dbcf87dd8592a82e48ce87713d28948a851",
        "paper_1411_3691_amd/csrc/lu_device.h":
            "905740ed3c6efd9d38d88961bc63339a3272e4b59a6a2f6ae2ffeeb88306414a",
        "paper_1411_3691_amd/csrc/mhc_plan.hip":
            "f9a4ed751e1cfb8dbd00a756eded95ce7a1d00cd71de4bdd405c9271b8c5a2e0",
        "paper_1411_3691_amd/csrc/contract_kernels.h":
            "69b507bda7c87dcc9ddb9c8a51f27b26736039c902a045f74f29122b034c9759",
    },
}


def measured_traffic(workload: str):
    """TRAFFIC["bytes"] if the kernel sources are the ones it was measured
    on, else None."""
    import hashlib
    if workload != TRAFFIC["workload"]:
        return None
    for rel, sha in TRAFFIC["sources"].items():
        try:
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != sha:
                    return None
        except OSError:
            return None
    return TRAFFIC["bytes"]
METRIC = "complex128 det-pairs/sec: update-tree vs plain batched LU, same GPU, 1e-11"


# Algorithmic flop counts (complex MAC = 8, complex multiply = 6, complex
# reciprocal = 6; pivot search and row exchanges are not counted).
def f_lu(n: int) -> int:
    return 8 * (n - 1) * n * (2 * n - 1) // 6 + 3 * n * (n - 1) + 12 * (n - 1)


def f_solve(n: int) -> int:
    return 8 * (n * n - n) + 6 * n + 6


def f_ratio(n: int) -> int:
    return 8 * n + 12 + 5


def f_solve_executed(n: int, r: int) -> int:
    """Flops the narrow kernels execute for x = G^-1 e_r: with column
    pivoting the unit vector stays at row r, so the forward part has
    (n-r-1)(n-r-2)/2 complex MACs; the backward part n(n-1)/2 MACs, r of them
    plain complex multiplies (rows above r start from zero), and n complex
    multiplies by 1/U_mm.  f_solve (the paper's n^2 - n MACs) counts the
    forward part in full."""
    return 8 * ((n - r - 1) * (n - r - 2) // 2 + n * (n - 1) // 2) - 2 * r + 6 * n


def tree_flops(T, n_snk, nf, tree, executed: bool = False) -> float:
    """Per (slice, sink): every dominator's blocks factorised (and the
    weighted product), one solve per (dominator, flavour, changed row) group
    and one ratio per child, each at its own flavour's block size; ``tree``
    is the exported tree (owner, flavour and row of every term).  With
    ``executed`` the solves are counted as the kernels execute them
    (f_solve_executed) instead of by the convention (f_solve)."""
    import numpy as np
    owner, flav, pos = tree["owner"], tree["flav"], tree["pos"]
    child = owner != np.arange(len(owner))
    per_sink = tree["n_dom"] * float(sum(f_lu(n) for n in nf) + 11)
    groups = set(zip(owner[child].tolist(), flav[child].tolist(), pos[child].tolist()))
    if executed:
        per_sink += sum(f_solve_executed(nf[f], r) for _, f, r in groups)
    else:
        per_sink += sum(f_solve(nf[f]) for _, f, _ in groups)
    per_sink += sum(f_ratio(nf[f]) for f in flav[child].tolist())
    return float(T) * n_snk * per_sink


def _per_flavour(tree, F):
    """Per dominator: children and (row, flavour) groups in each flavour."""
    import numpy as np
    owner, flav, pos = tree["owner"], tree["flav"], tree["pos"]
    doms = np.flatnonzero(owner == np.arange(len(owner)))
    index = {int(d): k for k, d in enumerate(doms)}
    ch = np.zeros((len(doms), F))
    gr = np.zeros((len(doms), F))
    seen = set()
    for u in np.flatnonzero(owner != np.arange(len(owner))).tolist():
        k, f = index[int(owner[u])], int(flav[u])
        ch[k, f] += 1
        key = (k, f, int(pos[u]))
        if key not in seen:
            seen.add(key)
            gr[k, f] += 1
    return ch, gr


def two_sided_flops(T, nf, src_tree, snk_tree) -> float:
    """Per slice, over every (source dominator, sink dominator): the
    dominators' blocks factorised; one column solve per source group and one
    row solve per sink group; one ratio per child on either side; one column
    solve q_d per sink child in each flavour where the source dominator has
    children; per same-block (source child, sink child) pair a dot of n
    plus the corner and the weight (8n + 6) and per (source group, sink
    child) the kappa product (10)."""
    F = len(nf)
    n = nf[0]
    cs, gs = _per_flavour(src_tree, F)
    ck, gk = _per_flavour(snk_tree, F)
    na, nb = len(cs), len(ck)
    total = na * nb * float(F * f_lu(n) + 11)
    total += nb * float((gs * f_solve(n) + cs * f_ratio(n)).sum())
    total += na * float((gk * f_solve(n) + ck * f_ratio(n)).sum())
    for f in range(F):
        total += ck[:, f].sum() * float((cs[:, f] > 0).sum()) * f_solve(n)
        total += cs[:, f].sum() * ck[:, f].sum() * (8 * n + 6)
        total += gs[:, f].sum() * ck[:, f].sum() * 10
    return float(T) * total


def fma_probe(dev, iters: int = 4096, n_blocks: int = 4096, reps: int = 10) -> float:
    """Measured FP64 vector FMA rate (TFLOP/s) of this GPU: the probe kernel
    of the library (16 independent v_fma_f64 chains per thread), timed with
    HIP events on the launch stream over `reps` launches after 3 warm-ups."""
    import torch
    from paper_1411_3691_amd import mhc
    out = torch.empty(n_blocks * mhc.PROBE_BLOCK, dtype=torch.float64, device=dev)
    for _ in range(3):
        mhc.probe_fma64(out, iters)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    flop = 0
    for _ in range(reps):
        flop += mhc.probe_fma64(out, iters)
    e1.record()
    torch.cuda.synchronize()
    return flop / (e0.elapsed_time(e1) * 1e-3) / 1e12


def mfma_probe(dev, with_valu: bool, iters: int = 2048, n_blocks: int = 4096,
               reps: int = 5) -> float:
    """Measured FP64 matrix-core rate (TFLOP/s) of this GPU: 4 independent
    v_mfma_f64_16x16x4_f64 chains per wave (with_valu: plus the 16 vector
    FMA chains per thread, counted in the rate), timed as fma_probe."""
    import torch
    from paper_1411_3691_amd import mhc
    out = torch.empty(n_blocks * mhc.PROBE_BLOCK, dtype=torch.float64, device=dev)
    for _ in range(2):
        mhc.probe_mfma64(out, iters, with_valu)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    flop = 0
    for _ in range(reps):
        flop += mhc.probe_mfma64(out, iters, with_valu)
    e1.record()
    torch.cuda.synchronize()
    return flop / (e0.elapsed_time(e1) * 1e-3) / 1e12


def plain_flops(T, n_src, n_snk, nf) -> float:
    return float(T) * n_src * n_snk * (sum(f_lu(n) for n in nf) + 11)


def log(msg: str) -> None:
    """One progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(w, target_s: float = 15.0):
    """The CPU oracle on a bounded sample of the same workload: the first
    slices (or, below one slice, the first source terms of slice 0) x all
    sink terms, over worker processes."""
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
    want = target_s * n_workers / per_pair          # pairs in ~target_s
    slice_pairs = len(w.src) * len(w.snk)
    if want >= slice_pairs:
        n_sl = int(min(w.T, want // slice_pairs))
        n_rows = len(w.src)
    else:
        n_sl = 1
        n_rows = int(max(rows, want // len(w.snk)))
    t0 = time.perf_counter()
    oracle_pool.correlator(w.S, w.src[:n_rows], w.snk, w.nf, w.w_src[:n_rows], w.w_snk,
                           list(range(n_sl)), n_workers=n_workers)
    dt = time.perf_counter() - t0
    pairs = n_sl * n_rows * len(w.snk)
    return {"value": pairs / dt, "unit": "det-pairs/s", "cores": n_workers, "kind": "oracle",
            "host_cpu_count": os.cpu_count(),
            "sample": f"slices 0..{n_sl - 1}, source terms 0..{n_rows - 1} x all "
                      f"{len(w.snk)} sink terms ({pairs} pairs, {dt:.1f} s)"}


def cpu_baseline_batch(ws, pairs_per_job: int = 60_000):
    """The CPU oracle on a fixed 16-job subset of the batch: per job, slice 0
    and the first source terms (about pairs_per_job pairs) x all sink terms."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle_pool
    n_workers = oracle_pool.workers()
    pairs = 0
    t0 = time.perf_counter()
    for w in ws[:16]:
        rows = max(1, min(len(w.src), pairs_per_job // len(w.snk)))
        oracle_pool.correlator(w.S, w.src[:rows], w.snk, w.nf, w.w_src[:rows], w.w_snk, [0],
                               n_workers=n_workers)
        pairs += rows * len(w.snk)
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "det-pairs/s", "cores": n_workers, "kind": "oracle",
            "host_cpu_count": os.cpu_count(),
            "sample": f"jobs 0..15 of the batch, slice 0, about {pairs_per_job} pairs each "
                      f"({pairs} pairs, {dt:.1f} s)"}


def run_timed(run, steps: int, warmup: int):
    """W untimed calls, then K timed calls bracketed by device syncs: the
    wall time of the K calls and each call's HIP-event time (ms) on torch's
    current stream, the launch stream of the library's kernels."""
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        run()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in evs]


def roofline(flops: float, kernel_ms: float, traffic=None) -> dict:
    ach = flops / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP64_PEAK_TFLOPS, "traffic": traffic}


def bench_batch(args, steps: int, warmup: int, plain_steps: int, plain_warmup: int,
                cpu=None, with_pruned: bool = False) -> dict:
    """The 256-job batch: one graph launch per step, on the autotuner's
    cached schedule for these shapes (the library's default when the cache
    has no entry)."""
    import numpy as np
    import torch
    from paper_1411_3691_amd import autotune, mhc
    from paper_1411_3691_amd import workloads as W

    shapes = W.batch_shapes()
    ws = [W.batch_job(j, shapes[j]) for j in range(len(shapes))]
    dev = torch.device("cuda", 0)
    plans, S, a, b, C = [], [], [], [], []
    fl_tree = fl_plain = 0.0
    t0 = time.perf_counter()
    for w in ws:
        tree = mhc.Tree(mhc.Terms(w.src, w.nf, w.M))
        plans.append(mhc.Plan(tree, mhc.Terms(w.snk, w.nf, w.M)))
        fl_tree += tree_flops(w.T, len(w.snk), w.nf, tree.export())
        fl_plain += plain_flops(w.T, len(w.src), len(w.snk), w.nf)
        S.append(torch.from_numpy(w.S).to(dev))
        a.append(torch.from_numpy(w.w_src).to(dev))
        b.append(torch.from_numpy(w.w_snk).to(dev))
        C.append(torch.empty(w.T, dtype=torch.complex128, device=dev))
    t_plan = time.perf_counter() - t0
    pairs = sum(w.n_pairs for w in ws)
    Ts = [w.T for w in ws]
    torch.cuda.synchronize()
    log(f"batch: {len(ws)} plans built in {t_plan:.1f} s")

    def timed(method, sched, k, wu):
        batch = mhc.Batch(plans, Ts, method, sched)
        wall, ev = run_timed(lambda: batch.run(S, a, b, C), k, wu)
        return wall, float(np.mean(ev)), [c.cpu().numpy().copy() for c in C], batch.info()

    cache = os.path.join(ROOT, "paper_1411_3691_amd", "schedules.json")
    if args.tune_cache:
        # time every candidate schedule and store the choices (slow)
        for method in ("tree", "plain"):
            log(f"batch: tuning the {method} schedule")
            autotune.tune(plans, Ts, method, S, a, b, cache=args.tune_cache, verbose=True)
        cache = args.tune_cache
    sched_tree = autotune.cached(plans, Ts, "tree", cache)
    sched_plain = autotune.cached(plans, Ts, "plain", cache)
    wall_tree, ev_tree, C_tree, info = timed("tree", sched_tree, steps, warmup)
    log(f"batch: tree {wall_tree / steps:.3f} s per step")
    wall_plain, ev_plain, C_plain, _ = timed("plain", sched_plain, plain_steps, plain_warmup)
    log(f"batch: plain {wall_plain / plain_steps:.3f} s per step")
    rel = max(float(np.max(np.abs(x - y)) / max(1e-300, float(np.max(np.abs(y)))))
              for x, y in zip(C_tree, C_plain))
    pruned = None
    if with_pruned:
        # every job's tree on its reverse-delete dominating set
        plans_main, plans = plans, []
        fl_pr, n_dom_g, n_dom_p = 0.0, 0, 0
        for w in ws:
            terms = mhc.Terms(w.src, w.nf, w.M)
            tree = mhc.Tree(terms, prune=True)
            plans.append(mhc.Plan(tree, mhc.Terms(w.snk, w.nf, w.M)))
            fl_pr += tree_flops(w.T, len(w.snk), w.nf, tree.export())
            n_dom_p += tree.stats()["n_dom"]
            n_dom_g += mhc.Tree(terms).stats()["n_dom"]
        wall_pr, ev_pr, C_pr, _ = timed("tree", sched_tree, steps, warmup)
        plans = plans_main
        pruned = {"value": pairs / (wall_pr / steps), "ms_per_step": wall_pr * 1e3 / steps,
                  "kernel_ms": ev_pr, "n_dom": n_dom_p, "n_dom_greedy": n_dom_g,
                  "flops_per_step": fl_pr, "tflops": fl_pr / (ev_pr * 1e-3) / 1e12,
                  "max_rel_diff_vs_plain": max(
                      float(np.max(np.abs(x - y)) / max(1e-300, float(np.max(np.abs(y)))))
                      for x, y in zip(C_pr, C_plain))}
    nfs = sorted({n for w in ws for n in w.nf})
    return {
        "metric": METRIC,
        "value": pairs / (wall_tree / steps),
        "unit": "det-pairs/s",
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall_tree * 1e3 / steps,
        "config": {
            "workload": f"batch: {len(ws)} jobs, flavour blocks {nfs[0]}..{nfs[-1]}, "
                        f"T 8..64, M 24/48/96, 50..5000 tree terms per side",
            "pairs_per_step": pairs,
            "method": "update tree (greedy R2 dominating set), one graph launch",
            "schedule_tree": sched_tree, "schedule_plain": sched_plain,
        },
        "plain_lu": {"value": pairs / (wall_plain / plain_steps),
                     "ms_per_step": wall_plain * 1e3 / plain_steps, "kernel_ms": ev_plain,
                     "steps": plain_steps, "warmup": plain_warmup,
                     "flops_per_step": fl_plain,
                     "tflops": fl_plain / (ev_plain * 1e-3) / 1e12},
        "speedup_vs_plain": (wall_plain / plain_steps) / (wall_tree / steps),
        "tree_vs_plain_max_rel_diff": rel,
        "tree": {"kernel_ms": ev_tree, "flops_per_step": fl_tree, "plan_s": t_plan, **info},
        "tree_pruned_dominators": pruned,
        "roofline": roofline(fl_tree, ev_tree),
        "cpu_baseline": cpu,
    }


def bench_workload(w, args, steps: int, warmup: int, plain_steps: int, plain_warmup: int,
                   cpu=None, extras: bool = True, settle: bool = True, probe: bool = True) -> dict:
    """One workload: the update tree (K timed calls after W warm-ups) and the
    plain LU; with ``extras`` also the paper's ablations (mid), the
    reverse-delete dominating set, the adjoint (grad) and the two-sided
    trees (one block size <= 8)."""
    import numpy as np
    import torch
    from paper_1411_3691_amd import mhc

    dev = torch.device("cuda", 0)
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
    if args.copy_probe:
        a_ = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        b_ = torch.empty_like(a_)
        torch.cuda.synchronize()
        b_.copy_(a_)          # 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        del a_, b_
    torch.cuda.synchronize()
    name = w.name

    # The GPU raises its clocks over the first tens of milliseconds of
    # sustained work (back-to-back launches of one kernel run about 10 %
    # faster after ~50 ms): run the update tree untimed for SETTLE_S seconds
    # before the first timed method, then W warm-up steps per method.
    if settle:
        t_settle = time.perf_counter()
        while time.perf_counter() - t_settle < SETTLE_S:
            mhc.contract_into(plan, S, ws, wk, C, "tree")
            torch.cuda.synchronize()

    fma = fma_probe(dev) if probe else None
    mfma = ({"tflops": mfma_probe(dev, False), "tflops_with_vector_fma": mfma_probe(dev, True)}
            if probe else None)

    cur = {"plan": plan}

    def timed(method, k=steps, wu=warmup):
        p = cur["plan"]
        wall, per = run_timed(lambda: mhc.contract_into(p, S, ws, wk, C, method), k, wu)
        return wall, per, C.cpu().numpy().copy()

    wall_tree, ev_tree, C_tree = timed("tree")
    log(f"{name}: tree {wall_tree * 1e3 / steps:.3f} ms per step")
    wall_plain, ev_plain, C_plain = timed("plain", plain_steps, plain_warmup)
    log(f"{name}: plain {wall_plain * 1e3 / plain_steps:.3f} ms per step")
    fl_tree = tree_flops(w.T, len(w.snk), w.nf, tree.export())
    # blocks of at most 8 take the lane-per-matrix kernels, whose solves
    # skip the zero head of e_r
    narrow = len(set(w.nf)) == 1 and max(w.nf) <= 8
    fl_tree_exec = (tree_flops(w.T, len(w.snk), w.nf, tree.export(), executed=True)
                    if narrow else None)
    abl = None
    if extras and name == "mid":
        # the paper's variants (Sec. 4, Fig. 1 caption) on the same inputs:
        # LU without pivoting, and updates without shared solves; and LU
        # with threshold partial pivoting
        abl = {}
        for lbl, method in (("plain_unpivoted", "plain_unpivoted"),
                            ("tree_unpivoted", "tree_unpivoted"),
                            ("plain_threshold_pivoting", "plain_threshold"),
                            ("tree_threshold_pivoting", "tree_threshold")):
            wall_a, ev_a, _ = timed(method)
            abl[lbl] = {"ms_per_step": wall_a * 1e3 / steps,
                        "kernel_ms": float(np.mean(ev_a)),
                        "value": w.n_pairs / (wall_a / steps)}
            if method == "tree_threshold":
                a_t = fl_tree / (float(np.mean(ev_a)) * 1e-3) / 1e12
                abl[lbl]["tflops"] = a_t
                abl[lbl]["frac"] = a_t / FP64_PEAK_TFLOPS
        tree_ns = mhc.Tree(src, share=False)
        cur["plan"] = mhc.Plan(tree_ns, snk)
        wall_a, ev_a, _ = timed("tree")
        cur["plan"] = plan
        abl["tree_without_sharing"] = {"ms_per_step": wall_a * 1e3 / steps,
                                       "kernel_ms": float(np.mean(ev_a)),
                                       "value": w.n_pairs / (wall_a / steps),
                                       "n_groups": tree_ns.stats()["n_groups"]}
        # weighted-row aggregation (an extension: one dot per group of
        # siblings; no per-pair values, so it is not the headline)
        wall_a, ev_a, C_agg = timed("tree_agg")
        abl["tree_aggregation"] = {
            "ms_per_step": wall_a * 1e3 / steps, "kernel_ms": float(np.mean(ev_a)),
            "value": w.n_pairs / (wall_a / steps),
            "max_rel_diff_vs_tree": float(np.max(np.abs(C_agg - C_tree)) /
                                          max(1e-300, float(np.max(np.abs(C_tree)))))}
        # set-based edges: the same terms with every flavour block listed in
        # a random order; positional edges then see few neighbours, set
        # edges (with the permutation sign) see the forest again
        rng = np.random.default_rng(20141113)
        offs = np.concatenate([[0], np.cumsum(w.nf)])
        perm_idx = {}
        for side, terms in (("src", w.src), ("snk", w.snk)):
            t2 = terms.copy()
            for u in range(len(t2)):
                for f in range(len(w.nf)):
                    o, k = offs[f], w.nf[f]
                    t2[u, o:o + k] = t2[u, o:o + k][rng.permutation(k)]
            perm_idx[side] = t2
        src_p = mhc.Terms(perm_idx["src"], w.nf, w.M)
        snk_p = mhc.Terms(perm_idx["snk"], w.nf, w.M)
        set_res = {}
        for lbl, se in (("positional_edges", False), ("set_edges", True)):
            tr_p = mhc.Tree(src_p, set_edges=se)
            cur["plan"] = mhc.Plan(tr_p, snk_p)
            wall_a, ev_a, C_p = timed("tree")
            set_res[lbl] = {"ms_per_step": wall_a * 1e3 / steps,
                            "kernel_ms": float(np.mean(ev_a)),
                            "value": w.n_pairs / (wall_a / steps),
                            "n_dom": tr_p.stats()["n_dom"], "C": C_p}
        cur["plan"] = plan
        c_pos, c_set = set_res["positional_edges"].pop("C"), set_res["set_edges"].pop("C")
        set_res["max_rel_diff"] = float(np.max(np.abs(c_set - c_pos)) /
                                        max(1e-300, float(np.max(np.abs(c_pos)))))
        abl["permuted_terms"] = set_res
        log(f"{name}: ablations done")
    if extras and name in ("mid", "large"):
        # reverse-delete dominating set: fewer dominators, same sum
        abl = abl if abl is not None else {}
        tree_pr = mhc.Tree(src, prune=True)
        cur["plan"] = mhc.Plan(tree_pr, snk)
        wall_a, ev_a, C_pr = timed("tree")
        cur["plan"] = plan
        fl_pr = tree_flops(w.T, len(w.snk), w.nf, tree_pr.export())
        st_pr = tree_pr.stats()
        abl["tree_pruned_dominators"] = {
            "ms_per_step": wall_a * 1e3 / steps,
            "kernel_ms": float(np.mean(ev_a)),
            "value": w.n_pairs / (wall_a / steps),
            "n_dom": st_pr["n_dom"], "n_groups": st_pr["n_groups"],
            "flops_per_step": fl_pr,
            "tflops": fl_pr / (float(np.mean(ev_a)) * 1e-3) / 1e12,
            "max_rel_diff_vs_tree": float(np.max(np.abs(C_pr - C_tree))
                                          / max(1e-300, float(np.max(np.abs(C_tree)))))}
        log(f"{name}: reverse-delete dominating set done")
    back = None
    if extras and name == "grad":
        # the adjoint (mhc_contract_backward): grad S and both weight
        # gradients for a random upstream gradient
        gC = torch.from_numpy(np.random.default_rng(0).standard_normal(w.T)
                              + 1j * np.random.default_rng(1).standard_normal(w.T)).to(dev)
        back = {}
        for bm in ("tree", "plain"):
            wall_b, ev_b = run_timed(lambda: mhc.contract_backward(plan, S, ws, wk, gC, bm),
                                     steps, warmup)
            ms_b = float(np.mean(ev_b))
            back[bm] = {"ms_per_step": wall_b * 1e3 / steps, "kernel_ms": ms_b,
                        "det_pairs_per_s": w.n_pairs / (ms_b * 1e-3)}
    two = None
    if extras and narrow:
        # the two-sided extension: sink terms in their own update tree
        t0 = time.perf_counter()
        stree = mhc.Tree(snk)
        t_stree = time.perf_counter() - t0
        plan.attach_sink_tree(stree)
        wall_two, ev_two, C_two = timed("tree2")
        ev_two_ms = float(np.mean(ev_two))
        fl_two = two_sided_flops(w.T, w.nf, tree.export(), stree.export())
        ach_two = fl_two / (ev_two_ms * 1e-3) / 1e12
        two = {"value": w.n_pairs / (wall_two / steps),
               "ms_per_step": wall_two * 1e3 / steps, "kernel_ms": ev_two_ms,
               "flops_per_step": fl_two, "tflops": ach_two,
               "frac": ach_two / FP64_PEAK_TFLOPS,
               "speedup_vs_plain": (wall_plain / plain_steps) / (wall_two / steps),
               "speedup_vs_one_sided": wall_tree / wall_two,
               "max_rel_diff_vs_plain": float(np.max(np.abs(C_two - C_plain)) /
                                              max(1e-300, float(np.max(np.abs(C_plain))))),
               "sink_tree": {**stree.stats(), "build_s": t_stree}}
        # both trees on reverse-delete dominating sets: fewer (source
        # dominator, sink dominator) LUs
        tree_p2, stree_p2 = mhc.Tree(src, prune=True), mhc.Tree(snk, prune=True)
        plan_p2 = mhc.Plan(tree_p2, snk)
        plan_p2.attach_sink_tree(stree_p2)
        cur["plan"] = plan_p2
        wall_p2, ev_p2, C_p2 = timed("tree2")
        cur["plan"] = plan
        fl_p2 = two_sided_flops(w.T, w.nf, tree_p2.export(), stree_p2.export())
        two["pruned_dominators"] = {
            "value": w.n_pairs / (wall_p2 / steps),
            "ms_per_step": wall_p2 * 1e3 / steps,
            "kernel_ms": float(np.mean(ev_p2)),
            "n_dom_src": tree_p2.stats()["n_dom"], "n_dom_snk": stree_p2.stats()["n_dom"],
            "flops_per_step": fl_p2,
            "tflops": fl_p2 / (float(np.mean(ev_p2)) * 1e-3) / 1e12,
            "max_rel_diff_vs_plain": float(np.max(np.abs(C_p2 - C_plain)) /
                                           max(1e-300, float(np.max(np.abs(C_plain)))))}
        log(f"{name}: two-sided trees done")
    pairs = w.n_pairs
    ev_tree_ms = float(np.mean(ev_tree))
    ev_plain_ms = float(np.mean(ev_plain))
    fl_plain = plain_flops(w.T, len(w.src), len(w.snk), w.nf)
    rel = float(np.max(np.abs(C_tree - C_plain)) / max(1e-300, float(np.max(np.abs(C_plain)))))
    rf = roofline(fl_tree, ev_tree_ms, measured_traffic(name))
    out = {
        "metric": METRIC,
        "value": pairs / (wall_tree / steps),
        "unit": "det-pairs/s",
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall_tree * 1e3 / steps,
        "config": {
            "workload": f"{name}: T={w.T} slices, M={w.M}, flavour blocks "
                        f"{list(w.nf)}, {len(w.src)} x {len(w.snk)} single-substitution "
                        f"tree terms",
            "pairs_per_step": pairs,
            "method": "update tree (greedy R2 dominating set)",
        },
        "plain_lu": {"value": pairs / (wall_plain / plain_steps),
                     "ms_per_step": wall_plain * 1e3 / plain_steps,
                     "kernel_ms": ev_plain_ms, "steps": plain_steps, "warmup": plain_warmup,
                     "flops_per_step": fl_plain,
                     "tflops": fl_plain / (ev_plain_ms * 1e-3) / 1e12},
        "speedup_vs_plain": (wall_plain / plain_steps) / (wall_tree / steps),
        "tree_vs_plain_max_rel_diff": rel,
        "tree": {**st, "rho": st["n_dom"] / st["n_terms"], "build_s": t_tree,
                 "kernel_ms": ev_tree_ms, "flops_per_step": fl_tree,
                 "flops_executed_per_step": fl_tree_exec,
                 "frac_executed": (fl_tree_exec / (ev_tree_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS
                                   if narrow else None)},
        "roofline": rf,
        "cpu_baseline": cpu,
    }
    if fma is not None:
        out["fp64_fma_probe"] = {"tflops": fma, "frac_of_peak": fma / FP64_PEAK_TFLOPS,
                                 "tree_frac_of_probe": rf["achieved"] / fma}
    if mfma is not None:
        out["fp64_mfma_probe"] = mfma
    if extras:
        out["two_sided"] = two
        out["ablations"] = abl
        out["backward"] = back
    return out


def headline(obj: dict, args) -> dict:
    """The contract's top-level fields around one workload's object."""
    out = {"metric": obj["metric"], "value": obj["value"], "unit": obj["unit"],
           "n_gpus": 1, "steps": obj["steps"], "warmup": obj["warmup"],
           "ms_per_step": obj["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    out.update({k: v for k, v in obj.items() if k not in out})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None,
                    help="mid | large | batch | grad: that workload alone (default: mid "
                         "with the large and batch sub-objects)")
    ap.add_argument("--large-steps", type=int, default=3)
    ap.add_argument("--large-warmup", type=int, default=1)
    ap.add_argument("--large-plain-steps", type=int, default=1)
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--batch-warmup", type=int, default=1)
    ap.add_argument("--batch-plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="batch: run the autotuner for both methods first and store its "
                         "choices in this JSON file")
    ap.add_argument("--copy-probe", action="store_true",
                    help="one 256 MiB device-to-device copy before timing (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the contraction has no multi-GPU path "
              "in this library (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    from paper_1411_3691_amd import workloads as W
    wl = args.workload
    # CPU legs first, before the process touches the GPU (the oracle's
    # worker processes are forked)
    cpu = {}
    if not args.no_cpu_baseline:
        if wl in (None, "mid", "large", "grad"):
            for name in ([wl] if wl else ["mid", "large"]):
                log(f"{name}: CPU oracle sample")
                cpu[name] = cpu_baseline(W.workload(name), 15.0 if name == "mid" else 10.0)
        if wl in (None, "batch"):
            log("batch: CPU oracle sample (16 jobs)")
            shapes = W.batch_shapes()
            cpu["batch"] = cpu_baseline_batch([W.batch_job(j, shapes[j]) for j in range(16)])

    import torch
    torch.cuda.set_device(0)
    if wl == "batch":
        out = bench_batch(args, args.steps, args.warmup, args.steps, args.warmup,
                          cpu.get("batch"), with_pruned=True)
        print(json.dumps(headline(out, args)), flush=True)
        return
    if wl is not None:
        out = bench_workload(W.workload(wl), args, args.steps, args.warmup, args.steps,
                             args.warmup, cpu.get(wl))
        print(json.dumps(headline(out, args)), flush=True)
        return
    # default: the mid headline, then the large and batch workloads
    log("mid: headline")
    out = bench_workload(W.workload("mid"), args, args.steps, args.warmup, args.steps,
                         args.warmup, cpu.get("mid"))
    log("large: full workload")
    large = bench_workload(W.workload("large"), args, args.large_steps, args.large_warmup,
                           args.large_plain_steps, 0, cpu.get("large"), extras=False,
                           settle=False, probe=False)
    log("batch: 256 jobs")
    batch = bench_batch(args, args.batch_steps, args.batch_warmup, args.batch_plain_steps, 0,
                        cpu.get("batch"))
    line = headline(out, args)
    line["large"] = large
    line["batch"] = batch
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
