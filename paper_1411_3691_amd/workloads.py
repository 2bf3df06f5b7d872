"""Seeded synthetic inputs for the multi-hadron correlator contraction.

This module only draws random inputs: propagators, wavefunction term lists and
weights.  It contains none of the contraction arithmetic, so the CPU oracle,
the tests and the benchmark can all use it without sharing any part of the
method with the GPU path.

Shapes and structure follow the paper's workload (alpha-particle
wavefunctions, Sec. 4): two flavour blocks, six-quark blocks (6x6 matrices),
thousands of terms per side, terms of one wavefunction related to each other
by single-index substitutions (the structure the update tree of Sec. 3
exploits).  The paper's own wavefunctions are not available, so trees of
single-index substitutions stand in for them.

Propagator convention: ``S[t, p, q]`` is the propagator from source quark
index ``p`` (the row, an index of a source term) to sink quark index ``q``
(the column, an index of a sink term), as in the definition of G^(ij) in
Sec. 1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 14113691

# Named workloads.  ``k`` selects the seed family; ``decay`` is the rate of the
# exponential fall-off of |S_t| with t.
CONFIGS = {
    # 1 slice, one site (3 colours x 4 spins), two flavours of 3 quarks,
    # 64 x 64 independently drawn terms.
    "tiny": dict(k=1, T=1, M=12, nf=(3, 3), n_src=64, n_snk=64,
                 terms="plain", decay=0.0),
    # 32 slices, 4 sites, two flavours of 6 quarks, 2000 x 2000 terms in
    # single-substitution trees (branching 8, depth <= 4).
    "mid": dict(k=2, T=32, M=48, nf=(6, 6), n_src=2000, n_snk=2000,
                terms="tree", branching=8, depth=4, decay=0.5),
    # 64 slices, 8 sites, two flavours of 12 quarks, 20000 x 20000 terms
    # (branching 16, depth <= 5).
    "large": dict(k=3, T=64, M=96, nf=(12, 12), n_src=20000, n_snk=20000,
                  terms="tree", branching=16, depth=5, decay=0.4),
    # Shapes of "mid", own seeds: the differentiation workload.
    "grad": dict(k=5, T=32, M=48, nf=(6, 6), n_src=2000, n_snk=2000,
                 terms="tree", branching=8, depth=4, decay=0.5),
}


def rng_for(k: int, stream: int) -> np.random.Generator:
    """Generator for workload family ``k``: stream 0 = S, 1/2 = source/sink
    terms, 3/4 = source/sink weights."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + 100 * k + stream))


def make_propagator(rng, T: int, M: int, decay: float = 0.0,
                    shared: bool = False) -> np.ndarray:
    """complex128 [T][M][M]: exp(-decay*t) * (X + iY), X, Y iid N(0,1).

    ``shared=True`` draws one slice S_0 and sets S_t = exp(-decay*t) S_0.
    """
    shape = (1 if shared else T, M, M)
    x = rng.standard_normal(shape)
    y = rng.standard_normal(shape)
    s = (x + 1j * y).astype(np.complex128)
    if shared:
        s = np.repeat(s, T, axis=0)
    scale = np.exp(-decay * np.arange(T, dtype=np.float64))
    s *= scale[:, None, None]
    return np.ascontiguousarray(s)


def make_plain_terms(rng, n_terms: int, M: int, nf) -> np.ndarray:
    """int32 [n_terms][sum(nf)]: per flavour, nf[f] distinct indices of
    [0, M) in the order drawn."""
    # (duplicates are possible; the caller decides whether that matters)
    out = np.empty((n_terms, int(sum(nf))), dtype=np.int32)
    for i in range(n_terms):
        parts = [rng.choice(M, size=n, replace=False) for n in nf]
        out[i] = np.concatenate(parts)
    return out


def make_tree_terms(rng, n_terms: int, M: int, nf, branching: int,
                    depth: int, max_retry: int = 100) -> np.ndarray:
    """int32 [n_terms][sum(nf)]: a forest of single-index substitutions.

    Each tree gets a random root (as ``make_plain_terms``) and a depth d drawn
    uniformly from 1..depth.  It is expanded breadth first: every node above
    depth d gets ``branching`` children.  A child copies its parent and puts a
    new index, not already used in that flavour, into one uniformly chosen
    slot.  Children that repeat an existing term are redrawn (up to
    ``max_retry`` times, then skipped).  Generation stops at ``n_terms``.
    """
    nf = [int(n) for n in nf]
    sn = sum(nf)
    flav_of_slot = np.repeat(np.arange(len(nf)), nf)
    offs = np.concatenate([[0], np.cumsum(nf)])
    terms: list[tuple] = []
    seen: set[tuple] = set()

    def add(t):
        tt = tuple(int(v) for v in t)
        if tt in seen:
            return False
        seen.add(tt)
        terms.append(tt)
        return True

    failed_roots = 0
    while len(terms) < n_terms:
        root = np.concatenate([rng.choice(M, size=n, replace=False)
                               for n in nf]).astype(np.int64)
        if not add(root):
            failed_roots += 1
            if failed_roots > 1000:
                raise ValueError(f"cannot draw {n_terms} distinct terms "
                                 f"from M={M}, nf={tuple(nf)}")
            continue
        d = int(rng.integers(1, depth + 1))
        frontier = [root]
        for _ in range(d):
            nxt = []
            for node in frontier:
                for _b in range(branching):
                    if len(terms) >= n_terms:
                        break
                    for _try in range(max_retry):
                        slot = int(rng.integers(sn))
                        f = int(flav_of_slot[slot])
                        cur = set(int(v) for v in node[offs[f]:offs[f + 1]])
                        free = [c for c in range(M) if c not in cur]
                        child = node.copy()
                        child[slot] = free[int(rng.integers(len(free)))]
                        if add(child):
                            nxt.append(child)
                            break
                if len(terms) >= n_terms:
                    break
            frontier = nxt
            if len(terms) >= n_terms or not frontier:
                break
    return np.asarray(terms, dtype=np.int32).reshape(n_terms, sn)


@dataclasses.dataclass
class Workload:
    name: str
    S: np.ndarray          # complex128 [T][M][M]
    src: np.ndarray        # int32 [n_src][sum(nf)]
    snk: np.ndarray        # int32 [n_snk][sum(nf)]
    w_src: np.ndarray      # float64 [n_src]
    w_snk: np.ndarray      # float64 [n_snk]
    nf: tuple
    cfg: dict

    @property
    def T(self):
        return self.S.shape[0]

    @property
    def M(self):
        return self.S.shape[1]

    @property
    def n_pairs(self):
        return self.T * len(self.src) * len(self.snk)


def workload(name: str, shared_S: bool = False, **over) -> Workload:
    """Build a named workload; keyword overrides change its shape (e.g.
    ``workload("mid", T=2, n_src=300, n_snk=200)``) while keeping the seed
    family and the generator."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    k = cfg["k"]
    nf = tuple(int(n) for n in cfg["nf"])
    S = make_propagator(rng_for(k, 0), cfg["T"], cfg["M"], cfg["decay"],
                        shared=shared_S)
    if cfg["terms"] == "plain":
        src = make_plain_terms(rng_for(k, 1), cfg["n_src"], cfg["M"], nf)
        snk = make_plain_terms(rng_for(k, 2), cfg["n_snk"], cfg["M"], nf)
    else:
        src = make_tree_terms(rng_for(k, 1), cfg["n_src"], cfg["M"], nf,
                              cfg["branching"], cfg["depth"])
        snk = make_tree_terms(rng_for(k, 2), cfg["n_snk"], cfg["M"], nf,
                              cfg["branching"], cfg["depth"])
    w_src = rng_for(k, 3).standard_normal(cfg["n_src"])
    w_snk = rng_for(k, 4).standard_normal(cfg["n_snk"])
    return Workload(name, S, src, snk, w_src, w_snk, nf, cfg)


def random_pairs(rng, T: int, n_src: int, n_snk: int, count: int) -> np.ndarray:
    """int64 [count][3] of (t, i, j) drawn uniformly (with replacement)."""
    return np.stack([rng.integers(0, T, count), rng.integers(0, n_src, count),
                     rng.integers(0, n_snk, count)], axis=1).astype(np.int64)


def log_uniform_int(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


# Batched uneven jobs: 256 independent correlators.  Per job, each flavour's
# block size is drawn from U{2..18} independently, the term count per side
# from round(exp(U[ln 50, ln 5000])), the slice count from U{8..64} and the
# number of sites from {2, 4, 8} (M = 12 x sites); terms are single-
# substitution forests with branching 8 and depth <= 4; S is N(0,1)+iN(0,1)
# without decay.  Every job's shape is drawn first from one generator, so a
# subset of jobs has the same shapes as in the full batch.
BATCH_SEED_K = 4
BATCH_JOBS = 256


def batch_shapes(n_jobs: int = BATCH_JOBS) -> list[dict]:
    rng = rng_for(BATCH_SEED_K, 0)
    out = []
    for _ in range(n_jobs):
        nf = (int(rng.integers(2, 19)), int(rng.integers(2, 19)))
        n_src = log_uniform_int(rng, 50, 5000)
        n_snk = log_uniform_int(rng, 50, 5000)
        T = int(rng.integers(8, 65))
        sites = int(rng.choice([2, 4, 8]))
        out.append(dict(nf=nf, n_src=n_src, n_snk=n_snk, T=T, M=12 * sites))
    return out


def batch_job(j: int, shape: dict | None = None, **over) -> Workload:
    """Job ``j`` of the batched workload (its own seeds); keyword overrides
    shrink it for tests (e.g. ``T=2, n_src=100``)."""
    cfg = dict(batch_shapes(j + 1)[j] if shape is None else shape)
    cfg.update(over)
    nf = tuple(int(n) for n in cfg["nf"])

    def g(stream):
        return np.random.Generator(np.random.PCG64(
            np.random.SeedSequence([SEED_BASE, BATCH_SEED_K, j, stream])))

    S = make_propagator(g(0), cfg["T"], cfg["M"], 0.0)
    src = make_tree_terms(g(1), cfg["n_src"], cfg["M"], nf, 8, 4)
    snk = make_tree_terms(g(2), cfg["n_snk"], cfg["M"], nf, 8, 4)
    w_src = g(3).standard_normal(cfg["n_src"])
    w_snk = g(4).standard_normal(cfg["n_snk"])
    full = dict(cfg, k=BATCH_SEED_K, terms="tree", branching=8, depth=4, decay=0.0, job=j)
    return Workload(f"batch[{j}]", S, src, snk, w_src, w_snk, nf, full)
