"""Source-term graph and greedy dominating set (oracle; test infrastructure
only).  Integer work: the library's planner must reproduce these arrays
bit for bit.

Sec. 3 of the paper: put the matrices in a graph with an edge wherever two of
them differ in a single row, pick a dominating set with the greedy rule
(take the vertex of highest degree, drop it and its neighbours, repeat), and
build the graph over source terms only, since that is O(N^2) rather than
O(N^4) and does not depend on the gauge configuration.  Sec. 2: source terms
i and j that differ only in their r-th element give G^(jk) = G^(ik) + u v^T
with u the unit vector of row r.

Readings taken here (the paper leaves them open):
* edge: positional Hamming distance exactly 1 between the concatenated
  flavour-major index tuples; the differing position (f, r) is the row r of
  flavour block f that changes;
* "R2" (default): the set-cover form of the greedy rule on closed
  neighbourhoods.  Every vertex stays eligible; each step picks the vertex
  whose closed neighbourhood holds the most still-uncovered vertices (lowest
  index on ties), makes it a dominator (taking it out of an earlier
  dominator's children if it was already covered) and gives it every
  still-uncovered vertex of its neighbourhood as children;
* "R1": the literal rule.  Only remaining vertices are eligible, degree is
  counted in the graph induced on the remaining vertices (lowest index on
  ties), and the chosen vertex and its remaining neighbours are removed.
  The dominators it returns are pairwise non-adjacent.
* "prune" (optional, after either rule): Sec. 3 names a better
  dominating-set approximation as the first improvement.  Here that is the
  classic reverse-delete pass: dominators are visited in reverse pick order
  and one is dropped when every vertex of its closed neighbourhood is still
  dominated by another kept dominator.  The result is an irredundant
  dominating set, never larger than the greedy one.  A vertex whose owner
  was dropped (the dropped dominator included) moves to the kept dominator
  of its closed neighbourhood that was picked first; every other vertex
  keeps its owner.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

R2 = 2
R1 = 1


def hamming1_pairs(terms, chunk=256):
    """All (i, j), i < j, whose tuples differ in exactly one position, by
    brute-force comparison of every pair.  Returns int64 [E][2]."""
    terms = np.asarray(terms)
    n = len(terms)
    out = []
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        diff = (terms[lo:hi, None, :] != terms[None, :, :]).sum(axis=2)
        ii, jj = np.nonzero(diff == 1)
        ii = ii + lo
        keep = ii < jj
        out.append(np.stack([ii[keep], jj[keep]], axis=1))
    if not out:
        return np.zeros((0, 2), dtype=np.int64)
    return np.concatenate(out).astype(np.int64)


def adjacency(terms) -> sp.csr_matrix:
    n = len(terms)
    e = hamming1_pairs(terms)
    data = np.ones(2 * len(e), dtype=np.int64)
    rows = np.concatenate([e[:, 0], e[:, 1]])
    cols = np.concatenate([e[:, 1], e[:, 0]])
    return sp.csr_matrix((data, (rows, cols)), shape=(n, n))


def differing_position(a, b) -> int:
    d = np.nonzero(np.asarray(a) != np.asarray(b))[0]
    assert len(d) == 1, "not at Hamming distance 1"
    return int(d[0])


def greedy(terms, policy=R2, adj=None):
    """Run the greedy rule.  Returns (dom_order list, owner int64[N]);
    owner[d] == d for a dominator."""
    terms = np.asarray(terms)
    n = len(terms)
    if adj is None:
        adj = adjacency(terms)
    owner = np.full(n, -1, dtype=np.int64)
    dom_order = []
    if policy == R2:
        closed = adj + sp.identity(n, dtype=np.int64, format="csr")
        uncovered = np.ones(n, dtype=np.int64)
        while uncovered.any():
            gain = closed @ uncovered            # recomputed from scratch
            v = int(np.argmax(gain))             # first maximum = lowest index
            dom_order.append(v)
            nb = closed.indices[closed.indptr[v]:closed.indptr[v + 1]]
            for u in nb:
                if uncovered[u]:
                    uncovered[u] = 0
                    owner[u] = v
            owner[v] = v
    elif policy == R1:
        remaining = np.ones(n, dtype=np.int64)
        while remaining.any():
            deg = adj @ remaining                # degree in the induced graph
            deg = np.where(remaining == 1, deg, -1)
            v = int(np.argmax(deg))
            dom_order.append(v)
            owner[v] = v
            remaining[v] = 0
            nb = adj.indices[adj.indptr[v]:adj.indptr[v + 1]]
            for u in nb:
                if remaining[u]:
                    remaining[u] = 0
                    owner[u] = v
    else:
        raise ValueError("policy must be R1 or R2")
    return dom_order, owner


def prune(dom_order, owner, adj):
    """Reverse delete (module header, "prune").  Returns the kept dominators
    in pick order and the new owner array."""
    n = adj.shape[0]
    closed = (adj + sp.identity(n, dtype=np.int64, format="csr")).tocsr()
    cover = np.zeros(n, dtype=np.int64)       # kept dominators over each vertex
    for v in dom_order:
        cover[closed.indices[closed.indptr[v]:closed.indptr[v + 1]]] += 1
    kept = set(int(v) for v in dom_order)
    for v in reversed(dom_order):
        nb = closed.indices[closed.indptr[v]:closed.indptr[v + 1]]
        if np.all(cover[nb] >= 2):
            cover[nb] -= 1
            kept.discard(int(v))
    order = [int(v) for v in dom_order if int(v) in kept]
    new_owner = np.array(owner, dtype=np.int64, copy=True)
    for u in range(n):
        if int(new_owner[u]) in kept:
            continue
        nb = set(closed.indices[closed.indptr[u]:closed.indptr[u + 1]].tolist())
        new_owner[u] = next(v for v in order if v in nb)
    return order, new_owner


def build(terms, nf, policy=R2, prune_set=False):
    """Tree arrays in the library's export format.

    Returns dict with n_dom, dom_order (int32[N], -1 past n_dom), owner,
    flav, pos (int32[N]; flav = pos = -1 for dominators)."""
    terms = np.asarray(terms)
    n = len(terms)
    adj = adjacency(terms)
    dom_order, owner = greedy(terms, policy, adj)
    if prune_set:
        dom_order, owner = prune(dom_order, owner, adj)
    offs = np.concatenate([[0], np.cumsum(nf)]).astype(int)
    flav = np.full(n, -1, dtype=np.int32)
    pos = np.full(n, -1, dtype=np.int32)
    for u in range(n):
        d = int(owner[u])
        if d == u:
            continue
        p = differing_position(terms[u], terms[d])
        f = int(np.searchsorted(offs, p, side="right") - 1)
        flav[u] = f
        pos[u] = p - offs[f]
    order = np.full(n, -1, dtype=np.int32)
    order[:len(dom_order)] = dom_order
    return dict(n_dom=len(dom_order), dom_order=order,
                owner=owner.astype(np.int32), flav=flav, pos=pos)


def groups(tree):
    """Per dominator (in dom_order): list of ((f, r), [children ascending])
    with (f, r) ascending."""
    n_dom = tree["n_dom"]
    owner = tree["owner"]
    kids = {}
    for u in range(len(owner)):           # ascending u
        d = int(owner[u])
        if d != u:
            kids.setdefault(d, []).append(u)
    out = []
    for d in tree["dom_order"][:n_dom]:
        d = int(d)
        by = {}
        for u in kids.get(d, []):
            by.setdefault((int(tree["flav"][u]), int(tree["pos"][u])), []).append(u)
        out.append((d, sorted(by.items())))
    return out
