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
* "set" edges (an ablation; Sec. 3 speaks of matrices that differ by a
  single row without fixing the row order): two terms are neighbours when
  their flavour blocks, taken as sets of indices, differ in exactly one
  element.  A child's matrix is then a row permutation of its dominator's
  with one row replaced, so its determinant carries the sign of that
  permutation.
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


def adjacency(terms, nf=None, edges="position") -> sp.csr_matrix:
    """Neighbour graph: positional Hamming distance 1 (default) or, with
    edges="set", set distance 1 (set1_pairs; needs nf)."""
    n = len(terms)
    e = hamming1_pairs(terms) if edges == "position" else set1_pairs(terms, nf)
    data = np.ones(2 * len(e), dtype=np.int64)
    rows = np.concatenate([e[:, 0], e[:, 1]])
    cols = np.concatenate([e[:, 1], e[:, 0]])
    return sp.csr_matrix((data, (rows, cols)), shape=(n, n))


def set_distance(a, b, nf) -> int:
    """Sec. 3 edges read as sets (the set-edge ablation): the number of
    elements of a's flavour blocks that b's blocks lack (blocks of equal
    size, indices distinct within a block)."""
    offs = np.concatenate([[0], np.cumsum(nf)]).astype(int)
    return sum(len(set(np.asarray(a)[offs[f]:offs[f + 1]].tolist())
                   - set(np.asarray(b)[offs[f]:offs[f + 1]].tolist()))
               for f in range(len(nf)))


def set1_pairs(terms, nf, chunk=128):
    """All (i, j), i < j, at set distance exactly 1 (one flavour block
    differs in one element, every other block holds the same indices), by
    comparing every pair: for each block, the elements of i's block found
    anywhere in j's block are counted.  Returns int64 [E][2]."""
    terms = np.asarray(terms)
    n = len(terms)
    offs = np.concatenate([[0], np.cumsum(nf)]).astype(int)
    out = []
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        missing = np.zeros((hi - lo, n), dtype=np.int64)
        for f in range(len(nf)):
            a = terms[lo:hi, offs[f]:offs[f + 1]]          # [c][n_f]
            b = terms[:, offs[f]:offs[f + 1]]              # [N][n_f]
            found = (a[:, :, None, None] == b[None, None, :, :]).any(axis=3)   # [c][n_f][N]
            missing += nf[f] - found.sum(axis=1)
        ii, jj = np.nonzero(missing == 1)
        ii = ii + lo
        keep = ii < jj
        out.append(np.stack([ii[keep], jj[keep]], axis=1))
    if not out:
        return np.zeros((0, 2), dtype=np.int64)
    return np.concatenate(out).astype(np.int64)


def permutation_sign(src, dst) -> int:
    """Sign of the permutation that reorders the distinct values src into
    dst (dst[m] = src[p(m)]), by counting inversions of p."""
    where = {v: k for k, v in enumerate(src)}
    p = [where[v] for v in dst]
    inv = sum(1 for x in range(len(p)) for y in range(x + 1, len(p)) if p[x] > p[y])
    return -1 if inv % 2 else 1


def set_child(dom, child, nf):
    """For terms at set distance 1: (flavour f, row r of the dominator's
    block f that is replaced, the new index, sign).  With b the dominator's
    tuple with row r of block f replaced by the new index, every block of
    the child holds the indices of b's block in some order, so G of the
    child is a row permutation of G with b's rows, and its determinant is
    sign * det(b's G) (Sec. 2: b's block f is the dominator's with one row
    changed)."""
    offs = np.concatenate([[0], np.cumsum(nf)]).astype(int)
    dom = [int(v) for v in dom]
    child = [int(v) for v in child]
    fc = r = new = None
    for f in range(len(nf)):
        bd, bu = dom[offs[f]:offs[f + 1]], child[offs[f]:offs[f + 1]]
        gone = [v for v in bd if v not in bu]
        if gone:
            assert len(gone) == 1 and fc is None, "not at set distance 1"
            fc, r = f, bd.index(gone[0])
            new = [v for v in bu if v not in bd][0]
    assert fc is not None, "not at set distance 1"
    sign = 1
    for f in range(len(nf)):
        b = dom[offs[f]:offs[f + 1]]
        if f == fc:
            b[r] = new
        sign *= permutation_sign(b, child[offs[f]:offs[f + 1]])
    return fc, r, new, sign


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


def build(terms, nf, policy=R2, prune_set=False, edges="position"):
    """Tree arrays in the library's export format.

    Returns dict with n_dom, dom_order (int32[N], -1 past n_dom), owner,
    flav, pos (int32[N]; flav = pos = -1 for dominators), and per child the
    new index of its changed row and the sign of its row permutation
    (new = -1, sign = 0 for dominators; sign 1 for positional edges)."""
    terms = np.asarray(terms)
    n = len(terms)
    adj = adjacency(terms, nf, edges)
    dom_order, owner = greedy(terms, policy, adj)
    if prune_set:
        dom_order, owner = prune(dom_order, owner, adj)
    offs = np.concatenate([[0], np.cumsum(nf)]).astype(int)
    flav = np.full(n, -1, dtype=np.int32)
    pos = np.full(n, -1, dtype=np.int32)
    new = np.full(n, -1, dtype=np.int32)
    sign = np.zeros(n, dtype=np.int32)
    for u in range(n):
        d = int(owner[u])
        if d == u:
            continue
        if edges == "position":
            p = differing_position(terms[u], terms[d])
            f = int(np.searchsorted(offs, p, side="right") - 1)
            flav[u], pos[u], new[u], sign[u] = f, p - offs[f], terms[u][p], 1
        else:
            flav[u], pos[u], new[u], sign[u] = set_child(terms[d], terms[u], nf)
    order = np.full(n, -1, dtype=np.int32)
    order[:len(dom_order)] = dom_order
    return dict(n_dom=len(dom_order), dom_order=order,
                owner=owner.astype(np.int32), flav=flav, pos=pos, new=new, sign=sign)


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
