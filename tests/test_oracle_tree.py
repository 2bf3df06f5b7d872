"""Pins of the oracle's source-term graph and greedy dominating set (Sec. 3)
against brute force, hand-checkable graphs and the greedy-choice property,
all computed here with plain Python loops that share nothing with
``oracle.tree``."""
import itertools

import numpy as np
import pytest

from oracle import tree as ot
from paper_1411_3691_amd import workloads as W


def plain_neighbours(terms):
    n = len(terms)
    nb = [set() for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if i != j and sum(int(a != b) for a, b in zip(terms[i], terms[j])) == 1:
                nb[i].add(j)
    return nb


def random_terms(seed, n=60, sn=4, M=5):
    rng = np.random.default_rng(seed)
    return rng.integers(0, M, size=(n, sn))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_hamming_pairs_brute_force(seed):
    terms = random_terms(seed)
    nb = plain_neighbours(terms.tolist())
    e = ot.hamming1_pairs(terms)
    got = {(int(a), int(b)) for a, b in e}
    want = {(i, j) for i in range(len(terms)) for j in nb[i] if i < j}
    assert got == want


def replay_r2(terms, tree):
    """Check every step of R2 against gains recomputed with plain loops."""
    nb = plain_neighbours(terms.tolist())
    n = len(terms)
    covered = [False] * n
    owner = [-1] * n
    for step in range(tree["n_dom"]):
        gains = [int(not covered[v]) + sum(1 for u in nb[v] if not covered[u])
                 for v in range(n)]
        best = max(gains)
        v = gains.index(best)        # lowest index among the maxima
        assert int(tree["dom_order"][step]) == v, step
        for u in [v] + sorted(nb[v]):
            if not covered[u]:
                covered[u] = True
                owner[u] = v
        owner[v] = v
    assert all(covered)
    assert list(tree["owner"]) == owner


def replay_r1(terms, tree):
    nb = plain_neighbours(terms.tolist())
    n = len(terms)
    remaining = set(range(n))
    owner = [-1] * n
    for step in range(tree["n_dom"]):
        degs = {v: sum(1 for u in nb[v] if u in remaining) for v in remaining}
        best = max(degs.values())
        v = min(u for u in remaining if degs[u] == best)
        assert int(tree["dom_order"][step]) == v, step
        owner[v] = v
        remaining.discard(v)
        for u in nb[v]:
            if u in remaining:
                owner[u] = v
                remaining.discard(u)
    assert not remaining
    assert list(tree["owner"]) == owner


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_r2_greedy_choice_property(seed):
    terms = random_terms(seed, n=80)
    tree = ot.build(terms, (2, 2), policy=ot.R2)
    replay_r2(terms, tree)


@pytest.mark.parametrize("seed", [6, 7])
def test_r1_greedy_choice_property_and_independence(seed):
    terms = random_terms(seed, n=80)
    tree = ot.build(terms, (2, 2), policy=ot.R1)
    replay_r1(terms, tree)
    nb = plain_neighbours(terms.tolist())
    doms = [int(d) for d in tree["dom_order"][:tree["n_dom"]]]
    for a, b in itertools.combinations(doms, 2):
        assert b not in nb[a]


def check_invariants(terms, nf, tree):
    n = len(terms)
    offs = np.concatenate([[0], np.cumsum(nf)])
    doms = set(int(d) for d in tree["dom_order"][:tree["n_dom"]])
    assert len(doms) == tree["n_dom"]
    assert all(int(d) == -1 for d in tree["dom_order"][tree["n_dom"]:])
    for u in range(n):
        d = int(tree["owner"][u])
        if u in doms:
            assert d == u and tree["flav"][u] == -1 and tree["pos"][u] == -1
            continue
        assert d in doms
        diff = [p for p in range(len(terms[u])) if terms[u][p] != terms[d][p]]
        assert len(diff) == 1
        f = int(tree["flav"][u])
        assert offs[f] + int(tree["pos"][u]) == diff[0]
        assert 0 <= tree["pos"][u] < nf[f]


def test_special_graphs():
    # star: one centre, leaves differ from it in one position each and from
    # each other in two -> a single dominator (the centre, index 3)
    centre = [0, 1, 2, 3]
    star = [[5, 1, 2, 3], [0, 6, 2, 3], [0, 1, 7, 3], centre, [0, 1, 2, 8]]
    for pol in (ot.R1, ot.R2):
        t = ot.build(np.array(star), (2, 2), policy=pol)
        assert t["n_dom"] == 1 and t["dom_order"][0] == 3
        check_invariants(star, (2, 2), t)
    # clique of same-position siblings: complete graph -> lowest index wins
    clique = np.array([[c, 1, 2, 3] for c in (4, 5, 6, 7, 0)])
    t = ot.build(clique, (2, 2))
    assert t["n_dom"] == 1 and t["dom_order"][0] == 0
    assert list(t["pos"]) == [-1, 0, 0, 0, 0] and list(t["flav"]) == [-1, 0, 0, 0, 0]
    # no edges: every term is its own dominator, in index order
    far = np.array([[i, i + 10, i + 20, i + 30] for i in range(6)])
    t = ot.build(far, (2, 2))
    assert t["n_dom"] == 6 and list(t["dom_order"]) == list(range(6))
    # duplicates are at distance 0: not neighbours of each other
    dup = np.array([[0, 1, 2, 3], [0, 1, 2, 3]])
    t = ot.build(dup, (2, 2))
    assert t["n_dom"] == 2
    # path a-b-c-d-e (each step changes one position, ends are far apart)
    path = np.array([[0, 0, 0, 0], [1, 0, 0, 0], [1, 1, 0, 0], [1, 1, 1, 0], [1, 1, 1, 1]])
    t = ot.build(path, (2, 2), policy=ot.R2)
    # gains: 2,3,3,3,2 -> pick 1 (covers 0,1,2), then gains of 3 and 4... 3 covers {3,4}
    assert list(t["dom_order"][:t["n_dom"]]) == [1, 3]
    assert list(t["owner"]) == [1, 1, 1, 3, 3]
    t = ot.build(path, (2, 2), policy=ot.R1)
    assert list(t["dom_order"][:t["n_dom"]]) == [1, 3]


def test_r2_can_promote_a_covered_vertex():
    # 0 covers 1 and 2; later 1 (already covered) is the best choice to
    # cover 3, 4, 5, so it becomes a dominator and leaves 0's children.
    terms = np.array([
        [0, 0, 0, 0],   # 0
        [1, 0, 0, 0],   # 1  (nb of 0)
        [0, 1, 0, 0],   # 2  (nb of 0)
        [1, 2, 0, 0],   # 3  (nb of 1)
        [1, 0, 2, 0],   # 4  (nb of 1)
        [1, 0, 0, 2],   # 5  (nb of 1)
        [0, 0, 3, 0],   # 6  (nb of 0)
        [0, 0, 0, 3],   # 7  (nb of 0)
    ])
    t = ot.build(terms, (2, 2), policy=ot.R2)
    replay_r2(terms, t)
    check_invariants(terms, (2, 2), t)
    assert list(t["dom_order"][:t["n_dom"]]) == [0, 1]
    assert t["owner"][1] == 1 and t["owner"][3] == 1 and t["owner"][2] == 0


def test_greedy_close_to_minimum_on_tiny_graphs():
    # R2 is the set-cover greedy: |D| <= H(max closed degree) * |D_min|.
    rng = np.random.default_rng(21)
    for _ in range(5):
        terms = rng.integers(0, 3, size=(11, 3))
        terms = np.unique(terms, axis=0)
        nb = plain_neighbours(terms.tolist())
        n = len(terms)
        best = None
        for k in range(1, n + 1):
            for D in itertools.combinations(range(n), k):
                cov = set(D)
                for v in D:
                    cov |= nb[v]
                if len(cov) == n:
                    best = k
                    break
            if best:
                break
        t = ot.build(terms, (1, 2))
        delta = max(len(s) for s in nb) + 1
        H = sum(1.0 / k for k in range(1, delta + 1))
        assert best <= t["n_dom"] <= H * best + 1e-9


def test_workload_tree_statistics():
    # Synthetic "mid" source terms (2000 terms of 2 x 6 quarks): the greedy
    # leaves roughly one term in eight as a dominator, inside the range of
    # dominating-set fractions the paper reports (Sec. 4, about 0.09-0.13).
    w = W.workload("mid", T=1)
    t = ot.build(w.src, w.nf)
    check_invariants(w.src, w.nf, t)
    rho = t["n_dom"] / len(w.src)
    assert 0.08 <= rho <= 0.14


def brute_force_minimum(nb, n):
    for k in range(1, n + 1):
        for D in itertools.combinations(range(n), k):
            cov = set(D)
            for v in D:
                cov |= nb[v]
            if len(cov) == n:
                return k
    return n


def test_prune_gives_irredundant_dominating_sets():
    # Reverse delete after either greedy rule: the kept set still dominates,
    # no kept dominator can be dropped, it keeps the greedy pick order, it is
    # no larger than the greedy set and no smaller than the minimum (brute
    # force); owners are kept dominators next to their children, a child
    # keeps its greedy owner when that one was kept and otherwise takes the
    # kept neighbour picked first.  R1's dominators are pairwise
    # non-adjacent, each the only dominator over itself: nothing to drop.
    rng = np.random.default_rng(33)
    shrunk = 0
    for _ in range(40):
        terms = np.unique(rng.integers(0, 3, size=(14, 3)), axis=0)
        n = len(terms)
        nb = plain_neighbours(terms.tolist())
        best = brute_force_minimum(nb, n)
        for pol in (ot.R1, ot.R2):
            g = ot.build(terms, (1, 2), policy=pol)
            p = ot.build(terms, (1, 2), policy=pol, prune_set=True)
            G = [int(v) for v in g["dom_order"][:g["n_dom"]]]
            D = [int(v) for v in p["dom_order"][:p["n_dom"]]]
            it = iter(G)
            assert all(v in it for v in D)
            cov = [0] * n
            for v in D:
                cov[v] += 1
                for u in nb[v]:
                    cov[u] += 1
            assert min(cov) >= 1
            for v in D:
                assert any(cov[u] == 1 for u in [v, *nb[v]])
            assert best <= len(D) <= len(G)
            for u in range(n):
                o = int(p["owner"][u])
                if u in D:
                    assert o == u
                    continue
                assert o in D and o in nb[u]
                if int(g["owner"][u]) in D:
                    assert o == int(g["owner"][u])
                else:
                    assert o == next(v for v in D if v in nb[u])
                d = next(q for q in range(3) if terms[u][q] != terms[o][q])
                assert (p["flav"][u], p["pos"][u]) == ((0, 0) if d == 0 else (1, d - 1))
            if pol == ot.R1:
                assert D == G
            else:
                shrunk += len(D) < len(G)
    assert shrunk > 0


def test_prune_near_minimum_on_mid_terms():
    # 2000 mid source terms: the exact minimum dominating set from an integer
    # program (every closed neighbourhood holds a chosen term; HiGHS through
    # scipy) bounds the pruned set from below; the greedy set is about 9 %
    # above it, the pruned one within 2 %.
    import scipy.sparse as sps
    from scipy.optimize import Bounds, LinearConstraint, milp
    w = W.workload("mid", T=1)
    terms = np.asarray(w.src)
    n = len(terms)
    nb = ot.hamming1_pairs(terms)
    rows = np.concatenate([nb[:, 0], nb[:, 1], np.arange(n)])
    cols = np.concatenate([nb[:, 1], nb[:, 0], np.arange(n)])
    A = sps.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    res = milp(c=np.ones(n), constraints=LinearConstraint(A, lb=1, ub=np.inf),
               integrality=np.ones(n), bounds=Bounds(0, 1))
    assert res.status == 0
    opt = int(round(res.fun))
    g = ot.build(terms, w.nf)["n_dom"]
    p = ot.build(terms, w.nf, prune_set=True)["n_dom"]
    assert opt <= p <= g
    assert p <= 1.02 * opt and g >= 1.05 * opt


# ------------------------------------------------------------ groups

def regroup_by_loops(tree, nf):
    """Groups of every dominator rebuilt with plain loops: for each dominator
    in pick order, for every flavour f and row r in ascending order, scan
    all terms in ascending index and keep the children owned by it that
    differ in (f, r).  Sec. 2: those children share the solve G_f^-1 e_r."""
    n = len(tree["owner"])
    out = []
    for k in range(tree["n_dom"]):
        d = int(tree["dom_order"][k])
        gl = []
        for f in range(len(nf)):
            for r in range(nf[f]):
                kids = []
                for u in range(n):
                    if u != d and int(tree["owner"][u]) == d and \
                            int(tree["flav"][u]) == f and int(tree["pos"][u]) == r:
                        kids.append(u)
                if kids:
                    gl.append(((f, r), kids))
        out.append((d, gl))
    return out


def test_groups_worked_example():
    # star of the special-graph test, with a second leaf in row 0 of
    # flavour 0: the centre (term 3) dominates every leaf; leaves 0 and 5
    # change the same row (flavour 0, row 0) and share one group, listed in
    # ascending term order; the groups are ordered by (flavour, row)
    star = np.array([[5, 1, 2, 3], [0, 6, 2, 3], [0, 1, 7, 3], [0, 1, 2, 3], [0, 1, 2, 8],
                     [4, 1, 2, 3]])
    t = ot.build(star, (2, 2))
    assert ot.groups(t) == [(3, [((0, 0), [0, 5]), ((0, 1), [1]), ((1, 0), [2]),
                                 ((1, 1), [4])])]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("policy", [ot.R1, ot.R2])
def test_groups_match_plain_regrouping(seed, policy):
    # dense index spaces: many same-row siblings, children in every flavour
    terms = random_terms(seed, n=80, sn=5, M=4)
    terms = np.unique(terms, axis=0)
    rng = np.random.default_rng(100 + seed)
    terms = terms[rng.permutation(len(terms))]
    nf = (3, 2)
    for prune in (False, True):
        t = ot.build(terms, nf, policy=policy, prune_set=prune)
        assert ot.groups(t) == regroup_by_loops(t, nf)
        n_groups = sum(len(g) for _, g in ot.groups(t))
        n_child = sum(len(c) for _, g in ot.groups(t) for _, c in g)
        assert n_child == len(terms) - t["n_dom"]
        assert n_groups <= n_child


def test_groups_match_plain_regrouping_mid():
    w = W.workload("mid", T=1, n_src=600)
    t = ot.build(w.src, w.nf)
    assert ot.groups(t) == regroup_by_loops(t, w.nf)


# ------------------------------------------------------------ set edges

def permuted_terms(seed, n=70, nf=(3, 2), M=6):
    """Random terms whose flavour blocks come in random orders."""
    rng = np.random.default_rng(seed)
    rows = set()
    while len(rows) < n:
        t = []
        for k in nf:
            t += [int(v) for v in rng.choice(M, k, replace=False)]
        rows.add(tuple(t))
    return np.array(sorted(rows))[rng.permutation(n)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_set_pairs_brute_force(seed):
    nf = (3, 2)
    terms = permuted_terms(seed)
    got = {tuple(e) for e in ot.set1_pairs(terms, nf).tolist()}
    want = set()
    for i in range(len(terms)):
        for j in range(i + 1, len(terms)):
            a, b = terms[i].tolist(), terms[j].tolist()
            d = len(set(a[:3]) - set(b[:3])) + len(set(a[3:]) - set(b[3:]))
            if d == 1:
                want.add((i, j))
    assert got == want
    # every positional neighbour is a set neighbour
    assert {tuple(e) for e in ot.hamming1_pairs(terms).tolist()} <= got


def test_set_child_worked_example():
    # dominator (0 1 2 | 3 4), child (2 5 0 | 4 3): block 0 loses 1 (row 1)
    # and gains 5; b = (0 5 2 | 3 4); the child's blocks are b's reordered by
    # a reversal of three (odd) and a swap (odd): sign +1
    assert ot.set_child([0, 1, 2, 3, 4], [2, 5, 0, 4, 3], (3, 2)) == (0, 1, 5, 1)
    # only the first block reordered by a swap: sign -1
    assert ot.set_child([0, 1, 2, 3, 4], [5, 0, 2, 3, 4], (3, 2)) == (0, 1, 5, -1)
    # positional change: sign +1
    assert ot.set_child([0, 1, 2, 3, 4], [0, 1, 2, 3, 7], (3, 2)) == (1, 1, 7, 1)


@pytest.mark.parametrize("seed", [3, 4])
def test_set_child_sign_by_determinants(seed):
    # det G(child) = sign * det G(b), b the dominator with row r of block f
    # replaced by the new index, checked with LAPACK on a random propagator
    nf = (3, 2)
    terms = permuted_terms(seed)
    rng = np.random.default_rng(50 + seed)
    S = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    snk = [int(v) for v in rng.choice(6, 3, replace=False)] + \
          [int(v) for v in rng.choice(6, 2, replace=False)]
    t = ot.build(terms, nf, edges="set")
    n_checked = 0
    for u in range(len(terms)):
        d = int(t["owner"][u])
        if d == u:
            continue
        f, r, new, sign = (int(t["flav"][u]), int(t["pos"][u]), int(t["new"][u]),
                           int(t["sign"][u]))
        b = terms[d].tolist()
        b[[0, 3][f] + r] = new
        lhs = rhs = 1.0
        for o, k in ((0, 3), (3, 2)):
            lhs *= np.linalg.det(S[np.ix_(terms[u][o:o + k], snk[o:o + k])])
            rhs *= np.linalg.det(S[np.ix_(b[o:o + k], snk[o:o + k])])
        assert abs(lhs - sign * rhs) <= 1e-12 * max(1.0, abs(lhs)), (u, d)
        n_checked += 1
    assert n_checked > 0


@pytest.mark.parametrize("policy", [ot.R1, ot.R2])
def test_set_edges_tree_invariants(policy):
    nf = (3, 2)
    terms = permuted_terms(5)
    t = ot.build(terms, nf, policy=policy, edges="set")
    nb = [set() for _ in range(len(terms))]
    for i, j in ot.set1_pairs(terms, nf).tolist():
        nb[i].add(j)
        nb[j].add(i)
    doms = set(int(d) for d in t["dom_order"][:t["n_dom"]])
    for u in range(len(terms)):
        d = int(t["owner"][u])
        assert d in doms and (d == u or d in nb[u])
    # on permuted blocks the set graph has more edges than the positional
    # one, so the greedy rule needs fewer dominators
    tp = ot.build(terms, nf, policy=policy)
    assert t["n_dom"] <= tp["n_dom"]
