"""Host side of the C ABI, no GPU needed: the library loads and exports every
declared symbol, the planner's tree is bit-exact with the oracle's, and
invalid input is rejected with the documented status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import tree as ot
from paper_1411_3691_amd import _lib, mhc
from paper_1411_3691_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mhc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mhc_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert "mhc_contract" in names and "mhc_tree_build" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"
    assert L.mhc_version() >= 202
    assert "mhc_probe_fma64" in names


def test_probe_rejects_bad_arguments_before_launching():
    # host-side checks only: nothing is enqueued on these paths
    L = _lib.lib()
    E_ARG = -1
    assert L.mhc_probe_fma64(None, 1, 1, None) == E_ARG


def tree_matches_oracle(terms, nf, M, policy, prune=False):
    t = mhc.Tree(mhc.Terms(terms, nf, M), policy=policy, prune=prune)
    got = t.export()
    want = ot.build(terms, nf, policy=ot.R2 if policy == "R2" else ot.R1,
                    prune_set=prune)
    assert got["n_dom"] == want["n_dom"]
    for k in ("dom_order", "owner", "flav", "pos"):
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)
    st = t.stats()
    g = ot.groups(want)
    assert st["n_dom"] == want["n_dom"]
    assert st["n_groups"] == sum(len(x[1]) for x in g)
    assert st["n_children"] == len(terms) - want["n_dom"]
    groups_match_oracle(t.groups(), g)


def groups_match_oracle(got, want_groups, share=True):
    """The library's group tables (what the kernels read) equal the oracle's
    groups bit for bit: per dominator in pick order, (f, r) ascending,
    children ascending; without sharing every child is its own group."""
    dom_grp, gf, gr, gp, gc = (got[k] for k in ("dom_grp", "grp_f", "grp_r", "grp_ptr",
                                                "grp_child"))
    assert dom_grp[0] == 0 and gp[0] == 0
    flat = []
    for d, gl in want_groups:
        if share:
            flat.append(gl)
        else:
            flat.append([((f, r), [c]) for (f, r), kids in gl for c in kids])
    assert len(dom_grp) == len(flat) + 1
    for k, gl in enumerate(flat):
        lo, hi = int(dom_grp[k]), int(dom_grp[k + 1])
        assert hi - lo == len(gl), k
        for q, ((f, r), kids) in enumerate(gl):
            g = lo + q
            assert (int(gf[g]), int(gr[g])) == (f, r), (k, q)
            assert gc[gp[g]:gp[g + 1]].tolist() == kids, (k, q)
    assert int(dom_grp[-1]) == len(gf) == len(gr) == len(gp) - 1
    assert int(gp[-1]) == len(gc)


@pytest.mark.parametrize("prune", [False, True])
@pytest.mark.parametrize("policy", ["R2", "R1"])
@pytest.mark.parametrize("name,over", [
    ("tiny", {}),
    ("mid", dict(T=1)),
    ("mid", dict(T=1, n_src=500, branching=3, depth=2)),
    ("grad", dict(T=1)),
])
def test_tree_bit_exact_workloads(name, over, policy, prune):
    w = W.workload(name, **over)
    tree_matches_oracle(w.src, w.nf, w.M, policy, prune)


def test_tree_bit_exact_large():
    # 20000 source terms of 2 x 12 quarks, 96 quark indices
    w = W.workload("large", T=1)
    tree_matches_oracle(w.src, w.nf, w.M, "R2")


@pytest.mark.parametrize("prune", [False, True])
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("policy", ["R2", "R1"])
def test_tree_bit_exact_adversarial(seed, policy, prune):
    rng = np.random.default_rng(seed)
    # dense small index space: many ties, stars, cliques and long chains
    M = 4 + seed
    nf = (2, 1)
    n = min(120, (M * (M - 1) * M * 3) // 4)   # leave some tuples unused
    rows = set()
    while len(rows) < n:
        a = tuple(rng.choice(M, 2, replace=False)) + (int(rng.integers(M)),)
        rows.add(a)
    terms = np.array(sorted(rows), dtype=np.int32)
    rng.shuffle(terms)
    tree_matches_oracle(terms, nf, M, policy, prune)


def test_tree_special_graphs():
    star = np.array([[5, 1, 2, 3], [0, 6, 2, 3], [0, 1, 7, 3], [0, 1, 2, 3], [0, 1, 2, 8]])
    no_edges = np.array([[i, i + 10, i + 20, i + 30] for i in range(6)])
    clique = np.array([[c, 1, 2, 3] for c in (4, 5, 6, 7, 0)])
    single = np.array([[0, 1, 2, 3]])
    for terms in (star, no_edges, clique, single):
        for pol in ("R1", "R2"):
            tree_matches_oracle(terms, (2, 2), 40, pol)


# -------------------------------------------------------------- errors

def status_of(fn, *args):
    return fn(*args)


def test_terms_errors():
    L = _lib.lib()
    nf = np.array([3], dtype=np.int32)
    h = ctypes.c_void_p()
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    # repeated index within a flavour -> MHC_E_TERM, message names the term
    bad = np.array([[0, 1, 2], [3, 3, 4]], dtype=np.int32)
    assert L.mhc_terms_create(2, 1, P(nf), P(bad), 10, ctypes.byref(h)) == -2
    assert b"term 1" in L.mhc_last_error()
    assert not h.value
    # index outside [0, M)
    bad = np.array([[0, 1, 10]], dtype=np.int32)
    assert L.mhc_terms_create(1, 1, P(nf), P(bad), 10, ctypes.byref(h)) == -2
    bad = np.array([[0, -1, 2]], dtype=np.int32)
    assert L.mhc_terms_create(1, 1, P(nf), P(bad), 10, ctypes.byref(h)) == -2
    # a repeat across flavours is allowed (different quark fields)
    nf2 = np.array([2, 1], dtype=np.int32)
    ok = np.array([[0, 1, 0]], dtype=np.int32)
    assert L.mhc_terms_create(1, 2, P(nf2), P(ok), 10, ctypes.byref(h)) == 0
    L.mhc_terms_destroy(h)
    # argument errors
    good = np.array([[0, 1, 2]], dtype=np.int32)
    assert L.mhc_terms_create(0, 1, P(nf), P(good), 10, ctypes.byref(h)) == -1
    assert L.mhc_terms_create(1, 0, P(nf), P(good), 10, ctypes.byref(h)) == -1
    assert L.mhc_terms_create(1, 1, P(nf), P(good), 0, ctypes.byref(h)) == -1
    assert L.mhc_terms_create(1, 1, P(nf), P(good), 256, ctypes.byref(h)) == -1
    assert L.mhc_terms_create(1, 1, None, P(good), 10, ctypes.byref(h)) == -1
    assert L.mhc_terms_create(1, 1, P(nf), None, 10, ctypes.byref(h)) == -1
    assert L.mhc_terms_create(1, 1, P(nf), P(good), 10, None) == -1
    big = np.array([40], dtype=np.int32)
    assert L.mhc_terms_create(1, 1, P(big), P(good), 100, ctypes.byref(h)) == -1
    with pytest.raises(_lib.MhcError) as ei:
        mhc.Terms([[1, 1, 2]], (3,), 10)
    assert ei.value.status == -2


def test_null_handles_and_destroy():
    L = _lib.lib()
    L.mhc_terms_destroy(None)
    L.mhc_tree_destroy(None)
    L.mhc_plan_destroy(None)
    h = ctypes.c_void_p()
    assert L.mhc_tree_build(None, 2, ctypes.byref(h)) == -1
    assert L.mhc_tree_export(None, None, None, None, None, None) == -1
    assert L.mhc_tree_stats(None, None, None, None) == -1
    assert L.mhc_plan_create(None, None, None, ctypes.byref(h)) == -1
    assert L.mhc_contract(None, 1, 1, None, None, None, None, None, None, None, 0, None) == -1
    assert L.mhc_plan_status(None, None, None) == -1
    assert L.mhc_plan_attach_sink_tree(None, None, None) == -1
    assert L.mhc_contract_backward(None, 1, 1, None, None, None, None, None, None, None,
                                   None) == -1
    assert L.mhc_terms_shape(None, None, None, None) == -1
    t = mhc.Terms([[0, 1]], (2,), 5)
    assert L.mhc_tree_build(t.handle, 3, ctypes.byref(h)) == -1   # unknown policy
    assert b"policy" in L.mhc_last_error()


def test_tree_without_sharing_has_one_group_per_child():
    w = W.workload("mid", T=1, n_src=500, n_snk=10)
    t = mhc.Terms(w.src, w.nf, w.M)
    shared, alone = mhc.Tree(t), mhc.Tree(t, share=False)
    a, b = shared.export(), alone.export()
    for key in ("dom_order", "owner", "flav", "pos"):
        assert np.array_equal(a[key], b[key])
    sa, sb = shared.stats(), alone.stats()
    assert sb["n_groups"] == sb["n_children"] == sa["n_children"]
    assert sa["n_groups"] < sa["n_children"]
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.mhc_tree_build(t.handle, 3 | _lib.TREE_NO_SHARING, ctypes.byref(h)) == -1


def test_batch_argument_errors_before_device_work():
    L = _lib.lib()
    L.mhc_batch_destroy(None)
    h = ctypes.c_void_p()
    plans = (ctypes.c_void_p * 1)(None)
    T = np.array([4], dtype=np.int32)
    Tp = T.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert L.mhc_batch_create(None, Tp, 1, 1, None, ctypes.byref(h)) == -1
    assert L.mhc_batch_create(plans, Tp, 0, 1, None, ctypes.byref(h)) == -1
    assert L.mhc_batch_create(plans, Tp, 1, 1, None, None) == -1
    assert L.mhc_batch_create(plans, Tp, 1, 5, None, ctypes.byref(h)) == -1
    assert b"method" in L.mhc_last_error()
    for bad in ((3, 0, 0), (0, 9, 0), (0, -1, 0), (0, 0, -4)):
        sc = _lib.Schedule(*bad)
        assert L.mhc_batch_create(plans, Tp, 1, 1, ctypes.byref(sc), ctypes.byref(h)) == -1
        assert b"schedule" in L.mhc_last_error()
    assert not h.value
    assert L.mhc_batch_run(None, None, None, None, None, None, None) == -1
    assert L.mhc_batch_info(None, None, None, None) == -1


def test_plan_shape_mismatch_is_reported_before_device_work():
    # differing M or flavour structure between source and sink terms
    src = mhc.Terms([[0, 1, 2]], (2, 1), 10)
    tree = mhc.Tree(src)
    L = _lib.lib()
    h = ctypes.c_void_p()
    for snk in (mhc.Terms([[0, 1, 2]], (2, 1), 11), mhc.Terms([[0, 1, 2]], (1, 2), 10),
                mhc.Terms([[0, 1]], (2,), 10)):
        assert L.mhc_plan_create(tree.handle, snk.handle, None, ctypes.byref(h)) == -3
    # blocks above the kernels' limit are refused as unsupported (checked
    # before any device work)
    src = mhc.Terms([list(range(25))], (25,), 30)
    snk = mhc.Terms([list(range(25))], (25,), 30)
    assert L.mhc_plan_create(mhc.Tree(src).handle, snk.handle, None, ctypes.byref(h)) == -7
    src = mhc.Terms([[0, 1]], (2,), 100)
    snk = mhc.Terms([[0, 1]], (2,), 100)
    assert L.mhc_plan_create(mhc.Tree(src).handle, snk.handle, None, ctypes.byref(h)) == -7


def test_terms_shape():
    t = mhc.Terms([[0, 1, 2], [3, 4, 5]], (2, 1), 9)
    L = _lib.lib()
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert L.mhc_terms_shape(t.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == 0
    assert (a.value, b.value, c.value) == (2, 2, 9)


def test_prune_flag_combines_with_no_sharing_and_rejects_bad_policy():
    w = W.workload("mid", T=1, n_src=500, n_snk=10)
    t = mhc.Terms(w.src, w.nf, w.M)
    a = mhc.Tree(t, prune=True)
    b = mhc.Tree(t, share=False, prune=True)
    ea, eb = a.export(), b.export()
    for key in ("n_dom", "dom_order", "owner", "flav", "pos"):
        assert np.array_equal(ea[key], eb[key])
    assert b.stats()["n_groups"] == b.stats()["n_children"]
    assert ea["n_dom"] <= mhc.Tree(t).export()["n_dom"]
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.mhc_tree_build(t.handle, 3 | _lib.TREE_PRUNE, ctypes.byref(h)) == -1
    assert b"policy" in L.mhc_last_error()


@pytest.mark.parametrize("name,over", [("tiny", {}), ("mid", dict(T=1))])
def test_group_tables_without_sharing(name, over):
    # the ablation's tables: every child its own group, same order
    w = W.workload(name, **over)
    t = mhc.Tree(mhc.Terms(w.src, w.nf, w.M), share=False)
    want = ot.build(w.src, w.nf)
    groups_match_oracle(t.groups(), ot.groups(want), share=False)


def permuted_workload(seed=7, **over):
    """The mid workload with every flavour block of every term in a random
    order (the input of the set-edge ablation)."""
    w = W.workload("mid", **over)
    rng = np.random.default_rng(seed)
    for terms in (w.src, w.snk):
        for u in range(len(terms)):
            for o, k in ((0, w.nf[0]), (w.nf[0], w.nf[1])):
                terms[u, o:o + k] = terms[u, o:o + k][rng.permutation(k)]
    return w


@pytest.mark.parametrize("prune", [False, True])
@pytest.mark.parametrize("policy", ["R2", "R1"])
def test_set_edge_tree_bit_exact(policy, prune):
    w = permuted_workload(T=1, n_src=400)
    t = mhc.Tree(mhc.Terms(w.src, w.nf, w.M), policy=policy, prune=prune, set_edges=True)
    got = t.export()
    want = ot.build(w.src, w.nf, policy=ot.R2 if policy == "R2" else ot.R1, prune_set=prune,
                    edges="set")
    assert got["n_dom"] == want["n_dom"]
    for k in ("dom_order", "owner", "flav", "pos"):
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)
    new, sign = t.children()
    np.testing.assert_array_equal(new, want["new"])
    np.testing.assert_array_equal(sign, want["sign"])
    groups_match_oracle(t.groups(), ot.groups(want))
    assert (sign == -1).any() and (sign == 1).any()


def test_positional_tree_children_export():
    w = W.workload("mid", T=1, n_src=300)
    t = mhc.Tree(mhc.Terms(w.src, w.nf, w.M))
    want = ot.build(w.src, w.nf)
    new, sign = t.children()
    np.testing.assert_array_equal(new, want["new"])
    np.testing.assert_array_equal(sign, want["sign"])
