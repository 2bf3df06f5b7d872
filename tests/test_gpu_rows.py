"""GPU parity of the multi-row group kernels (several rows of a matrix per
lane, blocks up to 24, rows of S staged per tile): the correlator of the
fast path, the scale A and the weighted-row aggregation against the CPU
oracle, on uneven and M = 96 shapes, dominators split over several tiles,
singular dominator blocks and repeated runs."""
import numpy as np
import pytest
import torch

from oracle import contract as oc
from paper_1411_3691_amd import mhc
from paper_1411_3691_amd import workloads as W

pytestmark = pytest.mark.gpu


def setup(w, **tree_kw):
    plan = mhc.Plan(mhc.Tree(mhc.Terms(w.src, w.nf, w.M), **tree_kw),
                    mhc.Terms(w.snk, w.nf, w.M))
    dev = plan.device
    return (plan, torch.from_numpy(w.S).to(dev), torch.from_numpy(w.w_src).to(dev),
            torch.from_numpy(w.w_snk).to(dev))


def check_all_methods(w, plan, S, ws, wk, methods=("plain", "tree", "tree_agg")):
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    for method in methods:
        C = mhc.contract(plan, S, ws, wk, method).cpu().numpy()
        assert np.all(np.abs(C - Cw) <= 1e-9 * Aw), (method, np.max(np.abs(C - Cw) / Aw))
        if method != "tree_agg":
            C2, A2 = (x.cpu().numpy() for x in
                      mhc.contract(plan, S, ws, wk, method, with_scale=True))
            assert np.all(np.abs(C2 - Cw) <= 1e-9 * Aw)
            assert np.allclose(A2, Aw, rtol=1e-10, atol=0)
            assert np.all(np.abs(C2 - C) <= 1e-12 * Aw)


@pytest.mark.parametrize("nf,M,n_src,n_snk", [
    ((3, 5), 20, 150, 37),          # bucket 8, uneven
    ((2, 7, 4), 24, 120, 45),       # bucket 8, three flavours
    ((8, 6), 40, 160, 70),          # bucket 8, 4 lanes x 2 rows exactly
    ((12, 12), 40, 180, 50),        # bucket 12, 4 lanes x 3 rows exactly
    ((10, 11), 30, 140, 33),        # bucket 12, uneven
    ((16,), 30, 90, 21),            # bucket 16, 8 lanes x 2 rows exactly
    ((9, 16), 40, 80, 26),          # bucket 16, uneven
    ((17, 5), 40, 60, 20),          # bucket 18, 16 lanes x 2 rows
    ((18, 2), 30, 60, 9),           # bucket 18, the batch's largest block
    ((24,), 30, 24, 7),             # bucket 24, the largest supported block
    ((20, 13), 48, 50, 12),         # bucket 24, uneven
])
def test_rows_kernels_match_oracle(nf, M, n_src, n_snk):
    w = W.workload("mid", T=2, M=M, nf=nf, n_src=n_src, n_snk=n_snk, branching=4, depth=3)
    print(f"rows: nf={nf} M={M} {n_src}x{n_snk}", flush=True)
    plan, S, ws, wk = setup(w)
    check_all_methods(w, plan, S, ws, wk)


@pytest.mark.parametrize("nf", [(5, 7), (12, 12), (16, 10), (18, 9), (22,)])
def test_rows_kernels_m96(nf):
    # 96 quark indices: a full slice would not fit beside the pivot-row
    # buffers; the tiles stage only their units' rows
    w = W.workload("mid", T=2, M=96, nf=nf, n_src=160, n_snk=90, branching=5, depth=3)
    print(f"rows m96: nf={nf}", flush=True)
    plan, S, ws, wk = setup(w)
    check_all_methods(w, plan, S, ws, wk)


def test_rows_dominator_split_over_tiles():
    # one root with 150 children changing one of 24 rows to one of 84 new
    # indices: the dominator's rows and its children's distinct new rows
    # (more than 81 at M = 96 for blocks of 12) do not fit one workgroup's
    # LDS, so the dominator is split into units by ranges of its children
    w = W.workload("mid", T=2, M=96, nf=(12, 12), n_src=302, n_snk=40, branching=150, depth=1)
    tree = mhc.Tree(mhc.Terms(w.src, w.nf, w.M))
    g = tree.groups()
    new, _ = tree.children()
    ptr = g["grp_ptr"]
    rows_per_dom = []
    for d in range(len(g["dom_grp"]) - 1):
        kids = g["grp_child"][ptr[g["dom_grp"][d]]:ptr[g["dom_grp"][d + 1]]]
        rows_per_dom.append(24 + len(set(new[kids].tolist())))
    assert max(rows_per_dom) > 81, rows_per_dom
    plan, S, ws, wk = setup(w)
    check_all_methods(w, plan, S, ws, wk, methods=("tree", "tree_agg"))


def test_rows_singular_dominator_blocks():
    # a zero row and two equal columns of S: dominator blocks with an exact
    # zero pivot send their whole (unit, sink) items through the direct route
    w = W.workload("mid", T=2, M=20, nf=(9, 5), n_src=220, n_snk=40, branching=6, depth=3)
    w.S[:, 4, :] = 0
    w.S[:, :, 7] = w.S[:, :, 2]
    plan, S, ws, wk = setup(w)
    check_all_methods(w, plan, S, ws, wk)
    assert plan.fallback_count() > 0


def test_rows_set_edges():
    w = W.workload("mid", T=2, M=30, nf=(9, 5), n_src=200, n_snk=50)
    rng = np.random.default_rng(2)
    offs = np.concatenate([[0], np.cumsum(w.nf)])
    for terms in (w.src, w.snk):
        for u in range(len(terms)):
            for f in range(len(w.nf)):
                o, k = offs[f], w.nf[f]
                terms[u, o:o + k] = terms[u, o:o + k][rng.permutation(k)]
    plan, S, ws, wk = setup(w, set_edges=True)
    assert (plan.tree.children()[1] == -1).any()
    check_all_methods(w, plan, S, ws, wk, methods=("tree", "tree_agg"))


def test_rows_repeatable_bitwise():
    w = W.workload("large", T=2, n_src=500, n_snk=300)
    plan, S, ws, wk = setup(w)
    for method in ("plain", "tree", "tree_agg"):
        a = mhc.contract(plan, S, ws, wk, method).cpu().numpy()
        b = mhc.contract(plan, S, ws, wk, method).cpu().numpy()
        assert a.tobytes() == b.tobytes()
