"""GPU parity of the weighted-row aggregation (MHC_UPDATE_TREE_AGG): the
children of a group replace the same row of their dominator's block, and
the determinant is linear in that row, so the group contributes one dot of
the summed weighted rows with the shared solve.  Checked against the CPU
oracle on one-matrix-per-lane and group-kernel shapes, with singular
dominator blocks and with set edges (signed children)."""
import numpy as np
import pytest
import torch

from oracle import contract as oc
from paper_1411_3691_amd import mhc
from paper_1411_3691_amd import workloads as W
from paper_1411_3691_amd._lib import MhcError
from parity_util import check_pair_list

pytestmark = pytest.mark.gpu


def upload(w, **tree_kw):
    plan = mhc.Plan(mhc.Tree(mhc.Terms(w.src, w.nf, w.M), **tree_kw),
                    mhc.Terms(w.snk, w.nf, w.M))
    dev = plan.device
    return (plan, torch.from_numpy(w.S).to(dev), torch.from_numpy(w.w_src).to(dev),
            torch.from_numpy(w.w_snk).to(dev))


SHAPES = [
    dict(T=3, n_src=400, n_snk=150),                           # 6 + 6, one matrix per lane
    dict(T=2, M=20, nf=(4, 2, 3), n_src=250, n_snk=90),        # uneven blocks <= 8
    dict(T=2, M=30, nf=(9, 5), n_src=220, n_snk=70),           # group kernels (16, 12)
    dict(T=1, M=48, nf=(20, 14), n_src=120, n_snk=40, branching=5, depth=3),   # (32, 24)
]


@pytest.mark.parametrize("shape", SHAPES)
def test_aggregation_matches_oracle(shape):
    w = W.workload("mid", **shape)
    print(f"agg: {shape}", flush=True)
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    plan, S, ws, wk = upload(w)
    C = mhc.contract(plan, S, ws, wk, "tree_agg").cpu().numpy()
    assert np.all(np.abs(C - Cw) <= 1e-9 * Aw), np.max(np.abs(C - Cw) / Aw)
    Ct = mhc.contract(plan, S, ws, wk, "tree").cpu().numpy()
    assert np.all(np.abs(C - Ct) <= 1e-12 * Aw)


def test_aggregation_singular_dominator_blocks():
    # a zero row and two equal columns of S: blocks with an exact zero pivot
    # send their children through the direct route, outside the aggregate
    w = W.workload("mid", T=2, M=14, nf=(5, 3), n_src=200, n_snk=40, branching=6, depth=3)
    w.S[:, 4, :] = 0
    w.S[:, :, 7] = w.S[:, :, 2]
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    plan, S, ws, wk = upload(w)
    C = mhc.contract(plan, S, ws, wk, "tree_agg").cpu().numpy()
    assert np.all(np.abs(C - Cw) <= 1e-9 * Aw)
    assert plan.status()["n_fallback"] > 0


def test_aggregation_with_set_edges():
    # signed children: the aggregate carries each child's permutation sign
    w = W.workload("mid", T=2, n_src=300, n_snk=100)
    rng = np.random.default_rng(11)
    for terms in (w.src, w.snk):
        for u in range(len(terms)):
            for o in (0, 6):
                terms[u, o:o + 6] = terms[u, o:o + 6][rng.permutation(6)]
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    plan, S, ws, wk = upload(w, set_edges=True)
    assert (plan.tree.children()[1] == -1).any()
    C = mhc.contract(plan, S, ws, wk, "tree_agg").cpu().numpy()
    assert np.all(np.abs(C - Cw) <= 1e-9 * Aw)


def test_aggregation_sampled_pairs_and_refusals():
    w = W.workload("mid", T=2, n_src=300, n_snk=100)
    plan, S, ws, wk = upload(w)
    rng = np.random.default_rng(5)
    pq = W.random_pairs(rng, w.T, len(w.src), len(w.snk), 2000)
    C, P = mhc.contract(plan, S, ws, wk, "tree_agg", pairs=pq)
    torch.cuda.synchronize()
    check_pair_list(w, P.cpu().numpy(), pq[:, 0], pq[:, 1], pq[:, 2])
    with pytest.raises(MhcError, match="aggregation"):
        mhc.contract(plan, S, ws, wk, "tree_agg", with_scale=True)
    with pytest.raises(MhcError, match="aggregation"):
        mhc.contract(plan, S, ws, wk, "tree_agg", with_pairs=True)
