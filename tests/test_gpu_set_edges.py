"""GPU parity of the set-edge ablation: terms whose flavour blocks come in
random orders, trees on set edges (a child's matrix is its dominator's
with one row replaced, up to a row permutation whose sign multiplies the
determinant), against the CPU oracle; refusals where set edges are not
supported."""
import numpy as np
import pytest
import torch

from oracle import contract as oc
from paper_1411_3691_amd import mhc
from paper_1411_3691_amd import workloads as W
from paper_1411_3691_amd._lib import MhcError
from parity_util import all_pairs, check_C, check_pair_list, check_pairs

pytestmark = pytest.mark.gpu


def permuted(w, seed=7):
    rng = np.random.default_rng(seed)
    offs = np.concatenate([[0], np.cumsum(w.nf)])
    for terms in (w.src, w.snk):
        for u in range(len(terms)):
            for f in range(len(w.nf)):
                o, k = offs[f], w.nf[f]
                terms[u, o:o + k] = terms[u, o:o + k][rng.permutation(k)]
    return w


def setup(w, set_edges):
    plan = mhc.Plan(mhc.Tree(mhc.Terms(w.src, w.nf, w.M), set_edges=set_edges),
                    mhc.Terms(w.snk, w.nf, w.M))
    dev = plan.device
    return (plan, torch.from_numpy(w.S).to(dev), torch.from_numpy(w.w_src).to(dev),
            torch.from_numpy(w.w_snk).to(dev))


@pytest.mark.parametrize("shape", [
    dict(T=3, n_src=300, n_snk=130),                          # one matrix per lane, 6 + 6
    dict(T=2, M=30, nf=(9, 5), n_src=200, n_snk=60),          # group kernels
])
def test_set_edge_tree_every_pair(shape):
    w = permuted(W.workload("mid", **shape))
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    plan, S, ws, wk = setup(w, True)
    assert (plan.tree.children()[1] == -1).any()
    C, A, P = mhc.contract(plan, S, ws, wk, "tree", with_scale=True, with_pairs=True)
    torch.cuda.synchronize()
    check_pairs(w, P.cpu().numpy(), *all_pairs(w))
    check_C(C.cpu().numpy(), A.cpu().numpy(), Cw, Aw)
    Cf = mhc.contract(plan, S, ws, wk, "tree").cpu().numpy()
    assert np.all(np.abs(Cf - Cw) <= 1e-9 * Aw)
    rng = np.random.default_rng(3)
    pq = W.random_pairs(rng, w.T, len(w.src), len(w.snk), 3000)
    _, Ps = mhc.contract(plan, S, ws, wk, "tree", pairs=pq)
    torch.cuda.synchronize()
    check_pair_list(w, Ps.cpu().numpy(), pq[:, 0], pq[:, 1], pq[:, 2])


def test_set_edge_tree_singular_dominators():
    # a zero row of S: dominator blocks with a zero pivot send their
    # children (signed) through the direct route
    w = permuted(W.workload("mid", T=2, M=14, nf=(5, 3), n_src=200, n_snk=40, branching=6,
                            depth=3))
    w.S[:, 4, :] = 0
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    plan, S, ws, wk = setup(w, True)
    C, A = mhc.contract(plan, S, ws, wk, "tree", with_scale=True)
    torch.cuda.synchronize()
    check_C(C.cpu().numpy(), A.cpu().numpy(), Cw, Aw)


def test_set_edges_refused_by_adjoint_and_two_sided():
    w = permuted(W.workload("mid", T=1, n_src=120, n_snk=80))
    plan, S, ws, wk = setup(w, True)
    g = torch.ones(1, dtype=torch.complex128)
    with pytest.raises(MhcError, match="positional edges"):
        mhc.contract_backward(plan, S, ws, wk, g, "tree")
    with pytest.raises(MhcError, match="positional edges"):
        plan.attach_sink_tree(mhc.Tree(mhc.Terms(w.snk, w.nf, w.M), set_edges=True))
