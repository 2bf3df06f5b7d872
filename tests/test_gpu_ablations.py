"""GPU ablations of the paper's variants (Sec. 4 and the Fig. 1 caption):
LU without pivoting, and updates without sibling sharing of the solves,
against the CPU oracle and against the default methods."""
import numpy as np
import pytest
import torch

from oracle import contract as oc
from paper_1411_3691_amd import mhc
from paper_1411_3691_amd import workloads as W
from paper_1411_3691_amd._lib import MhcError

pytestmark = pytest.mark.gpu


def upload(w, share=True):
    src = mhc.Terms(w.src, w.nf, w.M)
    tree = mhc.Tree(src, share=share)
    plan = mhc.Plan(tree, mhc.Terms(w.snk, w.nf, w.M))
    dev = plan.device
    return (plan, tree, torch.from_numpy(w.S).to(dev), torch.from_numpy(w.w_src).to(dev),
            torch.from_numpy(w.w_snk).to(dev))


def test_updates_without_sharing_match():
    # every child its own solve: same dominators, as many groups as children
    w = W.workload("mid", T=3, n_src=300, n_snk=200)
    plan, tree, S, ws, wk = upload(w, share=False)
    shared = mhc.Tree(mhc.Terms(w.src, w.nf, w.M))
    st, ss = tree.stats(), shared.stats()
    assert st["n_groups"] == st["n_children"] == ss["n_children"]
    assert st["n_dom"] == ss["n_dom"] and ss["n_groups"] < ss["n_children"]
    C, A = mhc.contract(plan, S, ws, wk, "tree", with_scale=True)
    C, A = C.cpu().numpy(), A.cpu().numpy()
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    assert np.all(np.abs(C - Cw) <= 1e-9 * Aw)
    plan2 = mhc.Plan(shared, mhc.Terms(w.snk, w.nf, w.M))
    C2 = mhc.contract(plan2, S, ws, wk, "tree").cpu().numpy()
    assert np.all(np.abs(C - C2) <= 1e-12 * Aw)


def test_pruned_dominating_set_matches():
    # reverse-delete dominating set (fewer dominators, more children; a
    # child may move to another dominator): the oracle's sum on a small
    # shape, and the plain LU's on every slice of the full mid workload
    w = W.workload("mid", T=3, n_src=600, n_snk=200)
    src = mhc.Terms(w.src, w.nf, w.M)
    tree = mhc.Tree(src, prune=True)
    assert tree.stats()["n_dom"] < mhc.Tree(src).stats()["n_dom"]
    plan = mhc.Plan(tree, mhc.Terms(w.snk, w.nf, w.M))
    dev = plan.device
    S, ws, wk = (torch.from_numpy(x).to(dev) for x in (w.S, w.w_src, w.w_snk))
    C = mhc.contract(plan, S, ws, wk, "tree").cpu().numpy()
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    assert np.all(np.abs(C - Cw) <= 1e-9 * Aw)
    w = W.workload("mid")
    src = mhc.Terms(w.src, w.nf, w.M)
    plan = mhc.Plan(mhc.Tree(src, prune=True), mhc.Terms(w.snk, w.nf, w.M))
    S, ws, wk = (torch.from_numpy(x).to(dev) for x in (w.S, w.w_src, w.w_snk))
    C = mhc.contract(plan, S, ws, wk, "tree").cpu().numpy()
    Cp, Ap = (x.cpu().numpy() for x in mhc.contract(plan, S, ws, wk, "plain", with_scale=True))
    assert np.all(np.abs(C - Cp) <= 2e-9 * Ap)


@pytest.mark.parametrize("method", ["plain_unpivoted", "tree_unpivoted"])
def test_unpivoted_lu_on_gaussian_blocks(method):
    # Gaussian blocks rarely have a tiny leading pivot, so without pivoting
    # the sum still agrees with the oracle; the pivoted methods are the
    # product path (this is the paper's custom-LU variant, measured only)
    w = W.workload("mid", T=3, n_src=300, n_snk=200)
    plan, tree, S, ws, wk = upload(w)
    C = mhc.contract(plan, S, ws, wk, method).cpu().numpy()
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    assert np.all(np.abs(C - Cw) <= 1e-9 * Aw), np.max(np.abs(C - Cw) / Aw)


def test_unpivoted_lu_refuses_uneven_blocks():
    w = W.workload("mid", T=2, M=24, nf=(3, 5), n_src=60, n_snk=40, branching=4, depth=3)
    plan, tree, S, ws, wk = upload(w)
    with pytest.raises(MhcError, match="MHC_E_UNSUPPORTED"):
        mhc.contract(plan, S, ws, wk, "plain_unpivoted")


def run_pairs(plan, S, ws, wk, method):
    C, A, P = mhc.contract(plan, S, ws, wk, method, with_scale=True, with_pairs=True)
    torch.cuda.synchronize()
    return C.cpu().numpy(), A.cpu().numpy(), P.cpu().numpy()


@pytest.mark.parametrize("method", ["plain_threshold", "tree_threshold"])
def test_threshold_pivoting_every_pair(method):
    # threshold partial pivoting must meet the same per-pair tolerance as
    # partial pivoting (3 slices, 300 x 200 tree terms: every pair)
    from parity_util import all_pairs, check_C, check_pairs
    w = W.workload("mid", T=3, n_src=300, n_snk=200)
    plan, tree, S, ws, wk = upload(w)
    C, A, P = run_pairs(plan, S, ws, wk, method)
    check_pairs(w, P, *all_pairs(w))
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    check_C(C, A, Cw, Aw)


@pytest.mark.parametrize("method", ["plain_threshold", "tree_threshold"])
def test_threshold_pivoting_near_singular(method):
    # two equal rows of S (blocks holding both are singular up to rounding)
    from parity_util import all_pairs, check_C, check_pairs
    w = W.workload("mid", T=2, M=12, n_src=300, n_snk=100, branching=6, depth=3)
    w.S[:, 5, :] = w.S[:, 3, :]
    plan, tree, S, ws, wk = upload(w)
    C, A, P = run_pairs(plan, S, ws, wk, method)
    check_pairs(w, P, *all_pairs(w))
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    check_C(C, A, Cw, Aw)
