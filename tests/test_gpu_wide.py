"""GPU parity of the group-per-matrix kernels: flavour blocks larger than 8
(up to 24) and flavour blocks of different sizes, against the CPU oracle."""
import numpy as np
import pytest
import torch

from oracle import contract as oc
from paper_1411_3691_amd import mhc
from paper_1411_3691_amd import workloads as W
from parity_util import all_pairs, check_C, check_pairs

pytestmark = pytest.mark.gpu


def setup(w, policy="R2", prune=False):
    plan = mhc.Plan(mhc.Tree(mhc.Terms(w.src, w.nf, w.M), policy, prune=prune),
                    mhc.Terms(w.snk, w.nf, w.M))
    dev = plan.device
    return (plan, torch.from_numpy(w.S).to(dev), torch.from_numpy(w.w_src).to(dev),
            torch.from_numpy(w.w_snk).to(dev))


def run(plan, S, ws, wk, method, pairs=True):
    out = mhc.contract(plan, S, ws, wk, method, with_scale=True, with_pairs=pairs)
    torch.cuda.synchronize()
    out = tuple(x.cpu().numpy() for x in out)
    return out if pairs else out + (None,)


@pytest.mark.parametrize("nf,M,n_src,n_snk", [
    ((3, 5), 20, 120, 37),          # uneven blocks below 8
    ((2, 7, 4), 24, 100, 40),       # three flavours, uneven
    ((12, 12), 40, 150, 19),        # the large workload's block size
    ((16,), 30, 80, 21),            # largest block of a 16-lane group
    ((9, 17), 40, 60, 15),          # 32-lane group, uneven
    ((18, 2), 30, 60, 9),           # largest block of the batched workload
    ((24,), 30, 20, 5),             # largest supported block
])
def test_wide_blocks_all_pairs(nf, M, n_src, n_snk):
    w = W.workload("mid", T=2, M=M, nf=nf, n_src=n_src, n_snk=n_snk, branching=4, depth=3)
    plan, S, ws, wk = setup(w)
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    for method in ("plain", "tree"):
        C, A, P = run(plan, S, ws, wk, method)
        check_pairs(w, P, *all_pairs(w))
        check_C(C, A, Cw, Aw)


@pytest.mark.parametrize("nf,M,n_src,n_snk", [
    ((3, 5), 20, 120, 37),
    ((12, 12), 40, 150, 19),
    ((9, 17), 40, 60, 15),
])
def test_wide_blocks_pruned_dominating_set(nf, M, n_src, n_snk):
    # reverse-delete dominators (fewer LUs, children moved to other
    # dominators) through the group kernels: every pair det and C
    w = W.workload("mid", T=2, M=M, nf=nf, n_src=n_src, n_snk=n_snk, branching=4, depth=3)
    plan, S, ws, wk = setup(w, prune=True)
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    C, A, P = run(plan, S, ws, wk, "tree")
    check_pairs(w, P, *all_pairs(w))
    check_C(C, A, Cw, Aw)


@pytest.mark.parametrize("nf,n_src,n_snk", [
    ((3, 5), 60, 23),       # uneven blocks below 8
    ((12, 12), 60, 17),
    ((16,), 50, 13),
    ((9, 17), 40, 9),
    ((18, 2), 40, 9),
    ((24,), 16, 5),
])
def test_wide_blocks_with_m96_slices(nf, n_src, n_snk):
    # a 96-index slice (147 KB of LDS, one workgroup per compute unit)
    # selects the 1024-thread kernels, whose pivot rows go through LDS row
    # buffers, and for the tree's blocks above 12 the 768-thread kernels;
    # every pair against the oracle
    w = W.workload("mid", T=2, M=96, nf=nf, n_src=n_src, n_snk=n_snk, branching=4, depth=3)
    plan, S, ws, wk = setup(w)
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    for method in ("plain", "tree"):
        C, A, P = run(plan, S, ws, wk, method)
        check_pairs(w, P, *all_pairs(w))
        check_C(C, A, Cw, Aw)
        Cf = mhc.contract(plan, S, ws, wk, method).cpu().numpy()
        assert np.all(np.abs(Cf - C) <= 1e-12 * Aw)


def test_large_shape_subset():
    # 96 quark indices (a 147 KB slice in LDS), blocks of 12, tree terms with
    # branching 16 and depth <= 5; 3 slices, 400 x 130 terms
    w = W.workload("large", T=3, n_src=400, n_snk=130)
    plan, S, ws, wk = setup(w)
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    for method in ("plain", "tree"):
        C, A, P = run(plan, S, ws, wk, method)
        rng = np.random.default_rng(4)
        idx = W.random_pairs(rng, w.T, len(w.src), len(w.snk), 6000)
        check_pairs(w, P, idx[:, 0], idx[:, 1], idx[:, 2])
        check_C(C, A, Cw, Aw)
        Cf = mhc.contract(plan, S, ws, wk, method).cpu().numpy()
        assert np.all(np.abs(Cf - C) <= 1e-12 * Aw)


def test_wide_singular_dominators_take_the_direct_route():
    w = W.workload("mid", T=2, M=14, nf=(5, 3), n_src=200, n_snk=40, branching=6, depth=3)
    w.S[:, 4, :] = 0
    plan, S, ws, wk = setup(w)
    Cw, Aw = oc.correlator(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk)
    for method in ("plain", "tree"):
        C, A, P = run(plan, S, ws, wk, method)
        check_pairs(w, P, *all_pairs(w))
        check_C(C, A, Cw, Aw)
    assert plan.fallback_count() > 0


def test_wide_repeatable_bitwise():
    w = W.workload("mid", T=2, M=30, nf=(9, 5), n_src=100, n_snk=50)
    plan, S, ws, wk = setup(w)
    for method in ("plain", "tree"):
        a = mhc.contract(plan, S, ws, wk, method).cpu().numpy()
        b = mhc.contract(plan, S, ws, wk, method).cpu().numpy()
        assert a.tobytes() == b.tobytes()
