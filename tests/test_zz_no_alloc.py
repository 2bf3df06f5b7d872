"""The allocation-free contraction entry point (mhc_contract_noalloc), called
through the C ABI, against mhc_contract on the same inputs: two calls in a
row on one device, the second with fewer slices and another plan, so the
shared static scratch must not carry anything from the first call."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1411_3691_amd import _lib, mhc
from paper_1411_3691_amd import workloads as W

pytestmark = pytest.mark.gpu


def noalloc(plan, method, S, ws, wk, with_scale=True):
    T = S.shape[0]
    C = torch.empty(T, dtype=torch.complex128, device=plan.device)
    A = torch.empty(T, dtype=torch.float64, device=plan.device) if with_scale else None
    st = _lib.lib().mhc_contract_noalloc(
        plan._h, mhc.METHODS[method], T, ctypes.c_void_p(S.data_ptr()),
        ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(wk.data_ptr()),
        ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(A.data_ptr() if A is not None else 0),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(st)
    return C, A


def setup(w):
    plan = mhc.Plan(mhc.Tree(mhc.Terms(w.src, w.nf, w.M)), mhc.Terms(w.snk, w.nf, w.M))
    dev = plan.device
    return (plan, torch.from_numpy(w.S).to(dev), torch.from_numpy(w.w_src).to(dev),
            torch.from_numpy(w.w_snk).to(dev))


@pytest.mark.parametrize("method", ["tree", "plain"])
def test_noalloc_matches_contract_twice(method):
    big = W.workload("mid", T=6, n_src=600, n_snk=300)
    small = W.workload("mid", T=2, M=30, nf=(9, 5), n_src=120, n_snk=50)
    for w in (big, small):
        print(f"noalloc/{method}: T={w.T} M={w.M} blocks {w.nf} {len(w.src)}x{len(w.snk)}",
              flush=True)
        plan, S, ws, wk = setup(w)
        C1, A1 = noalloc(plan, method, S, ws, wk)
        C0, A0 = mhc.contract(plan, S, ws, wk, method, with_scale=True)
        torch.cuda.synchronize()
        C0, A0, C1, A1 = (x.cpu().numpy() for x in (C0, A0, C1, A1))
        # the same kernels on the same inputs: the same fixed-order sums
        assert C1.tobytes() == C0.tobytes()
        assert A1.tobytes() == A0.tobytes()
        assert np.all(np.abs(C1 - C0) <= 1e-9 * A0)


def test_noalloc_two_sided_twice():
    # the two-sided method also leaves a flag per workgroup in the static
    # scratch; the second call has singular blocks (a zero row of S), so
    # its flagged workgroups' pairs are added by the direct-LU pass
    big = W.workload("mid", T=6, n_src=600, n_snk=300)
    small = W.workload("mid", T=2, M=24, nf=(4, 4), n_src=120, n_snk=60, branching=4, depth=3)
    small.S[:, 3, :] = 0
    for w in (big, small):
        print(f"noalloc/tree2: T={w.T} M={w.M} blocks {w.nf} {len(w.src)}x{len(w.snk)}",
              flush=True)
        plan, S, ws, wk = setup(w)
        plan.attach_sink_tree(mhc.Tree(mhc.Terms(w.snk, w.nf, w.M)))
        C1, _ = noalloc(plan, "tree2", S, ws, wk, with_scale=False)
        C0 = mhc.contract(plan, S, ws, wk, "tree2")
        _, A0 = mhc.contract(plan, S, ws, wk, "tree", with_scale=True)
        torch.cuda.synchronize()
        C0, C1, A0 = (x.cpu().numpy() for x in (C0, C1, A0))
        assert C1.tobytes() == C0.tobytes()
        assert np.all(np.abs(C1 - C0) <= 1e-9 * A0)
    assert plan.fallback_count() > 0


def test_noalloc_rejects_bad_arguments():
    w = W.workload("mid", T=1, n_src=40, n_snk=30)
    plan, S, ws, wk = setup(w)
    L = _lib.lib()
    C = torch.empty(1, dtype=torch.complex128, device=plan.device)
    E_ARG = -1
    assert L.mhc_contract_noalloc(None, 1, 1, ctypes.c_void_p(S.data_ptr()),
                                  ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(wk.data_ptr()),
                                  ctypes.c_void_p(C.data_ptr()), None, None) == E_ARG
    assert L.mhc_contract_noalloc(plan._h, 1, 0, ctypes.c_void_p(S.data_ptr()),
                                  ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(wk.data_ptr()),
                                  ctypes.c_void_p(C.data_ptr()), None, None) == E_ARG
