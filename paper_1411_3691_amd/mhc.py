"""Python API over the libmhc C ABI.

    terms_src = Terms(idx_src, nf, M)     # host int arrays [N][sum(nf)]
    tree = Tree(terms_src)                # greedy dominating set (Sec. 3)
    plan = Plan(tree, Terms(idx_snk, nf, M))
    C = contract(plan, S, w_src, w_snk, method="tree")   # complex128 [T]

Every step of the contraction runs in the library's HIP kernels; this
module only converts arguments (torch tensors on the plan's device, numpy
arrays for terms) into the pointers and sizes the C functions take.  There
is no CPU fallback: without the built library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

METHODS = {"plain": _lib.PLAIN_LU, "tree": _lib.UPDATE_TREE, "tree2": _lib.UPDATE_TREE2,
           # ablations: no pivoting (blocks of one size n <= 8)
           "plain_unpivoted": _lib.PLAIN_LU_UNPIVOTED,
           "tree_unpivoted": _lib.UPDATE_TREE_UNPIVOTED,
           # threshold partial pivoting (blocks of one size n <= 8)
           "plain_threshold": _lib.PLAIN_LU_THRESHOLD,
           "tree_threshold": _lib.UPDATE_TREE_THRESHOLD,
           # weighted-row aggregation: one dot per group (no per-pair values)
           "tree_agg": _lib.UPDATE_TREE_AGG}
POLICIES = {"R1": _lib.GREEDY_R1, "R2": _lib.GREEDY_R2}


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Terms:
    """Wavefunction terms: int [n_terms][sum(nf)], flavour-major."""

    def __init__(self, idx, nf, M: int):
        idx = np.ascontiguousarray(np.asarray(idx), dtype=np.int32)
        nfa = np.ascontiguousarray(np.asarray(nf), dtype=np.int32)
        if idx.ndim != 2 or idx.shape[1] != int(nfa.sum()):
            raise ValueError("idx must be [n_terms][sum(nf)]")
        self.idx = idx
        self.nf = tuple(int(v) for v in nfa)
        self.M = int(M)
        h = ctypes.c_void_p()
        check(lib().mhc_terms_create(idx.shape[0], len(nfa), _i32p(nfa),
                                     _i32p(idx), int(M), ctypes.byref(h)))
        self._h = h
        self._destroy = lib().mhc_terms_destroy

    def __len__(self):
        return self.idx.shape[0]

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None


class Tree:
    """Update tree over source terms (host only)."""

    def __init__(self, terms: Terms, policy: str = "R2", share: bool = True,
                 prune: bool = False, set_edges: bool = False):
        """share=False: every child its own group (no shared solves; an
        ablation).  prune=True: reverse-delete pass over the greedy
        dominators (an irredundant set, never larger; Sec. 3).
        set_edges=True: terms are adjacent when their index sets differ in
        one element per the whole term (Sec. 3 reads terms as sets of
        rows); a child's blocks are its dominator's with one row replaced,
        up to a row permutation whose sign multiplies the determinant
        (forward contraction only)."""
        self.terms = terms
        self.policy = policy
        self.share = share
        self.prune = prune
        self.set_edges = set_edges
        flags = ((0 if share else _lib.TREE_NO_SHARING) | (_lib.TREE_PRUNE if prune else 0) |
                 (_lib.TREE_SET_EDGES if set_edges else 0))
        h = ctypes.c_void_p()
        check(lib().mhc_tree_build(terms.handle, POLICIES[policy] | flags, ctypes.byref(h)))
        self._h = h
        self._destroy = lib().mhc_tree_destroy

    @property
    def handle(self):
        return self._h

    def export(self) -> dict:
        n = len(self.terms)
        n_dom = ctypes.c_int32()
        arrs = {k: np.empty(n, dtype=np.int32) for k in ("dom_order", "owner", "flav", "pos")}
        check(lib().mhc_tree_export(self._h, ctypes.byref(n_dom), _i32p(arrs["dom_order"]),
                                    _i32p(arrs["owner"]), _i32p(arrs["flav"]),
                                    _i32p(arrs["pos"])))
        arrs["n_dom"] = int(n_dom.value)
        return arrs

    def groups(self) -> dict:
        """The group tables the kernels read (mhc_tree_groups): dom_grp,
        grp_f, grp_r, grp_ptr, grp_child."""
        st = self.stats()
        nd, ng, nc = st["n_dom"], st["n_groups"], st["n_children"]
        out = dict(dom_grp=np.empty(nd + 1, dtype=np.int32),
                   grp_f=np.empty(ng, dtype=np.int32), grp_r=np.empty(ng, dtype=np.int32),
                   grp_ptr=np.empty(ng + 1, dtype=np.int32),
                   grp_child=np.empty(nc, dtype=np.int32))
        check(lib().mhc_tree_groups(self._h, *(_i32p(out[k]) for k in
                                               ("dom_grp", "grp_f", "grp_r", "grp_ptr",
                                                "grp_child"))))
        return out

    def children(self):
        """(new_index, sign) per term (mhc_tree_children): the index the
        child's changed row takes and the sign of the row permutation to its
        dominator's blocks; -1 and 0 for dominators."""
        n = len(self.terms)
        new = np.empty(n, dtype=np.int32)
        sign = np.empty(n, dtype=np.int32)
        check(lib().mhc_tree_children(self._h, _i32p(new), _i32p(sign)))
        return new, sign

    def stats(self) -> dict:
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().mhc_tree_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(n_dom=a.value, n_groups=b.value, n_children=c.value,
                    n_terms=len(self.terms))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """Source tree + sink terms uploaded to the current GPU."""

    def __init__(self, tree: Tree, snk: Terms):
        if not torch.cuda.is_available():
            raise RuntimeError("mhc.Plan needs a GPU (HIP device)")
        self.tree = tree
        self.snk = snk
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        check(lib().mhc_plan_create(tree.handle, snk.handle, _stream_ptr(),
                                    ctypes.byref(h)))
        self._h = h
        self._destroy = lib().mhc_plan_destroy

    @property
    def n_src(self):
        return len(self.tree.terms)

    @property
    def n_snk(self):
        return len(self.snk)

    @property
    def M(self):
        return self.snk.M

    def attach_sink_tree(self, tree: Tree) -> None:
        """Enables method "tree2" (source and sink update trees); ``tree``
        must be built on this plan's sink terms."""
        check(lib().mhc_plan_attach_sink_tree(self._h, tree.handle, _stream_ptr()))
        self.snk_tree = tree

    def status(self) -> dict:
        """Counters over completed calls (synchronises the device)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        check(lib().mhc_plan_status(self._h, ctypes.byref(a), ctypes.byref(b)))
        return dict(n_fallback=int(a.value), n_singular_grad=int(b.value))

    def fallback_count(self) -> int:
        return self.status()["n_fallback"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None


def _check_dev(x: torch.Tensor, dtype, shape, name, device):
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {x.dtype}")
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(x.shape)}")
    if x.device != device:
        raise ValueError(f"{name} must be on {device}, got {x.device}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def contract_into(plan: Plan, S: torch.Tensor, w_src: torch.Tensor, w_snk: torch.Tensor,
                  C: torch.Tensor, method: str = "tree", A: torch.Tensor | None = None,
                  pair_det: torch.Tensor | None = None,
                  pairs: torch.Tensor | None = None) -> None:
    """Enqueue the contraction on torch's current stream, writing C (and A,
    pair_det if given).  All tensors live on the plan's device.  pair_det is
    either every pair determinant [T][n_src][n_snk] (pairs None) or, with
    pairs an int32 [n][3] tensor of (t, i, j), the sampled ones [n]."""
    T = S.shape[0]
    dev = plan.device
    _check_dev(S, torch.complex128, (T, plan.M, plan.M), "S", dev)
    _check_dev(w_src, torch.float64, (plan.n_src,), "w_src", dev)
    _check_dev(w_snk, torch.float64, (plan.n_snk,), "w_snk", dev)
    _check_dev(C, torch.complex128, (T,), "C", dev)
    if A is not None:
        _check_dev(A, torch.float64, (T,), "A", dev)
    n_pairs = 0
    if pairs is not None:
        if pair_det is None:
            raise ValueError("pairs needs pair_det")
        n_pairs = pairs.shape[0]
        _check_dev(pairs, torch.int32, (n_pairs, 3), "pairs", dev)
        _check_dev(pair_det, torch.complex128, (n_pairs,), "pair_det", dev)
    elif pair_det is not None:
        _check_dev(pair_det, torch.complex128, (T, plan.n_src, plan.n_snk), "pair_det", dev)
    check(lib().mhc_contract(
        plan._h, METHODS[method], T, ctypes.c_void_p(S.data_ptr()),
        ctypes.c_void_p(w_src.data_ptr()), ctypes.c_void_p(w_snk.data_ptr()),
        ctypes.c_void_p(C.data_ptr()),
        ctypes.c_void_p(A.data_ptr() if A is not None else 0),
        ctypes.c_void_p(pair_det.data_ptr() if pair_det is not None else 0),
        ctypes.c_void_p(pairs.data_ptr() if pairs is not None else 0), n_pairs,
        _stream_ptr()))


PROBE_BLOCK = 256
PROBE_FLOP_PER_ROUND = 32


def probe_fma64(out: torch.Tensor, iters: int) -> int:
    """Enqueue the FP64 FMA probe (mhc_probe_fma64) on torch's current
    stream: out (float64, a multiple of 256 entries, on a GPU) gets one
    value per thread.  Returns the flop count of the launch."""
    if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 GPU tensor")
    if out.numel() == 0 or out.numel() % PROBE_BLOCK:
        raise ValueError(f"out must hold a positive multiple of {PROBE_BLOCK} values")
    n_blocks = out.numel() // PROBE_BLOCK
    check(lib().mhc_probe_fma64(ctypes.c_void_p(out.data_ptr()), n_blocks, iters,
                                _stream_ptr()))
    return out.numel() * iters * PROBE_FLOP_PER_ROUND


def probe_mfma64(out: torch.Tensor, iters: int, with_valu: bool = False) -> int:
    """Enqueue the FP64 matrix-core probe (mhc_probe_mfma64) on torch's
    current stream; out as for probe_fma64.  Returns the flop count of the
    launch (matrix and, with with_valu, vector)."""
    if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 GPU tensor")
    if out.numel() == 0 or out.numel() % PROBE_BLOCK:
        raise ValueError(f"out must hold a positive multiple of {PROBE_BLOCK} values")
    n_blocks = out.numel() // PROBE_BLOCK
    check(lib().mhc_probe_mfma64(ctypes.c_void_p(out.data_ptr()), n_blocks, iters,
                                 1 if with_valu else 0, _stream_ptr()))
    flop = n_blocks * (PROBE_BLOCK // 64) * iters * 4 * 2048
    if with_valu:
        flop += out.numel() * iters * PROBE_FLOP_PER_ROUND
    return flop


def contract(plan: Plan, S: torch.Tensor, w_src: torch.Tensor, w_snk: torch.Tensor,
             method: str = "tree", with_scale: bool = False, with_pairs: bool = False,
             pairs=None):
    """C(t) for every slice (complex128 [T] on the plan's device).  With
    with_scale / with_pairs also returns A(t) and the pair determinants:
    every one ([T][n_src][n_snk]), or with ``pairs`` (int [n][3] of
    (t, i, j), any array-like) the sampled ones ([n])."""
    T = S.shape[0]
    C = torch.empty(T, dtype=torch.complex128, device=plan.device)
    A = torch.empty(T, dtype=torch.float64, device=plan.device) if with_scale else None
    pt = None
    if pairs is not None:
        with_pairs = True
        pt = torch.as_tensor(np.ascontiguousarray(np.asarray(pairs, dtype=np.int32)))
        pt = pt.reshape(-1, 3).to(plan.device).contiguous()
        P = torch.empty(pt.shape[0], dtype=torch.complex128, device=plan.device)
    else:
        P = (torch.empty((T, plan.n_src, plan.n_snk), dtype=torch.complex128,
                         device=plan.device) if with_pairs else None)
    contract_into(plan, S, w_src, w_snk, C, method, A, P, pt)
    if not (with_scale or with_pairs):
        return C
    out = [C]
    if with_scale:
        out.append(A)
    if with_pairs:
        out.append(P)
    return tuple(out)


BACKWARD = {"plain": _lib.PLAIN_LU, "tree": _lib.UPDATE_TREE}


def contract_backward(plan: Plan, S: torch.Tensor, w_src: torch.Tensor, w_snk: torch.Tensor,
                      gC: torch.Tensor, method: str = "tree"):
    """(grad_S, grad_w_src, grad_w_snk) of a real loss whose gradient with
    respect to C is gC (PyTorch's complex convention), from the library's
    adjoint kernels (method "tree": by the source update tree; "plain":
    pair by pair)."""
    T = S.shape[0]
    dev = plan.device
    _check_dev(S, torch.complex128, (T, plan.M, plan.M), "S", dev)
    _check_dev(w_src, torch.float64, (plan.n_src,), "w_src", dev)
    _check_dev(w_snk, torch.float64, (plan.n_snk,), "w_snk", dev)
    gC = gC.to(device=dev, dtype=torch.complex128).contiguous()
    _check_dev(gC, torch.complex128, (T,), "gC", dev)
    gS = torch.empty_like(S)
    g_src = torch.empty_like(w_src)
    g_snk = torch.empty_like(w_snk)
    check(lib().mhc_contract_backward(
        plan._h, BACKWARD[method], T, ctypes.c_void_p(S.data_ptr()),
        ctypes.c_void_p(w_src.data_ptr()),
        ctypes.c_void_p(w_snk.data_ptr()), ctypes.c_void_p(gC.data_ptr()),
        ctypes.c_void_p(gS.data_ptr()), ctypes.c_void_p(g_src.data_ptr()),
        ctypes.c_void_p(g_snk.data_ptr()), _stream_ptr()))
    return gS, g_src, g_snk


KERNELS = {"auto": _lib.SCHED_AUTO, "lane": _lib.SCHED_LANE, "group": _lib.SCHED_GROUP}


class Batch:
    """Many independent contractions in one captured graph.

        batch = Batch(plans, T=[...], method="tree")
        batch.run(S_list, w_src_list, w_snk_list, C_list)   # torch's stream

    ``schedule`` = dict(kernel="auto"|"lane"|"group", blocks_per_cu=0,
    items_per_tile=0) (0 = the library's choice).  Plans must stay alive as
    long as the batch; the batch keeps references to them.
    """

    def __init__(self, plans, T, method: str = "tree", schedule: dict | None = None):
        plans = list(plans)
        T = np.ascontiguousarray(np.asarray(T), dtype=np.int32)
        if len(plans) == 0 or T.shape != (len(plans),):
            raise ValueError("need one slice count per plan")
        self.plans = plans
        self.T = [int(v) for v in T]
        self.method = method
        sc = dict(kernel="auto", blocks_per_cu=0, items_per_tile=0)
        sc.update(schedule or {})
        self.schedule = sc
        cs = _lib.Schedule(KERNELS[sc["kernel"]], int(sc["blocks_per_cu"]),
                           int(sc["items_per_tile"]))
        arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
        h = ctypes.c_void_p()
        check(lib().mhc_batch_create(arr, _i32p(T), len(plans), METHODS[method],
                                     ctypes.byref(cs), ctypes.byref(h)))
        self._h = h
        self._destroy = lib().mhc_batch_destroy
        self.device = plans[0].device

    def __len__(self):
        return len(self.plans)

    def info(self) -> dict:
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        check(lib().mhc_batch_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(n_tiles=a.value, n_kernels=b.value, n_pairs=int(c.value))

    def run(self, S, w_src, w_snk, C, A=None) -> None:
        """Enqueue every job on torch's current stream: C[j] (and A[j]) of
        job j from S[j], w_src[j], w_snk[j]."""
        n = len(self.plans)
        if not (len(S) == len(w_src) == len(w_snk) == len(C) == n) or \
                (A is not None and len(A) != n):
            raise ValueError(f"need {n} tensors per argument")
        for j, pl in enumerate(self.plans):
            T, dev = self.T[j], self.device
            _check_dev(S[j], torch.complex128, (T, pl.M, pl.M), f"S[{j}]", dev)
            _check_dev(w_src[j], torch.float64, (pl.n_src,), f"w_src[{j}]", dev)
            _check_dev(w_snk[j], torch.float64, (pl.n_snk,), f"w_snk[{j}]", dev)
            _check_dev(C[j], torch.complex128, (T,), f"C[{j}]", dev)
            if A is not None:
                _check_dev(A[j], torch.float64, (T,), f"A[{j}]", dev)

        def ptrs(xs):
            return (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])

        check(lib().mhc_batch_run(self._h, ptrs(S), ptrs(w_src), ptrs(w_snk), ptrs(C),
                                  ptrs(A) if A is not None else None, _stream_ptr()))

    def __call__(self, S, w_src, w_snk, with_scale: bool = False):
        C = [torch.empty(T, dtype=torch.complex128, device=self.device) for T in self.T]
        A = ([torch.empty(T, dtype=torch.float64, device=self.device) for T in self.T]
             if with_scale else None)
        self.run(S, w_src, w_snk, C, A)
        return (C, A) if with_scale else C

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None


class Contract(torch.autograd.Function):
    """C = Contract.apply(plan, S, w_src, w_snk, method): differentiable in S
    and both weight arrays; the backward pass is the library's adjoint."""

    @staticmethod
    def forward(ctx, plan, S, w_src, w_snk, method="tree"):
        ctx.plan = plan
        ctx.method = method
        ctx.save_for_backward(S, w_src, w_snk)
        return contract(plan, S.contiguous(), w_src.contiguous(), w_snk.contiguous(), method)

    @staticmethod
    def backward(ctx, gC):
        S, w_src, w_snk = ctx.saved_tensors
        gS, g_src, g_snk = contract_backward(ctx.plan, S.contiguous(), w_src.contiguous(),
                                             w_snk.contiguous(), gC,
                                             "plain" if ctx.method == "plain" else "tree")
        return (None, gS if ctx.needs_input_grad[1] else None,
                g_src if ctx.needs_input_grad[2] else None,
                g_snk if ctx.needs_input_grad[3] else None, None)
