"""GPU adjoint: the library's backward kernels against PyTorch's gradcheck,
the CPU gradient oracle and complex central finite differences."""
import numpy as np
import pytest
import torch

from oracle import grad as og
from paper_1411_3691_amd import mhc
from paper_1411_3691_amd import workloads as W

pytestmark = pytest.mark.gpu


def setup(w, prune=False):
    src = mhc.Terms(w.src, w.nf, w.M)
    snk = mhc.Terms(w.snk, w.nf, w.M)
    plan = mhc.Plan(mhc.Tree(src, prune=prune), snk)
    dev = plan.device
    return (plan, torch.from_numpy(w.S).to(dev), torch.from_numpy(w.w_src).to(dev),
            torch.from_numpy(w.w_snk).to(dev))


def test_gradcheck_tiny():
    # 1 slice, 7 quark indices, two flavours of 2, 5 x 4 terms
    w = W.workload("mid", T=1, M=7, nf=(2, 2), n_src=5, n_snk=4, branching=2, depth=2)
    plan, S, ws, wk = setup(w)
    S.requires_grad_(True)
    ws.requires_grad_(True)
    wk.requires_grad_(True)
    # grad S is summed with LDS atomics across waves: repeatable up to
    # rounding, hence a small nondeterminism tolerance
    for method in ("plain", "tree"):
        assert torch.autograd.gradcheck(
            lambda s, a, b: mhc.Contract.apply(plan, s, a, b, method), (S, ws, wk),
            eps=1e-6, atol=1e-7, rtol=1e-5, nondet_tol=1e-12)


@pytest.mark.parametrize("method", ["plain", "tree"])
def test_full_gradient_against_oracle_small(method):
    # every entry of grad S and both weight gradients, 2 slices, blocks of 3,
    # 20 x 70 terms (one full sink block of 64 and a ragged one)
    w = W.workload("mid", T=2, M=10, nf=(3, 3), n_src=20, n_snk=70, branching=3, depth=2)
    plan, S, ws, wk = setup(w)
    rng = np.random.default_rng(8)
    g = rng.standard_normal(w.T) + 1j * rng.standard_normal(w.T)
    gS, gws, gwk = mhc.contract_backward(plan, S, ws, wk, torch.from_numpy(g), method)
    torch.cuda.synchronize()
    gS, gws, gwk = gS.cpu().numpy(), gws.cpu().numpy(), gwk.cpu().numpy()
    oS, ows, owk = og.vjp(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk, g)
    scale = np.abs(oS).max()
    np.testing.assert_allclose(gS, oS, atol=1e-11 * scale, rtol=1e-9)
    np.testing.assert_allclose(gws, ows, atol=1e-11 * np.abs(ows).max(), rtol=1e-9)
    np.testing.assert_allclose(gwk, owk, atol=1e-11 * np.abs(owk).max(), rtol=1e-9)
    assert plan.status()["n_singular_grad"] == 0


@pytest.mark.parametrize("method", ["plain", "tree"])
def test_grad_workload_sampled_entries(method):
    # 32 slices, M = 48, blocks of 6, 2000 x 2000 tree terms: 16 random
    # entries of grad S and 16 random weights per side against the oracle
    # (within 1e-9 of the sum of the magnitudes of each entry's terms) and
    # against complex central differences of the GPU forward (h = 1e-6)
    w = W.workload("grad")
    plan, S, ws, wk = setup(w)
    rng = np.random.default_rng(9)
    g = rng.standard_normal(w.T) + 1j * rng.standard_normal(w.T)
    gS, gws, gwk = mhc.contract_backward(plan, S, ws, wk, torch.from_numpy(g), method)
    torch.cuda.synchronize()
    gS, gws, gwk = gS.cpu().numpy(), gws.cpu().numpy(), gwk.cpu().numpy()

    entries = [(int(rng.integers(w.T)), int(rng.integers(w.M)), int(rng.integers(w.M)))
               for _ in range(16)]
    for (t, p, q) in entries:
        d, sc = og.dC_dS_entry(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk, t, p, q,
                               with_scale=True)
        want = g[t] * np.conj(d)
        assert abs(gS[t, p, q] - want) <= 1e-9 * abs(g[t]) * sc + 1e-300, (t, p, q)
    isrc = rng.choice(len(w.src), 16, replace=False)
    isnk = rng.choice(len(w.snk), 16, replace=False)
    ds, dk = og.dC_dw_entries(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk, isrc, isnk)
    want_s = np.real(g[:, None] * np.conj(ds)).sum(axis=0)
    want_k = np.real(g[:, None] * np.conj(dk)).sum(axis=0)
    np.testing.assert_allclose(gws[isrc], want_s, rtol=1e-9, atol=1e-12 * np.abs(want_s).max())
    np.testing.assert_allclose(gwk[isnk], want_k, rtol=1e-9, atol=1e-12 * np.abs(want_k).max())

    # finite differences through the GPU forward: for an entry of slice t the
    # loss is that slice's term Re(conj(g_t) C_t) (the other slices do not
    # depend on S_t) and the step is 1e-6 of the slice's scale e^{-0.5 t};
    # for a weight the loss is L = Re(sum_t conj(g_t) C_t)
    gt = torch.from_numpy(g).to(plan.device)

    def L(S_, ws_, wk_, t=None):
        C = mhc.contract(plan, S_, ws_, wk_, "tree")
        z = torch.conj(gt) * C
        return float(torch.real(z[t] if t is not None else torch.sum(z)).item())

    # Tolerance: 1e-6 relative, plus the floor that rounding in the forward
    # sums puts on any central difference: each L carries an error of at
    # most eps_f * |g_t| A(t) (A the sum of |w w' d| over the slice's pairs,
    # eps_f = 1e-14, far above the measured ~1e-16 of the fixed-order
    # reductions), divided by the step 2h.  Where C(t) is a sum of 4e6
    # terms of random sign, that floor is above 1e-6 of the small entries.
    _, A_gpu = mhc.contract(plan, S, ws, wk, "tree", with_scale=True)
    A_gpu = A_gpu.cpu().numpy()
    eps_f = 1e-14
    worst = 0.0
    for (t, p, q) in entries:
        h = 1e-6 * float(np.abs(w.S[t]).max())
        E = torch.zeros_like(S)
        E[t, p, q] = h
        fx = (L(S + E, ws, wk, t) - L(S - E, ws, wk, t)) / (2 * h)
        fy = (L(S + 1j * E, ws, wk, t) - L(S - 1j * E, ws, wk, t)) / (2 * h)
        floor = 2 * eps_f * abs(g[t]) * A_gpu[t] / (2 * h)
        err = abs(complex(fx, fy) - gS[t, p, q])
        assert err <= 1e-6 * abs(gS[t, p, q]) + floor, (t, p, q, err, floor)
        worst = max(worst, err / abs(gS[t, p, q]))
    print(f"grad S vs central differences: worst relative difference {worst:.2e}")
    # weights: L is linear in each weight (Sec. 1), so a central difference
    # has no truncation error at any step; h = 1e-6 with the rounding floor,
    # and h = 1 where the floor is negligible
    A_all = float(np.sum(np.abs(g) * A_gpu))
    for h in (1e-6, 1.0):
        floor = 2 * eps_f * A_all / (2 * h)
        for i in isrc:
            e = torch.zeros_like(ws)
            e[i] = h
            fd = (L(S, ws + e, wk) - L(S, ws - e, wk)) / (2 * h)
            assert abs(fd - gws[i]) <= 1e-6 * abs(gws[i]) + floor, (h, i, fd, gws[i], floor)
        for j in isnk:
            e = torch.zeros_like(wk)
            e[j] = h
            fd = (L(S, ws, wk + e) - L(S, ws, wk - e)) / (2 * h)
            assert abs(fd - gwk[j]) <= 1e-6 * abs(gwk[j]) + floor, (h, j, fd, gwk[j], floor)


@pytest.mark.parametrize("method", ["plain", "tree"])
def test_backward_repeatable_in_weights(method):
    w = W.workload("mid", T=2, n_src=200, n_snk=130)
    plan, S, ws, wk = setup(w)
    g = torch.tensor([1.0 - 0.5j, 0.25 + 2j], dtype=torch.complex128)
    a = mhc.contract_backward(plan, S, ws, wk, g, method)
    b = mhc.contract_backward(plan, S, ws, wk, g, method)
    torch.cuda.synchronize()
    assert a[1].cpu().numpy().tobytes() == b[1].cpu().numpy().tobytes()
    assert a[2].cpu().numpy().tobytes() == b[2].cpu().numpy().tobytes()
    np.testing.assert_allclose(a[0].cpu().numpy(), b[0].cpu().numpy(), rtol=1e-12,
                               atol=1e-14 * float(a[0].abs().max()))


@pytest.mark.parametrize("prune", [False, True])
def test_tree_backward_matches_plain_backward(prune):
    # 3 slices, mid blocks, 400 x 150 tree terms (several sink blocks); also
    # on the reverse-delete dominating set (children moved between dominators)
    w = W.workload("mid", T=3, n_src=400, n_snk=150)
    plan, S, ws, wk = setup(w, prune)
    g = torch.tensor([0.5 + 1j, -1.0 + 0.25j, 2.0 - 1j], dtype=torch.complex128)
    p = [x.cpu().numpy() for x in mhc.contract_backward(plan, S, ws, wk, g, "plain")]
    t = [x.cpu().numpy() for x in mhc.contract_backward(plan, S, ws, wk, g, "tree")]
    for a, b in zip(p, t):
        np.testing.assert_allclose(b, a, rtol=1e-9, atol=1e-11 * np.abs(a).max())


def test_tree_backward_with_singular_dominators():
    # a zero row of S makes every block that uses source index 2 singular:
    # those dominators' partitions go pair by pair, the rest by the tree
    w = W.workload("mid", T=2, M=12, nf=(3, 3), n_src=60, n_snk=70, branching=4, depth=2)
    w.S[:, 2, :] = 0
    plan, S, ws, wk = setup(w)
    rng = np.random.default_rng(3)
    g = rng.standard_normal(w.T) + 1j * rng.standard_normal(w.T)
    gS, gws, gwk = mhc.contract_backward(plan, S, ws, wk, torch.from_numpy(g), "tree")
    torch.cuda.synchronize()
    gS, gws, gwk = gS.cpu().numpy(), gws.cpu().numpy(), gwk.cpu().numpy()
    oS, ows, owk = og.vjp(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk, g)
    # row 2 of grad S needs the adjugate of the singular blocks: taken from
    # their minors (the blocks are counted); every entry must match
    scale = np.abs(oS).max()
    assert np.abs(oS[:, 2, :]).max() > 1e-3 * scale    # the cofactors are there
    np.testing.assert_allclose(gS, oS, atol=1e-11 * scale, rtol=1e-9)
    np.testing.assert_allclose(gws, ows, atol=1e-11 * np.abs(ows).max(), rtol=1e-9)
    np.testing.assert_allclose(gwk, owk, atol=1e-11 * np.abs(owk).max(), rtol=1e-9)
    assert plan.status()["n_singular_grad"] > 0


@pytest.mark.parametrize("nf,M", [((1, 1), 12), ((4, 4), 12), ((5, 5), 14), ((7,), 12),
                                  ((8, 8), 20), ((3, 3, 3), 14), ((2, 2, 2, 2), 12)])
def test_tree_backward_block_sizes(nf, M):
    # block sizes of the update-tree adjoint (one matrix per lane, blocks of
    # one size n <= 8 in one to four flavours) against the gradient oracle
    w = W.workload("mid", T=2, M=M, nf=nf, n_src=40, n_snk=70, branching=3, depth=3)
    print(f"tree backward nf={nf} M={M}", flush=True)
    plan, S, ws, wk = setup(w)
    rng = np.random.default_rng(11)
    g = rng.standard_normal(w.T) + 1j * rng.standard_normal(w.T)
    gS, gws, gwk = (x.cpu().numpy() for x in
                    mhc.contract_backward(plan, S, ws, wk, torch.from_numpy(g), "tree"))
    oS, ows, owk = og.vjp(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk, g)
    np.testing.assert_allclose(gS, oS, atol=1e-11 * np.abs(oS).max(), rtol=1e-9)
    np.testing.assert_allclose(gws, ows, atol=1e-11 * np.abs(ows).max(), rtol=1e-9)
    np.testing.assert_allclose(gwk, owk, atol=1e-11 * np.abs(owk).max(), rtol=1e-9)


def test_tree_backward_singular_for_some_sinks():
    # a zero column of S: a dominator's blocks are singular only against the
    # sinks that use that column, so within one wave some lanes take the
    # update tree and the others the pair-by-pair route
    w = W.workload("mid", T=2, M=12, nf=(3, 3), n_src=60, n_snk=130, branching=4, depth=2)
    w.S[:, :, 5] = 0
    plan, S, ws, wk = setup(w)
    uses = (w.snk == 5).any(axis=1)
    assert 0 < uses.sum() < len(w.snk)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(w.T) + 1j * rng.standard_normal(w.T)
    gS, gws, gwk = (x.cpu().numpy() for x in
                    mhc.contract_backward(plan, S, ws, wk, torch.from_numpy(g), "tree"))
    oS, ows, owk = og.vjp(w.S, w.src, w.snk, w.nf, w.w_src, w.w_snk, g)
    assert np.abs(oS[:, :, 5]).max() > 1e-3 * np.abs(oS).max()
    np.testing.assert_allclose(gS, oS, atol=1e-11 * np.abs(oS).max(), rtol=1e-9)
    np.testing.assert_allclose(gws, ows, atol=1e-11 * np.abs(ows).max(), rtol=1e-9)
    np.testing.assert_allclose(gwk, owk, atol=1e-11 * np.abs(owk).max(), rtol=1e-9)
    assert plan.status()["n_singular_grad"] > 0
