"""Pins of the gradient oracle against identities and finite differences
that use only the forward definition."""
import numpy as np
import pytest

from oracle import contract as oc
from oracle import det as od
from oracle import grad as og


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def case(seed, T=2, M=7, nf=(2, 3), ns=6, nk=5):
    rng = np.random.default_rng(seed)
    S = rand_c(rng, (T, M, M))
    src = np.stack([np.concatenate([rng.choice(M, n, replace=False) for n in nf]) for _ in range(ns)])
    snk = np.stack([np.concatenate([rng.choice(M, n, replace=False) for n in nf]) for _ in range(nk)])
    return rng, S, src, snk, rng.standard_normal(ns), rng.standard_normal(nk), nf


def test_cofactors_exact_and_laplace():
    rng = np.random.default_rng(1)
    G = rand_c(rng, (4, 4))
    cof = og.cofactors(G[None])[0]
    for m in range(4):
        for n in range(4):
            minor = np.delete(np.delete(G, m, 0), n, 1)
            ex = od.det_exact(minor)
            want = (-1) ** (m + n) * complex(float(ex.re), float(ex.im))
            assert cof[m, n] == pytest.approx(want, rel=1e-12)
    # Laplace expansion along every row and column gives det G
    d = od.det_gepp(G)
    for m in range(4):
        assert np.sum(G[m] * cof[m]) == pytest.approx(d, rel=1e-12)
        assert np.sum(G[:, m] * cof[:, m]) == pytest.approx(d, rel=1e-12)


def test_euler_homogeneity():
    # C(t) is homogeneous of degree sum(nf) in S_t
    rng, S, src, snk, ws, wk, nf = case(2)
    C, _ = oc.correlator(S, src, snk, nf, ws, wk)
    dS = og.dC_dS(S, src, snk, nf, ws, wk)
    for t in range(S.shape[0]):
        assert np.sum(S[t] * dS[t]) == pytest.approx(sum(nf) * C[t], rel=1e-11)


def test_weight_derivatives_reproduce_C():
    rng, S, src, snk, ws, wk, nf = case(3)
    C, _ = oc.correlator(S, src, snk, nf, ws, wk)
    gs, gk = og.dC_dw(S, src, snk, nf, ws, wk)
    np.testing.assert_allclose(gs @ ws, C, rtol=1e-12)
    np.testing.assert_allclose(gk @ wk, C, rtol=1e-12)
    gs2, gk2 = og.dC_dw_entries(S, src, snk, nf, ws, wk, [0, 4], [1, 3])
    np.testing.assert_allclose(gs2, gs[:, [0, 4]], rtol=1e-13)
    np.testing.assert_allclose(gk2, gk[:, [1, 3]], rtol=1e-13)


def test_dS_against_complex_central_differences():
    rng, S, src, snk, ws, wk, nf = case(4)
    h = 1e-6
    for (t, p, q) in [(0, 1, 2), (1, 3, 3), (0, 6, 0), (1, 0, 5)]:
        want = og.dC_dS_entry(S, src, snk, nf, ws, wk, t, p, q)
        for step in (h, 1j * h):       # real and imaginary directions agree (holomorphic)
            Sp = S.copy()
            Sm = S.copy()
            Sp[t, p, q] += step
            Sm[t, p, q] -= step
            Cp, _ = oc.correlator(Sp, src, snk, nf, ws, wk, slices=[t])
            Cm, _ = oc.correlator(Sm, src, snk, nf, ws, wk, slices=[t])
            fd = (Cp[0] - Cm[0]) / (2 * step)
            assert abs(fd - want) <= 1e-7 * max(1.0, abs(want))


def test_vjp_against_finite_differences_of_a_real_loss():
    # L = Re(sum_t conj(g_t) C_t): dL/dw = Re(sum_t g_t conj(dC_t/dw)) and
    # dL/dRe(S) + i dL/dIm(S) = g_t conj(dC_t/dS_t)
    rng, S, src, snk, ws, wk, nf = case(5)
    g = rand_c(rng, S.shape[0])
    gS, gws, gwk = og.vjp(S, src, snk, nf, ws, wk, g)

    def L(S_, ws_, wk_):
        C, _ = oc.correlator(S_, src, snk, nf, ws_, wk_)
        return float(np.real(np.sum(np.conj(g) * C)))

    h = 1e-6
    for i in range(len(ws)):
        e = np.zeros(len(ws))
        e[i] = h
        fd = (L(S, ws + e, wk) - L(S, ws - e, wk)) / (2 * h)
        assert fd == pytest.approx(gws[i], rel=1e-7, abs=1e-9)
    for j in range(len(wk)):
        e = np.zeros(len(wk))
        e[j] = h
        fd = (L(S, ws, wk + e) - L(S, ws, wk - e)) / (2 * h)
        assert fd == pytest.approx(gwk[j], rel=1e-7, abs=1e-9)
    for (t, p, q) in [(0, 2, 2), (1, 5, 1)]:
        E = np.zeros(S.shape, complex)
        E[t, p, q] = h
        fx = (L(S + E, ws, wk) - L(S - E, ws, wk)) / (2 * h)
        fy = (L(S + 1j * E, ws, wk) - L(S - 1j * E, ws, wk)) / (2 * h)
        assert complex(fx, fy) == pytest.approx(gS[t, p, q], rel=1e-7, abs=1e-9)


def test_single_cofactor_matches_full_table():
    rng = np.random.default_rng(6)
    G = rand_c(rng, (20, 5, 5))
    m = rng.integers(0, 5, 20)
    n = rng.integers(0, 5, 20)
    full = og.cofactors(G)
    np.testing.assert_allclose(og.cofactor_at(G, m, n), full[np.arange(20), m, n], rtol=1e-13)
