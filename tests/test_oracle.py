"""Pins of the CPU oracle's determinant and correlator code against values
fixed by the mathematics, independently of the oracle itself.

* exact rational determinants (elimination and the Leibniz sum, Sec. 1);
* the literal double permutation sum of the correlator formula (Sec. 1);
* closed forms (triangular, permutation, diagonal, zero row);
* an independent library routine (LAPACK through numpy.linalg.det);
* a hand-worked example (tests/golden/worked_example.json);
* identities of the correlator: bilinearity in the weights, homogeneity in
  S, invariance under reordering terms, antisymmetry of the index tuples.
* the rank-1 update identity of Sec. 2 (matrix determinant lemma) and the
  sharing of one solve among siblings, which the GPU update path relies on.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import contract as oc
from oracle import det as od

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = np.finfo(np.float64).eps


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def qi_to_complex(q):
    return complex(float(q.re), float(q.im))


# ----------------------------------------------------------------- det_gepp

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gepp_matches_exact_rational(n):
    rng = np.random.default_rng(100 + n)
    G = rand_c(rng, (12, n, n))
    d = od.det_gepp(G)
    kap = oc.condition_1norm(G)
    for b in range(len(G)):
        ex = qi_to_complex(od.det_exact(G[b]))
        bound = 8 * n * EPS * kap[b] * abs(ex) + 1e-300
        assert abs(d[b] - ex) <= bound, (n, b, d[b], ex)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exact_elimination_equals_leibniz(n):
    rng = np.random.default_rng(200 + n)
    for _ in range(3):
        G = rand_c(rng, (n, n))
        a = od.det_exact(G)
        b = od.det_leibniz(G, exact=True)
        assert a == b


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_double_permutation_sum_is_nfactorial_det(n):
    # The correlator formula of Sec. 1 sums over two permutations; for one
    # pair this is n! det G exactly (the n! is dropped by the paper's restated
    # formula, which is what the oracle and the library compute).
    rng = np.random.default_rng(300 + n)
    M = 7
    S = rand_c(rng, (M, M))
    a = rng.choice(M, n, replace=False)
    b = rng.choice(M, n, replace=False)
    lhs = od.double_permutation_sum(S, a, b)
    G = S[np.ix_(a, b)]
    rhs = od.det_leibniz(G, exact=True)
    assert lhs.re == math.factorial(n) * rhs.re
    assert lhs.im == math.factorial(n) * rhs.im


def test_gepp_closed_forms():
    rng = np.random.default_rng(7)
    n = 6
    # upper triangular: no row exchange happens, det = product of diagonal
    U = np.triu(rand_c(rng, (n, n)))
    prod = np.prod(np.diag(U))
    assert od.det_gepp(U) == pytest.approx(prod, rel=4 * n * EPS)
    # lower triangular (elimination does exchange rows here)
    L = np.tril(rand_c(rng, (n, n)))
    ex = qi_to_complex(od.det_exact(L))
    assert abs(od.det_gepp(L) - np.prod(np.diag(L))) <= 1e-13 * abs(ex)
    # permutation matrices: det = sign, exactly
    for perm in itertools.islice(itertools.permutations(range(5)), 0, 120, 7):
        P = np.zeros((5, 5), complex)
        P[np.arange(5), perm] = 1
        assert od.det_gepp(P) == od.perm_sign(perm)
    # a zero row or zero column gives exactly 0
    Z = rand_c(rng, (n, n))
    Z[3] = 0
    assert od.det_gepp(Z) == 0
    Z = rand_c(rng, (n, n))
    Z[:, 2] = 0
    assert od.det_gepp(Z) == 0
    # identity
    assert od.det_gepp(np.eye(n, dtype=complex)) == 1


def test_gepp_row_operations():
    rng = np.random.default_rng(8)
    G = rand_c(rng, (50, 6, 6))
    d = od.det_gepp(G)
    Gs = G.copy()
    Gs[:, [1, 4]] = Gs[:, [4, 1]]
    np.testing.assert_allclose(od.det_gepp(Gs), -d, rtol=1e-12)
    lam = 0.3 - 1.7j
    Gl = G.copy()
    Gl[:, 2] *= lam
    np.testing.assert_allclose(od.det_gepp(Gl), lam * d, rtol=1e-12)
    # transposition leaves the determinant unchanged
    np.testing.assert_allclose(od.det_gepp(np.swapaxes(G, 1, 2)), d, rtol=1e-12)


def test_gepp_matches_lapack():
    rng = np.random.default_rng(9)
    for n in (2, 3, 6, 12):
        G = rand_c(rng, (200, n, n))
        np.testing.assert_allclose(od.det_gepp(G), np.linalg.det(G),
                                   rtol=1e-11)


def test_gepp_pivot_is_largest_magnitude():
    # A matrix whose unpivoted elimination divides by a tiny pivot: partial
    # pivoting keeps full accuracy (checked against the exact determinant).
    G = np.array([[1e-17, 1.0, 2.0], [1.0, 1.0, 0.5], [2.0, -1.0, 1.0]],
                 dtype=complex)
    ex = qi_to_complex(od.det_exact(G))
    assert abs(od.det_gepp(G) - ex) <= 4 * EPS * abs(ex)


# ------------------------------------------------------ flavour blocks (Sec. 1)

def test_block_diagonal_product():
    rng = np.random.default_rng(10)
    M = 20
    nf = (3, 2, 4)
    S = rand_c(rng, (1, M, M))
    src = np.concatenate([rng.choice(M, n, replace=False) for n in nf])
    snk = np.concatenate([rng.choice(M, n, replace=False) for n in nf])
    big = np.zeros((sum(nf), sum(nf)), complex)
    o = oc.flavour_offsets(nf)
    for f in range(len(nf)):
        big[o[f]:o[f + 1], o[f]:o[f + 1]] = oc.gather_block(S[0], src, snk, nf, f)
    ex = qi_to_complex(od.det_exact(big))
    d = oc.pair_dets(S, src[None], snk[None], nf, 0, 0, 0)
    assert abs(d - ex) <= 1e-13 * abs(ex)


# ------------------------------------------------------------ hand example

def load_worked():
    with open(os.path.join(HERE, "golden", "worked_example.json")) as fh:
        g = json.load(fh)
    S = (np.array(g["S_re"], float) + 1j * np.array(g["S_im"], float))[None]
    return g, S


def test_worked_example():
    g, S = load_worked()
    src = np.array(g["src"])
    snk = np.array(g["snk"])
    nf = tuple(g["nf"])
    C, A = oc.correlator(S, src, snk, nf, g["w_src"], g["w_snk"])
    assert C[0] == complex(g["C_re"], g["C_im"])
    assert A[0] == pytest.approx(g["A"], rel=1e-15)
    d = oc.slice_pair_dets(S, src, snk, nf, 0)
    expect = np.array(g["pair_det_re"]) + 1j * np.array(g["pair_det_im"])
    np.testing.assert_array_equal(d, expect)


# ------------------------------------------------------ correlator identities

def small_case(seed, T=2, M=10, nf=(3, 2), ns=7, nk=5):
    rng = np.random.default_rng(seed)
    S = rand_c(rng, (T, M, M))
    src = np.stack([np.concatenate([rng.choice(M, n, replace=False) for n in nf])
                    for _ in range(ns)])
    snk = np.stack([np.concatenate([rng.choice(M, n, replace=False) for n in nf])
                    for _ in range(nk)])
    return rng, S, src, snk, rng.standard_normal(ns), rng.standard_normal(nk), nf


def test_correlator_against_exact_brute_force():
    rng, S, src, snk, ws, wk, nf = small_case(11)
    C, A = oc.correlator(S, src, snk, nf, ws, wk)
    o = oc.flavour_offsets(nf)
    for t in range(S.shape[0]):
        acc_re = Fraction(0)
        acc_im = Fraction(0)
        for i in range(len(src)):
            for j in range(len(snk)):
                # the full G with zero cross-flavour blocks, determinant exact
                big = np.zeros((sum(nf), sum(nf)), complex)
                for f in range(len(nf)):
                    a = src[i, o[f]:o[f + 1]]
                    b = snk[j, o[f]:o[f + 1]]
                    big[o[f]:o[f + 1], o[f]:o[f + 1]] = S[t][np.ix_(a, b)]
                dq = od.det_leibniz(big, exact=True) if sum(nf) <= 5 else od.det_exact(big)
                wq = Fraction(ws[i]) * Fraction(wk[j])
                acc_re += wq * dq.re
                acc_im += wq * dq.im
        ex = complex(float(acc_re), float(acc_im))
        assert abs(C[t] - ex) <= 1e-13 * A[t]


def test_single_term_wavefunction():
    rng, S, src, snk, ws, wk, nf = small_case(12, ns=1, nk=1)
    C, _ = oc.correlator(S, src, snk, nf, ws, wk)
    o = oc.flavour_offsets(nf)
    for t in range(S.shape[0]):
        d = 1
        for f in range(len(nf)):
            d *= np.linalg.det(S[t][np.ix_(src[0, o[f]:o[f + 1]], snk[0, o[f]:o[f + 1]])])
        assert C[t] == pytest.approx(ws[0] * wk[0] * d, rel=1e-12)


def test_bilinear_in_weights():
    rng, S, src, snk, ws, wk, nf = small_case(13)
    ws2 = rng.standard_normal(len(ws))
    wk2 = rng.standard_normal(len(wk))
    a, b = 0.7, -1.3
    C1, A1 = oc.correlator(S, src, snk, nf, ws, wk)
    C2, A2 = oc.correlator(S, src, snk, nf, ws2, wk)
    C12, _ = oc.correlator(S, src, snk, nf, a * ws + b * ws2, wk)
    np.testing.assert_allclose(C12, a * C1 + b * C2, atol=1e-13 * (A1 + A2).max())
    C3, A3 = oc.correlator(S, src, snk, nf, ws, wk2)
    C13, _ = oc.correlator(S, src, snk, nf, ws, a * wk + b * wk2)
    np.testing.assert_allclose(C13, a * C1 + b * C3, atol=1e-13 * (A1 + A3).max())
    # a unit source weight picks out one row of pair determinants
    e = np.zeros(len(ws))
    e[2] = 1.0
    Ce, _ = oc.correlator(S, src, snk, nf, e, wk)
    d = oc.slice_pair_dets(S, src, snk, nf, 1)
    assert Ce[1] == pytest.approx(np.dot(d[2], wk), rel=1e-12)


def test_homogeneous_in_S():
    # S_t = lam_t S_0  =>  C(t) = lam_t^(sum nf) C(0)
    rng, S, src, snk, ws, wk, nf = small_case(14, T=3)
    lam = np.array([1.0, 0.5 - 0.25j, 2.0j])
    Ssh = lam[:, None, None] * S[0][None]
    C, A = oc.correlator(Ssh, src, snk, nf, ws, wk)
    for t in range(3):
        assert abs(C[t] - lam[t] ** sum(nf) * C[0]) <= 1e-13 * A[t]


def test_reordering_terms_invariant():
    rng, S, src, snk, ws, wk, nf = small_case(15)
    C, A = oc.correlator(S, src, snk, nf, ws, wk)
    ps = rng.permutation(len(src))
    pk = rng.permutation(len(snk))
    C2, _ = oc.correlator(S, src[ps], snk[pk], nf, ws[ps], wk[pk])
    np.testing.assert_allclose(C2, C, atol=1e-14 * A.max())


def test_antisymmetry_of_index_tuples():
    # Swapping two indices of one flavour in a source term flips the sign of
    # its determinants (w is antisymmetric, Sec. 1).
    rng, S, src, snk, ws, wk, nf = small_case(16)
    d = oc.slice_pair_dets(S, src, snk, nf, 0)
    src2 = src.copy()
    src2[3, [0, 2]] = src2[3, [2, 0]]
    d2 = oc.slice_pair_dets(S, src2, snk, nf, 0)
    np.testing.assert_allclose(d2[3], -d[3], rtol=1e-12)
    np.testing.assert_array_equal(np.delete(d2, 3, 0), np.delete(d, 3, 0))


# --------------------------------------------- rank-1 updates (Sec. 2 identities)

@pytest.mark.parametrize("n", [2, 3, 5])
def test_determinant_lemma_exact(n):
    # det(G + e_r v^T) = (1 + v^T G^-1 e_r) det G, in exact arithmetic; the
    # GPU update path evaluates it as  newrow . G^-1 e_r  (the two forms are
    # equal because oldrow . G^-1 e_r = 1).
    rng = np.random.default_rng(400 + n)
    G = rand_c(rng, (n, n))
    r = n - 1
    newrow = rand_c(rng, n)
    Gq = od._to_qi_matrix(G)
    dG = od.det_exact(G)
    # x = G^-1 e_r by Cramer's rule, exactly: x_m = det(G with column m := e_r)/det G
    x = []
    for m in range(n):
        H = [row[:] for row in Gq]
        for q in range(n):
            H[q][m] = od.QI(1 if q == r else 0)
        Hm = np.array([[complex(h) for h in row] for row in H])
        # exact: rebuild from QI (entries are exact small rationals)
        x.append(_det_qi(H) / dG)
    v = [od.QI.of(newrow[m]) - Gq[r][m] for m in range(n)]
    one_plus = od.QI(1)
    newdot = od.QI(0)
    for m in range(n):
        one_plus = one_plus + v[m] * x[m]
        newdot = newdot + od.QI.of(newrow[m]) * x[m]
    assert one_plus == newdot
    Gc = G.copy()
    Gc[r] = newrow
    assert od.det_exact(Gc) == one_plus * dG


def _det_qi(A):
    A = [row[:] for row in A]
    n = len(A)
    det = od.QI(1)
    for k in range(n):
        p = next((m for m in range(k, n) if not A[m][k].is_zero()), None)
        if p is None:
            return od.QI(0)
        if p != k:
            A[k], A[p] = A[p], A[k]
            det = -det
        det = det * A[k][k]
        for m in range(k + 1, n):
            l = A[m][k] / A[k][k]
            for c in range(k, n):
                A[m][c] = A[m][c] - l * A[k][c]
    return det


def test_sibling_sharing_and_multilinearity():
    # Children that change the same row r of one parent share x = G^-1 e_r
    # (Sec. 2); by multilinearity in row r their weighted sum is one
    # determinant with the weighted row.
    rng = np.random.default_rng(17)
    n = 6
    G = rand_c(rng, (n, n))
    r = 2
    rows = rand_c(rng, (5, n))
    w = rng.standard_normal(5)
    x = np.linalg.solve(G, np.eye(n)[:, r])
    dG = od.det_gepp(G)
    for k in range(5):
        Gk = G.copy()
        Gk[r] = rows[k]
        assert dG * (rows[k] @ x) == pytest.approx(od.det_gepp(Gk), rel=1e-11)
    Gw = G.copy()
    Gw[r] = w @ rows
    tot = sum(w[k] * od.det_gepp(np.vstack([G[:r], rows[k][None], G[r + 1:]]))
              for k in range(5))
    assert tot == pytest.approx(od.det_gepp(Gw), rel=1e-11)


def test_adjugate_norm_against_cofactors():
    # the tolerance helper's ||adj G||_1 against cofactors by brute force,
    # for a regular and an exactly singular matrix
    rng = np.random.default_rng(31)
    for singular in (False, True):
        G = rand_c(rng, (4, 4))
        if singular:
            G[2] = G[0]
        C = np.zeros((4, 4), complex)
        for r in range(4):
            for c in range(4):
                minor = np.delete(np.delete(G, r, 0), c, 1)
                C[r, c] = (-1) ** (r + c) * qi_to_complex(od.det_exact(minor))
        want = np.abs(C.T).sum(axis=0).max()
        assert oc.adjugate_1norm(G[None])[0] == pytest.approx(want, rel=1e-12)
