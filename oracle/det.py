"""Determinants of small complex matrices (oracle; test infrastructure only).

* ``det_gepp``   -- Sec. 2: the determinant from an LU factorisation.  The
  paper says the determinant is read from the LU decomposition and cites
  Golub & Van Loan; it is the product of U's diagonal times the sign of the
  row permutation.  Textbook Gaussian elimination with partial pivoting
  (GEPP): at step k the pivot is the remaining row with the largest
  |Re| + |Im| in column k, the lowest such row on ties.
* ``det_leibniz`` -- the permutation sum over one permutation (Sec. 1: the
  sum over orderings for one source/sink pair equals a determinant).
* ``double_permutation_sum`` -- the literal double sum over alpha and beta
  with both permutation signs, as printed in the correlator formula of Sec. 1.
* ``det_exact``  -- exact elimination over the Gaussian rationals; every
  float64 is a rational number, so this is the true determinant of the
  stored matrix.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def det_gepp(G) -> np.ndarray:
    """Batched GEPP determinant.  ``G``: complex [..., n, n] -> complex [...].

    Works on a batch axis so that a few million 6x6 matrices finish in
    seconds; the arithmetic per matrix is the textbook loop.
    """
    A = np.array(G, dtype=np.complex128, copy=True)
    batch_shape = A.shape[:-2]
    n = A.shape[-1]
    assert A.shape[-2] == n
    A = A.reshape(-1, n, n)
    B = A.shape[0]
    det = np.ones(B, dtype=np.complex128)
    rows = np.arange(B)
    for k in range(n):
        col = A[:, k:, k]
        mag = np.abs(col.real) + np.abs(col.imag)
        p = k + np.argmax(mag, axis=1)          # first maximum = lowest row
        swap = p != k
        if swap.any():
            rk = A[rows, k, :].copy()
            A[rows, k, :] = A[rows, p, :]
            A[rows, p, :] = rk
            det = np.where(swap, -det, det)
        piv = A[:, k, k]
        det = det * piv
        if k + 1 < n:
            safe = np.where(piv == 0, 1.0, piv)
            # a zero pivot means the whole remaining column is zero: the
            # determinant is already 0 and there is nothing to eliminate.
            lmul = np.where((piv == 0)[:, None], 0.0,
                            A[:, k + 1:, k] / safe[:, None])
            A[:, k + 1:, k + 1:] -= lmul[:, :, None] * A[:, None, k, k + 1:]
    return det.reshape(batch_shape)


def perm_sign(perm) -> int:
    """Sign of a permutation given as a sequence of 0..n-1 (inversion count)."""
    inv = 0
    for a in range(len(perm)):
        for b in range(a + 1, len(perm)):
            if perm[a] > perm[b]:
                inv += 1
    return -1 if inv % 2 else 1


class QI:
    """Exact Gaussian rational re + i*im (Fractions)."""
    __slots__ = ("re", "im")

    def __init__(self, re, im=Fraction(0)):
        self.re = Fraction(re)
        self.im = Fraction(im)

    @staticmethod
    def of(z) -> "QI":
        z = complex(z)
        return QI(Fraction(z.real), Fraction(z.imag))

    def __add__(self, o):
        return QI(self.re + o.re, self.im + o.im)

    def __sub__(self, o):
        return QI(self.re - o.re, self.im - o.im)

    def __mul__(self, o):
        return QI(self.re * o.re - self.im * o.im,
                  self.re * o.im + self.im * o.re)

    def __neg__(self):
        return QI(-self.re, -self.im)

    def __truediv__(self, o):
        d = o.re * o.re + o.im * o.im
        return QI((self.re * o.re + self.im * o.im) / d,
                  (self.im * o.re - self.re * o.im) / d)

    def is_zero(self):
        return self.re == 0 and self.im == 0

    def __eq__(self, o):
        return self.re == o.re and self.im == o.im

    def __complex__(self):
        return complex(float(self.re), float(self.im))


def _to_qi_matrix(G):
    G = np.asarray(G)
    n = G.shape[0]
    return [[QI.of(G[m, c]) for c in range(n)] for m in range(n)]


def det_exact(G) -> QI:
    """Exact determinant of one complex matrix (entries taken exactly)."""
    A = _to_qi_matrix(G)
    n = len(A)
    det = QI(1)
    for k in range(n):
        p = next((m for m in range(k, n) if not A[m][k].is_zero()), None)
        if p is None:
            return QI(0)
        if p != k:
            A[k], A[p] = A[p], A[k]
            det = -det
        det = det * A[k][k]
        for m in range(k + 1, n):
            if A[m][k].is_zero():
                continue
            l = A[m][k] / A[k][k]
            for c in range(k, n):
                A[m][c] = A[m][c] - l * A[k][c]
    return det


def det_leibniz(G, exact: bool = True):
    """Sum over permutations sigma of sgn(sigma) * prod_m G[m][sigma(m)].

    ``exact=True`` evaluates in Gaussian rationals (returns ``QI``)."""
    G = np.asarray(G)
    n = G.shape[0]
    if exact:
        A = _to_qi_matrix(G)
        acc = QI(0)
        for perm in itertools.permutations(range(n)):
            term = QI(perm_sign(perm))
            for m in range(n):
                term = term * A[m][perm[m]]
            acc = acc + term
        return acc
    acc = 0j
    for perm in itertools.permutations(range(n)):
        term = complex(perm_sign(perm))
        for m in range(n):
            term *= complex(G[m, perm[m]])
        acc += term
    return acc


def double_permutation_sum(S, src_idx, snk_idx) -> QI:
    """The pair term of the correlator formula of Sec. 1, taken literally:
    sum over two permutations alpha, beta of eps^alpha eps^beta times
    prod_m S(qbar(a_i^{alpha_m}), q(a_j^{beta_m})), exactly."""
    S = np.asarray(S)
    n = len(src_idx)
    acc = QI(0)
    for alpha in itertools.permutations(range(n)):
        sa = perm_sign(alpha)
        for beta in itertools.permutations(range(n)):
            term = QI(sa * perm_sign(beta))
            for m in range(n):
                term = term * QI.of(S[src_idx[alpha[m]], snk_idx[beta[m]]])
            acc = acc + term
    return acc
