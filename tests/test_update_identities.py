"""Exact checks (Gaussian rationals) of the determinant identities the
update kernels evaluate in floating point, on small integer matrices:

* row change (matrix determinant lemma, Sec. 2):
  det G' / det G = s . G^-1 e_r;
* column change (the same lemma on the transpose, Sec. 3 allows rows or
  columns): det G' / det G = e_c^T G^-1 v;
* row r and column c changed together (rank-2 form of the lemma):
  det G' / det G = rho sigma - kappa (beta - alpha), with rho and sigma the
  two rank-1 ratios, kappa = (G^-1)[c][r], beta = s^T G^-1 v (s the new row
  over the old columns, v the new column over the old rows) and alpha the
  new corner entry.
These are not the oracle: the oracle evaluates the definitions; this file
pins the algebra of the two-sided update kernels."""
from fractions import Fraction

import numpy as np
import pytest

from oracle.det import QI, det_exact


def qmat(a):
    return [[QI(Fraction(int(x.real)), Fraction(int(x.imag))) for x in row] for row in a]


def inverse(G):
    n = len(G)
    d = det_exact(G)
    inv = [[None] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            minor = [[G[a][b] for b in range(n) if b != i] for a in range(n) if a != j]
            c = det_exact(minor) if n > 1 else QI(Fraction(1))
            if (i + j) % 2:
                c = -c
            inv[i][j] = c / d
    return inv


def dot(u, v):
    acc = QI(Fraction(0))
    for a, b in zip(u, v):
        acc = acc + a * b
    return acc


@pytest.mark.parametrize("seed", range(6))
def test_rank1_and_rank2_update_identities(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 5))
    while True:
        A = rng.integers(-4, 5, (n + 1, n + 1)) + 1j * rng.integers(-4, 5, (n + 1, n + 1))
        G = qmat(A[:n, :n])
        if not (det_exact(G) == QI(Fraction(0))):
            break
    r, c = int(rng.integers(n)), int(rng.integers(n))
    s = qmat(A[n:, :n])[0]                     # new row over the old columns
    v = [row[0] for row in qmat(A[:n, n:])]    # new column over the old rows
    alpha = qmat(A[n:, n:])[0][0]
    Gi = inverse(G)
    D = det_exact(G)
    rho = dot(s, [Gi[m][r] for m in range(n)])
    sigma = dot(Gi[c], v)
    kappa = Gi[c][r]
    beta = dot(s, [dot(Gi[m], v) for m in range(n)])
    row_changed = [list(G[m]) for m in range(n)]
    row_changed[r] = list(s)
    assert det_exact(row_changed) == D * rho
    col_changed = [list(G[m]) for m in range(n)]
    for m in range(n):
        col_changed[m][c] = v[m]
    assert det_exact(col_changed) == D * sigma
    both = [list(row) for row in row_changed]
    for m in range(n):
        both[m][c] = v[m]
    both[r][c] = alpha
    assert det_exact(both) == D * (rho * sigma - kappa * (beta - alpha))
