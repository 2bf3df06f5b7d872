"""The correlator as a weighted double sum of determinants (oracle; test
infrastructure only).

Sec. 1 of the paper: for source term i and sink term j the sum over quark
orderings is det G^(ij) with G^(ij)[m][n] = S(qbar(a_i^m), q(a_j^n)); the
correlator at one time slice is  C = sum_i sum_j w_i w_j det G^(ij).
G is block diagonal over flavours, so det G is the product of the
determinants of the single-flavour blocks.

The gauge average (1/Z times the path integral) needs gauge ensembles and is
not computed: everything here is the integrand for one propagator per slice.

Terms are int arrays [n_terms][sum(nf)], flavour-major: the first nf[0]
entries are flavour 0's indices, then flavour 1's, and so on.
"""
from __future__ import annotations

import math

import numpy as np

from .det import det_gepp


def flavour_offsets(nf):
    return np.concatenate([[0], np.cumsum(nf)]).astype(int)


def gather_block(S_t, src_term, snk_term, nf, f):
    """G_f[m][n] = S_t[a_src^{f,m}][a_snk^{f,n}] for one pair (Sec. 1)."""
    o = flavour_offsets(nf)
    a = np.asarray(src_term)[o[f]:o[f + 1]]
    b = np.asarray(snk_term)[o[f]:o[f + 1]]
    return np.asarray(S_t)[np.ix_(a, b)]


def gather_full(S_t, src_term, snk_term):
    """The whole G (all flavours at once, no block structure assumed)."""
    a = np.asarray(src_term)
    b = np.asarray(snk_term)
    return np.asarray(S_t)[np.ix_(a, b)]


def pair_dets(S, src, snk, nf, t, i_idx, j_idx) -> np.ndarray:
    """d_ij(t) = prod_f det G_f^(ij)(t) for index arrays t, i_idx, j_idx
    (broadcast together).  Returns complex128 of the broadcast shape."""
    S = np.asarray(S)
    src = np.asarray(src)
    snk = np.asarray(snk)
    t, i_idx, j_idx = np.broadcast_arrays(np.asarray(t), np.asarray(i_idx),
                                          np.asarray(j_idx))
    shape = t.shape
    t = t.ravel()
    i_idx = i_idx.ravel()
    j_idx = j_idx.ravel()
    o = flavour_offsets(nf)
    d = np.ones(t.shape, dtype=np.complex128)
    for f in range(len(nf)):
        a = src[i_idx, o[f]:o[f + 1]]            # [P][n]
        b = snk[j_idx, o[f]:o[f + 1]]            # [P][n]
        G = S[t[:, None, None], a[:, :, None], b[:, None, :]]
        d = d * det_gepp(G)
    return d.reshape(shape)


def slice_pair_dets(S, src, snk, nf, t, chunk=1 << 18) -> np.ndarray:
    """All d_ij(t) for one slice: complex128 [n_src][n_snk]."""
    ns, nk = len(src), len(snk)
    out = np.empty((ns, nk), dtype=np.complex128)
    flat = out.reshape(-1)
    total = ns * nk
    for lo in range(0, total, chunk):
        hi = min(total, lo + chunk)
        idx = np.arange(lo, hi)
        flat[lo:hi] = pair_dets(S, src, snk, nf, t, idx // nk, idx % nk)
    return out


def weighted_terms(d, w_src, w_snk) -> np.ndarray:
    """w_i * w_j * d_ij for a [n_src][n_snk] block of determinants."""
    return (np.asarray(w_src)[:, None] * np.asarray(w_snk)[None, :]) * d


def exact_sum(z) -> complex:
    """Correctly rounded sum of the real and imaginary parts (math.fsum)."""
    z = np.asarray(z).ravel()
    return complex(math.fsum(z.real.tolist()), math.fsum(z.imag.tolist()))


def correlator(S, src, snk, nf, w_src, w_snk, slices=None):
    """C(t) = sum_i sum_j w_i w_j prod_f det G_f^(ij)(t) and the scale
    A(t) = sum_i sum_j |w_i w_j d_ij(t)|, for t in ``slices`` (default: all).

    Returns (C complex128 [len(slices)], A float64 [len(slices)])."""
    S = np.asarray(S)
    if slices is None:
        slices = range(S.shape[0])
    slices = list(slices)
    C = np.empty(len(slices), dtype=np.complex128)
    A = np.empty(len(slices), dtype=np.float64)
    for k, t in enumerate(slices):
        d = slice_pair_dets(S, src, snk, nf, t)
        z = weighted_terms(d, w_src, w_snk)
        C[k] = exact_sum(z)
        A[k] = math.fsum(np.abs(z).ravel().tolist())
    return C, A


def condition_1norm(G) -> np.ndarray:
    """kappa_1(G) = ||G||_1 ||G^-1||_1 for a batch [..., n, n] (used only to
    decide which tolerance a checked determinant is held to); inf for an
    exactly singular matrix."""
    G = np.asarray(G)
    shape = G.shape[:-2]
    n = G.shape[-1]
    flat = G.reshape(-1, n, n)
    n1 = np.abs(flat).sum(axis=-2).max(axis=-1)
    try:
        inv = np.linalg.inv(flat)
        ni = np.abs(inv).sum(axis=-2).max(axis=-1)
    except np.linalg.LinAlgError:
        ni = np.empty(len(flat))
        for b in range(len(flat)):
            try:
                ni[b] = np.abs(np.linalg.inv(flat[b])).sum(axis=-2).max()
            except np.linalg.LinAlgError:
                ni[b] = np.inf
    return (n1 * ni).reshape(shape)


def pair_condition(S, src, snk, nf, t, i_idx, j_idx) -> np.ndarray:
    """max over flavour blocks of kappa_1 for the given pairs."""
    S = np.asarray(S)
    src = np.asarray(src)
    snk = np.asarray(snk)
    t = np.asarray(t).ravel()
    i_idx = np.asarray(i_idx).ravel()
    j_idx = np.asarray(j_idx).ravel()
    o = flavour_offsets(nf)
    kap = np.zeros(t.shape)
    for f in range(len(nf)):
        a = src[i_idx, o[f]:o[f + 1]]
        b = snk[j_idx, o[f]:o[f + 1]]
        G = S[t[:, None, None], a[:, :, None], b[:, None, :]]
        with np.errstate(all="ignore"):
            k = condition_1norm(G)
        kap = np.maximum(kap, np.nan_to_num(k, nan=np.inf))
    return kap


def adjugate_1norm(G) -> np.ndarray:
    """||adj(G)||_1 for a batch [..., n, n], from the singular value
    decomposition (adj(G) = det(U) det(V^H) V diag(prod_{j != i} s_j) U^H),
    which stays defined when G is singular.  For a nonsingular G this is
    |det G| * ||G^-1||_1.  Used only to size test tolerances."""
    G = np.asarray(G)
    shape = G.shape[:-2]
    n = G.shape[-1]
    flat = G.reshape(-1, n, n)
    U, s, Vh = np.linalg.svd(flat)
    # prod_{j != i} s_j without dividing by a zero singular value
    cof = np.empty_like(s)
    for i in range(n):
        cof[:, i] = np.prod(np.delete(s, i, axis=1), axis=1)
    phase = np.linalg.det(U) * np.linalg.det(Vh)
    adj = phase[:, None, None] * np.einsum("bji,bj,bkj->bik", Vh.conj(), cof, U.conj())
    return np.abs(adj).sum(axis=-2).max(axis=-1).reshape(shape)


def pair_error_bound(S, src, snk, nf, t, i_idx, j_idx, c=4.0):
    """Per pair: (max over blocks of kappa_1, error bound).  A backward
    stable elimination of block f perturbs its entries by O(n eps ||G_f||),
    which moves det G_f by at most e_f = c n eps ||G_f||_1 ||adj G_f||_1; the
    product of the blocks then moves by at most
    prod_f (|det G_f| + e_f) - prod_f |det G_f|.  For regular blocks the
    first-order part is c n eps kappa_1 |d|; the bound stays finite and
    non-zero when blocks are singular.  Used only to size test tolerances."""
    S = np.asarray(S)
    src = np.asarray(src)
    snk = np.asarray(snk)
    t = np.asarray(t).ravel()
    i_idx = np.asarray(i_idx).ravel()
    j_idx = np.asarray(j_idx).ravel()
    o = flavour_offsets(nf)
    eps = np.finfo(np.float64).eps
    kap = np.zeros(t.shape)
    hi = np.ones(t.shape)
    lo = np.ones(t.shape)
    for f in range(len(nf)):
        n = nf[f]
        a = src[i_idx, o[f]:o[f + 1]]
        b = snk[j_idx, o[f]:o[f + 1]]
        G = S[t[:, None, None], a[:, :, None], b[:, None, :]]
        with np.errstate(all="ignore"):
            k = condition_1norm(G)
        kap = np.maximum(kap, np.nan_to_num(k, nan=np.inf))
        d = np.abs(det_gepp(G))
        e = c * n * eps * np.abs(G).sum(axis=-2).max(axis=-1) * adjugate_1norm(G)
        hi = hi * (d + e)
        lo = lo * d
    return kap, hi - lo
