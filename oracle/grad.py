"""Derivatives of the correlator (oracle; test infrastructure only).

The correlator of Sec. 1, C(t) = sum_ij w_i w'_j prod_f det G_f^(ij)(t), is
bilinear in the weights and holomorphic in the propagator entries.  Its
derivatives, written out from the definitions:

* dC(t)/dw_i  = sum_j w'_j d_ij(t),   dC(t)/dw'_j = sum_i w_i d_ij(t);
* dC(t)/dS_t[p][q] = sum_ij w_i w'_j sum_f (prod_{f' != f} det G_f')
                     sum_{m,n: a_i^{f,m} = p, a_j^{f,n} = q} adj(G_f)[n][m],
  by Jacobi's formula d det(G)/dG[m][n] = adj(G)[n][m], the (m, n)
  cofactor.  Cofactors are taken here as signed determinants of minors
  (``det_gepp``), not through an inverse.

Vector-Jacobian products follow PyTorch's convention for a real loss with
incoming gradient gC[t]: grad_S = gC[t] * conj(dC(t)/dS_t) and, for the real
weights, grad_w = Re(sum_t gC[t] * conj(dC(t)/dw)).
"""
from __future__ import annotations

import math

import numpy as np

from .contract import flavour_offsets, pair_dets, slice_pair_dets
from .det import det_gepp


def cofactors(G) -> np.ndarray:
    """cof[..., m, n] = (-1)^(m+n) det(G with row m and column n removed)."""
    G = np.asarray(G)
    n = G.shape[-1]
    out = np.empty(G.shape, dtype=np.complex128)
    if n == 1:
        out[...] = 1.0
        return out
    for m in range(n):
        rows = [r for r in range(n) if r != m]
        for c in range(n):
            cols = [k for k in range(n) if k != c]
            minor = G[..., rows, :][..., :, cols]
            out[..., m, c] = (-1) ** (m + c) * det_gepp(minor)
    return out


def dC_dw(S, src, snk, nf, w_src, w_snk):
    """(dC/dw_src [T][n_src], dC/dw_snk [T][n_snk]) as complex arrays."""
    T = np.asarray(S).shape[0]
    gs = np.empty((T, len(src)), dtype=np.complex128)
    gk = np.empty((T, len(snk)), dtype=np.complex128)
    for t in range(T):
        d = slice_pair_dets(S, src, snk, nf, t)
        for i in range(len(src)):
            gs[t, i] = complex(math.fsum((d[i].real * w_snk).tolist()),
                               math.fsum((d[i].imag * w_snk).tolist()))
        for j in range(len(snk)):
            gk[t, j] = complex(math.fsum((d[:, j].real * w_src).tolist()),
                               math.fsum((d[:, j].imag * w_src).tolist()))
    return gs, gk


def dC_dw_entries(S, src, snk, nf, w_src, w_snk, src_idx=(), snk_idx=()):
    """dC(t)/dw_i for i in src_idx and dC(t)/dw'_j for j in snk_idx, every t:
    complex [T][len(src_idx)] and [T][len(snk_idx)]."""
    S = np.asarray(S)
    src = np.asarray(src)
    snk = np.asarray(snk)
    T = S.shape[0]
    gs = np.empty((T, len(src_idx)), dtype=np.complex128)
    gk = np.empty((T, len(snk_idx)), dtype=np.complex128)
    for t in range(T):
        for k, i in enumerate(src_idx):
            d = pair_dets(S, src, snk, nf, t, i, np.arange(len(snk)))
            z = d * np.asarray(w_snk)
            gs[t, k] = complex(math.fsum(z.real.tolist()), math.fsum(z.imag.tolist()))
        for k, j in enumerate(snk_idx):
            d = pair_dets(S, src, snk, nf, t, np.arange(len(src)), j)
            z = d * np.asarray(w_src)
            gk[t, k] = complex(math.fsum(z.real.tolist()), math.fsum(z.imag.tolist()))
    return gs, gk


def cofactor_at(G, m, n) -> np.ndarray:
    """The single cofactor (-1)^(m+n) det(minor(m, n)) of each matrix of a
    batch G [B][k][k] at per-matrix positions m[B], n[B]."""
    G = np.asarray(G)
    B, k, _ = G.shape
    if k == 1:
        return np.ones(B, dtype=np.complex128)
    base = np.arange(k - 1)
    rows = base[None, :] + (base[None, :] >= np.asarray(m)[:, None])   # skip row m
    cols = base[None, :] + (base[None, :] >= np.asarray(n)[:, None])   # skip column n
    minor = G[np.arange(B)[:, None, None], rows[:, :, None], cols[:, None, :]]
    sign = np.where((np.asarray(m) + np.asarray(n)) % 2 == 0, 1.0, -1.0)
    return sign * det_gepp(minor)


def dC_dS_entry(S, src, snk, nf, w_src, w_snk, t, p, q, with_scale=False):
    """dC(t)/dS_t[p][q] for one propagator entry (and, with with_scale, the
    sum of the magnitudes of its terms)."""
    S = np.asarray(S)
    src = np.asarray(src)
    snk = np.asarray(snk)
    o = flavour_offsets(nf)
    terms = []
    for f in range(len(nf)):
        a = src[:, o[f]:o[f + 1]]
        b = snk[:, o[f]:o[f + 1]]
        src_hit = np.nonzero((a == p).any(axis=1))[0]
        snk_hit = np.nonzero((b == q).any(axis=1))[0]
        if len(src_hit) == 0 or len(snk_hit) == 0:
            continue
        ii, jj = np.meshgrid(src_hit, snk_hit, indexing="ij")
        ii = ii.ravel()
        jj = jj.ravel()
        m = np.argmax(a[ii] == p, axis=1)          # row of p in block f
        n = np.argmax(b[jj] == q, axis=1)          # column of q in block f
        G = S[t][a[ii][:, :, None], b[jj][:, None, :]]
        cof = cofactor_at(G, m, n)
        other = np.ones(len(ii), dtype=np.complex128)
        for g in range(len(nf)):
            if g == f:
                continue
            ag = src[ii, o[g]:o[g + 1]]
            bg = snk[jj, o[g]:o[g + 1]]
            other = other * det_gepp(S[t][ag[:, :, None], bg[:, None, :]])
        terms.append(np.asarray(w_src)[ii] * np.asarray(w_snk)[jj] * other * cof)
    if not terms:
        return (0j, 0.0) if with_scale else 0j
    z = np.concatenate(terms)
    val = complex(math.fsum(z.real.tolist()), math.fsum(z.imag.tolist()))
    if with_scale:
        return val, math.fsum(np.abs(z).tolist())
    return val


def dC_dS(S, src, snk, nf, w_src, w_snk) -> np.ndarray:
    """Every dC(t)/dS_t[p][q]: complex [T][M][M] (small cases only)."""
    S = np.asarray(S)
    T, M, _ = S.shape
    out = np.zeros((T, M, M), dtype=np.complex128)
    for t in range(T):
        for p in range(M):
            for q in range(M):
                out[t, p, q] = dC_dS_entry(S, src, snk, nf, w_src, w_snk, t, p, q)
    return out


def vjp(S, src, snk, nf, w_src, w_snk, gC, entries=None):
    """(grad_S, grad_w_src, grad_w_snk) for incoming gradient gC[T].

    ``entries``: optional list of (t, p, q); then grad_S holds only those
    entries (as a dict), else the full [T][M][M] array."""
    gC = np.asarray(gC)
    gs, gk = dC_dw(S, src, snk, nf, w_src, w_snk)
    g_wsrc = np.real(gC[:, None] * np.conj(gs)).sum(axis=0)
    g_wsnk = np.real(gC[:, None] * np.conj(gk)).sum(axis=0)
    if entries is None:
        d = dC_dS(S, src, snk, nf, w_src, w_snk)
        gS = gC[:, None, None] * np.conj(d)
    else:
        gS = {(t, p, q): gC[t] * np.conj(dC_dS_entry(S, src, snk, nf, w_src, w_snk, t, p, q))
              for (t, p, q) in entries}
    return gS, g_wsrc, g_wsnk


__all__ = ["cofactors", "cofactor_at", "dC_dw", "dC_dw_entries", "dC_dS_entry", "dC_dS", "vjp"]
