"""Shared parity checks (numpy only): per-pair determinant and correlator
tolerances against the CPU oracle."""
import numpy as np

from oracle import contract as oc


def check_pairs(w, P, t, i, j):
    """Per-pair determinants of a dense table P[t][i][j] (check_pair_list)."""
    return check_pair_list(w, P[t, i, j], t, i, j)


def all_pairs(w):
    t, i, j = np.meshgrid(np.arange(w.T), np.arange(len(w.src)), np.arange(len(w.snk)),
                          indexing="ij")
    return t.ravel(), i.ravel(), j.ravel()


def check_C(C, A, Cw, Aw):
    assert np.all(np.abs(C - Cw) <= 1e-9 * Aw), np.max(np.abs(C - Cw) / Aw)
    np.testing.assert_allclose(A, Aw, rtol=1e-9)


def pair_reference(w, t, i, j):
    """The oracle's determinants and tolerance data for check_pair_list."""
    want = oc.pair_dets(w.S, w.src, w.snk, w.nf, t, i, j)
    kap, ebound = oc.pair_error_bound(w.S, w.src, w.snk, w.nf, t, i, j)
    return want, kap, ebound


def check_pair_list(w, got, t, i, j, ref=None):
    """Per-pair determinants got[q] = d_{i[q] j[q]}(t[q]): 1e-11 relative
    when every block has kappa_1 <= 1e4; otherwise within the bound
    prod_f(|det G_f| + e_f) - prod_f |det G_f|, e_f = 4 n eps ||G_f||_1
    ||adj G_f||_1 (first order: 4 n eps kappa_1 |d| for regular blocks;
    finite when blocks are singular)."""
    want, kap, ebound = ref if ref is not None else pair_reference(w, t, i, j)
    err = np.abs(got - want)
    well = kap <= 1e4
    bound = np.where(well, 1e-11 * np.abs(want), ebound)
    bad = ~(err <= bound)
    with np.errstate(divide="ignore", invalid="ignore"):
        worst = (err / bound)[bad].max() if bad.any() else 0.0
    assert not bad.any(), f"{bad.sum()} of {bad.size} pairs out of tolerance; worst err/bound {worst:.3e}"
    return int(well.sum()), int((~well).sum())
