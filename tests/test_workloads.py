"""The seeded input generators: determinism, the structure the paper's
workload has (single-index substitution trees, distinct indices within a
flavour), and a clear error for impossible requests."""
import numpy as np
import pytest

from paper_1411_3691_amd import workloads as W


def test_deterministic():
    a = W.workload("mid", T=2, n_src=300, n_snk=100)
    b = W.workload("mid", T=2, n_src=300, n_snk=100)
    for x, y in ((a.S, b.S), (a.src, b.src), (a.snk, b.snk), (a.w_src, b.w_src)):
        np.testing.assert_array_equal(x, y)


def test_tree_terms_structure():
    w = W.workload("mid", T=1)
    o = np.concatenate([[0], np.cumsum(w.nf)])
    seen = set()
    for t in w.src:
        assert tuple(t) not in seen
        seen.add(tuple(t))
        for f in range(len(w.nf)):
            blk = t[o[f]:o[f + 1]]
            assert len(set(blk.tolist())) == len(blk)
            assert blk.min() >= 0 and blk.max() < w.M
    # most terms have a neighbour at Hamming distance 1
    src = w.src[:400]
    d = (src[:, None, :] != src[None, :, :]).sum(-1)
    assert ((d == 1).sum(1) > 0).mean() > 0.9


def test_propagator_decay_and_shared_variant():
    w = W.workload("mid", T=4, n_src=10, n_snk=10, shared_S=True)
    for t in range(4):
        np.testing.assert_allclose(w.S[t], np.exp(-0.5 * t) * w.S[0], rtol=1e-15)


def test_impossible_request_raises():
    with pytest.raises(ValueError):
        W.workload("mid", T=1, M=6, nf=(1, 1), n_src=70, n_snk=10)
