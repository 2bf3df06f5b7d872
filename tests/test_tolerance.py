"""The parity tolerances accept an independent backward-stable method
(LAPACK through numpy) on the hardest inputs the GPU tests use, and reject
a plausible mistake."""
import numpy as np
import pytest

from oracle import contract as oc
from paper_1411_3691_amd import workloads as W
from parity_util import all_pairs, check_pairs


def lapack_pairs(w):
    t, i, j = all_pairs(w)
    o = oc.flavour_offsets(w.nf)
    d = np.ones(t.shape, complex)
    for f in range(len(w.nf)):
        a = w.src[i, o[f]:o[f + 1]]
        b = w.snk[j, o[f]:o[f + 1]]
        d *= np.linalg.det(w.S[t[:, None, None], a[:, :, None], b[:, None, :]])
    return d.reshape(w.T, len(w.src), len(w.snk))


@pytest.mark.parametrize("mutate", ["none", "zero_row", "equal_rows"])
def test_lapack_passes_pair_tolerance(mutate):
    w = W.workload("mid", T=2, M=12, n_src=120, n_snk=70, branching=6, depth=3)
    if mutate == "zero_row":
        w.S[:, 5, :] = 0
    elif mutate == "equal_rows":
        w.S[:, 5, :] = w.S[:, 3, :]
    check_pairs(w, lapack_pairs(w), *all_pairs(w))


def test_pair_tolerance_rejects_a_dropped_flavour():
    w = W.workload("mid", T=1, n_src=40, n_snk=30)
    P = lapack_pairs(w)
    o = oc.flavour_offsets(w.nf)
    t, i, j = all_pairs(w)
    a = w.src[i, o[1]:o[2]]
    b = w.snk[j, o[1]:o[2]]
    P_wrong = P / np.linalg.det(w.S[t[:, None, None], a[:, :, None], b[:, None, :]]).reshape(P.shape)
    with pytest.raises(AssertionError):
        check_pairs(w, P_wrong, *all_pairs(w))
