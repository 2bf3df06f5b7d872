"""CPU oracle for the multi-hadron correlator contraction.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path (the C-ABI library,
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the benchmark's CPU-baseline leg use it.

It is a plain, slow, deliberately unoptimised restatement of what the paper
computes, in float64 (complex128) or exact rational arithmetic:

* ``det``      -- determinants: Gaussian elimination with partial pivoting
                  (Sec. 2, the LU route the paper names), the Leibniz
                  permutation sum and the double permutation sum of the
                  correlator formula (Sec. 1), and exact rational elimination.
* ``contract`` -- the correlator as the weighted double sum of per-pair
                  determinants of gathered flavour blocks (Sec. 1), with
                  exact (``math.fsum``) summation.
* ``tree``     -- the source-term graph and the greedy dominating set
                  (Sec. 3), in the readings listed in the design notes.
* ``grad``     -- derivatives of the correlator with respect to the weights
                  and the propagator (Jacobi's formula with cofactors).

It shares no code with the GPU path.  Every function is pinned by tests in
``tests/test_oracle.py``, ``tests/test_oracle_tree.py`` and
``tests/test_oracle_grad.py`` against values the
mathematics fixes (exact rational results, closed forms, brute force, an
independent library routine).
"""
from . import det, contract, tree, grad  # noqa: F401
