"""Runs the CPU oracle over chunks of source terms in worker processes
(orchestration only: every number comes from ``oracle.contract``)."""
from __future__ import annotations

import math
import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from oracle import contract as oc


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunk(args):
    S, src, snk, nf, w_src, w_snk, t, lo, hi = args
    d = oc.slice_pair_dets(S[t:t + 1], src[lo:hi], snk, nf, 0)
    z = oc.weighted_terms(d, w_src[lo:hi], w_snk)
    return (math.fsum(z.real.ravel().tolist()), math.fsum(z.imag.ravel().tolist()),
            math.fsum(np.abs(z).ravel().tolist()))


def correlator(S, src, snk, nf, w_src, w_snk, slices, n_workers=None, rows_per_chunk=None):
    """(C, A) of ``oracle.contract.correlator`` for the given slices, with
    the source terms split across processes."""
    n_workers = n_workers or workers()
    n_src = len(src)
    if rows_per_chunk is None:
        rows_per_chunk = max(1, math.ceil(n_src / (4 * n_workers)))
    jobs = []
    for t in slices:
        for lo in range(0, n_src, rows_per_chunk):
            jobs.append((S, src, snk, nf, w_src, w_snk, t, lo, min(n_src, lo + rows_per_chunk)))
    if n_workers == 1:
        res = [_chunk(j) for j in jobs]
    else:
        # workers only run numpy; fork keeps them free of any GPU state
        with ProcessPoolExecutor(n_workers, mp_context=multiprocessing.get_context("fork")) as ex:
            res = list(ex.map(_chunk, jobs))
    C = np.zeros(len(slices), dtype=np.complex128)
    A = np.zeros(len(slices))
    k = 0
    for si, t in enumerate(slices):
        parts = []
        while k < len(jobs) and jobs[k][6] == t:
            parts.append(res[k])
            k += 1
        C[si] = complex(math.fsum(p[0] for p in parts), math.fsum(p[1] for p in parts))
        A[si] = math.fsum(p[2] for p in parts)
    return C, A
