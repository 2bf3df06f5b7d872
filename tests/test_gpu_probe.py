"""GPU: the FP64 FMA probe (mhc_probe_fma64) computes what its header
states: each thread's 16 chains a <- a * b + c, summed, against the closed
form b^n a_0 + c (1 - b^n) / (1 - b)."""
import numpy as np
import pytest
import torch

from paper_1411_3691_amd import mhc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_blocks,iters", [(1, 1), (3, 100), (4, 1000)])
def test_probe_matches_closed_form(n_blocks, iters):
    out = torch.full((n_blocks * 256,), np.nan, dtype=torch.float64, device="cuda")
    flop = mhc.probe_fma64(out, iters)
    torch.cuda.synchronize()
    assert flop == n_blocks * 256 * iters * 32
    got = out.cpu().numpy()
    b = 1.0 - 2.0 ** -20
    tid = np.arange(n_blocks * 256)
    c = 2.0 ** -30 * (1 + (tid % 256 & 7))
    a0 = 1.0 + np.arange(16) / 1024.0
    bn = b ** iters
    want = (bn * a0[None, :] + (c * (1 - bn) / (1 - b))[:, None]).sum(axis=1)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)


def test_probe_refuses_bad_shapes():
    with pytest.raises(ValueError):
        mhc.probe_fma64(torch.empty(100, dtype=torch.float64, device="cuda"), 10)
    with pytest.raises(ValueError):
        mhc.probe_fma64(torch.empty(256, dtype=torch.float32, device="cuda"), 10)


@pytest.mark.parametrize("with_valu", [False, True])
def test_mfma_probe_accumulates_linearly(with_valu):
    # each round adds the same 16 x 16 x 4 products to the accumulators, so
    # (out(2n) - chains(2n)) = 2 (out(n) - chains(n)); without the vector
    # chains those stay at their start values
    n = 500
    outs = []
    for it in (n, 2 * n):
        out = torch.full((2 * 256,), np.nan, dtype=torch.float64, device="cuda")
        flop = mhc.probe_mfma64(out, it, with_valu)
        torch.cuda.synchronize()
        assert flop == 2 * 4 * it * 8192 + (2 * 256 * it * 32 if with_valu else 0)
        outs.append(out.cpu().numpy())
    b = 1.0 - 2.0 ** -20
    tid = np.arange(2 * 256)
    c = 2.0 ** -30 * (1 + (tid % 256 & 7))
    a0 = 1.0 + np.arange(16) / 1024.0

    def chains(it):
        if not with_valu:
            return np.full(tid.shape, a0.sum())
        bn = b ** it
        return (bn * a0[None, :] + (c * (1 - bn) / (1 - b))[:, None]).sum(axis=1)

    m1, m2 = outs[0] - chains(n), outs[1] - chains(2 * n)
    assert np.all(np.isfinite(outs[0])) and np.all(np.abs(m1) > 0)
    np.testing.assert_allclose(m2, 2 * m1, rtol=1e-12, atol=0)
