"""The FP64 FMA-rate probe (a measurement aid of the benchmark's roofline)
computes what it states, through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_fma_probe_values():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_01173_amd import hgks

    blocks, iters = 3, 50
    out = torch.full((blocks * 256,), float("nan"), dtype=torch.float64, device="cuda")
    hgks.hgks_fma_probe(out.data_ptr(), blocks, iters, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(blocks, 256)
    t = np.arange(256, dtype=np.float64)
    x = np.stack([1.0 + 1e-3 * t + j for j in range(8)])
    for _ in range(iters):
        x = x * 0.999999 + 1e-7
    ref = x.sum(axis=0)
    for b in range(blocks):
        np.testing.assert_allclose(got[b], ref, rtol=1e-14)
    with pytest.raises(hgks.HGKSError):
        hgks.hgks_fma_probe(out.data_ptr(), 0, iters, 0)
