"""The residual entry point that allocates nothing (hgks_residual_static:
no context, no workspace; the library's static device array per GPU) against
the existing entry point hgks_residual on a context of the same state,
through the C ABI: FP64 to the residual parity bar (1e-12 of each component's
maximum), the mixed path to its own rounding level, on two calls in a row
(the second on a smaller grid, so the array keeps the first call's larger
contents), and the size limit rejected with a message."""
import sys

import numpy as np
import pytest

from paper_2207_01173_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_01173_amd import hgks

    hgks.lib()
    return hgks


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(got, ref):
    axes = tuple(range(1, ref.ndim))
    return np.abs(got - ref).max(axis=axes) / np.maximum(np.abs(ref).max(axis=axes), 1e-300)


def residual_both(hg, p, q, dt, precision):
    """(L, dL) from hgks_residual on a fresh context and from
    hgks_residual_static on a dedicated stream, as numpy arrays."""
    import torch

    s = hg.Solver(p, q, precision=precision)
    L0, dL0 = s.residual(q, dt)
    L0, dL0 = L0.cpu().numpy(), dL0.cpu().numpy()
    s.close()
    cfg = hg.make_config(p, precision)
    qd = torch.as_tensor(np.ascontiguousarray(q), dtype=torch.float64, device="cuda").contiguous()
    L = torch.full_like(qd, float("nan"))
    dL = torch.full_like(qd, float("nan"))
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    hg.hgks_residual_static(cfg, qd.data_ptr(), dt, L.data_ptr(), dL.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    return (L0, dL0), (L.cpu().numpy(), dL.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_residual_matches_context_residual(hg, precision):
    prec = hg.FP64 if precision == "fp64" else hg.MIXED
    cases = [
        ("TGV 32^3 Ma 0.29", W.tgv_params(32, ma=0.29, re=1600.0), None),
        ("smooth random 21x13x17 (smaller, ragged)", W.tgv_params((21, 13, 17), ma=0.3, re=300.0), 5),
        ("channel 16x24x12 (walls, stretched y, force)", W.channel_params((16, 24, 12), ma_b=0.5, re_b=3000.0), "ch"),
    ]
    for name, p, kind in cases:
        if kind is None:
            q = W.tgv_initial(p)
        elif kind == "ch":
            q = W.channel_initial(p, seed=2207)
        else:
            q = W.smooth_random(p, seed=kind)
        dt = 0.004
        (L0, dL0), (L, dL) = residual_both(hg, p, q, dt, prec)
        eL, edL = rel_err(L, L0), rel_err(dL, dL0)
        same = np.array_equal(L, L0) and np.array_equal(dL, dL0)
        say(f"{precision} {name}: L err {eL} dL err {edL} bit-identical {same}")
        assert np.isfinite(L).all() and np.isfinite(dL).all()
        bar = 1e-12 if prec == hg.FP64 else 1e-6
        assert (eL <= bar).all() and (edL <= bar).all(), (name, eL, edL)


def test_static_residual_size_limit(hg):
    import torch

    p = W.tgv_params(37)  # 37^3 FP64 face buffers exceed the static array (36^3 fits)
    cfg = hg.make_config(p)
    q = torch.ones((5, 37, 37, 37), dtype=torch.float64, device="cuda")
    with pytest.raises(hg.HGKSError) as e:
        hg.hgks_residual_static(cfg, q.data_ptr(), 1e-3, q.data_ptr(), q.data_ptr(), 0)
    assert e.value.status == hg.HGKS_E_UNSUPPORTED
    assert "static array" in str(e.value)
    with pytest.raises(hg.HGKSError) as e:
        hg.hgks_residual_static(cfg, q.data_ptr(), -1.0, q.data_ptr(), q.data_ptr(), 0)
    assert e.value.status == hg.HGKS_E_INVALID
