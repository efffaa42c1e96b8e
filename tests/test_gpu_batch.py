"""GPU tests of the batched ensemble (one launch per kernel over all
instances, replayed HIP graph, per-instance CFL time step, autotuned launch
shapes), through the C ABI."""
import os
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


def small_ensemble():
    sizes = [(24, 24, 24), (20, 16, 12), (16, 24, 20), (12, 12, 12), (33, 17, 9)]
    rng = np.random.default_rng(7)
    out = []
    for n in sizes:
        p = W.tgv_params(n, ma=float(rng.uniform(0.1, 0.5)), re=float(rng.uniform(400, 3000)))
        out.append((p, W.tgv_initial(p)))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_batch_members_equal_standalone_runs(hg, tmp_path, precision):
    """Each member of a batched run equals its standalone run bit for bit:
    the same tile functions, per-face arithmetic and per-instance CFL step
    (whole-code FP32: the same rounding of the state into the FP32 working
    copy and back around each call)."""
    os.environ["HGKS_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    prec = {"fp64": hg.FP64, "mixed": hg.MIXED, "fp32": hg.FP32}[precision]
    ens = small_ensemble()
    b = hg.Batch([p for p, _ in ens], [q for _, q in ens], precision=prec)
    info = b.info()
    say("batch info", info)
    assert info["instances"] == len(ens) and info["flux_tile_x"] in (16, 32) and info["tune_source"] == 1
    assert info["group_mib"] in (0, 64, 128, 256) and 1 <= info["groups"] <= len(ens)
    b.step(3)
    for i, (p, q0) in enumerate(ens):
        s = hg.Solver(p, q0, precision=prec)
        s.step(3, 0.0)
        ref = s.state()
        st = s.stats()
        s.close()
        got = b.state(i)
        bs = b.stats(i)
        say(f"  member {i} {p['n']} max diff {np.abs(got - ref).max():.3e} dt {bs['dt_last']:.6e} {st['dt_last']:.6e}")
        np.testing.assert_array_equal(got, ref)
        assert bs["dt_last"] == st["dt_last"] and bs["steps"] == 3
    b.close()
    # the same ensemble again reads the tuned shapes from the cache file
    b2 = hg.Batch([p for p, _ in ens], [q for _, q in ens], precision=prec)
    assert b2.info()["tune_source"] == 2
    for k in ("flux_tile_x", "group_mib", "groups", "flux_tiles"):
        assert b2.info()[k] == info[k]
    b2.close()
    del os.environ["HGKS_TUNE_CACHE"]


def test_batch_replays_advance_time(hg):
    ens = small_ensemble()[:2]
    b = hg.Batch([p for p, _ in ens], [q for _, q in ens])
    b.step(2)
    t2 = [b.stats(i)["t"] for i in range(2)]
    b.step(3)
    t5 = [b.stats(i)["t"] for i in range(2)]
    assert all(t5[i] > t2[i] > 0 for i in range(2))
    assert [b.stats(i)["steps"] for i in range(2)] == [5, 5]
    b.close()


def test_batch_rejects_invalid_member(hg):
    ens = small_ensemble()[:2]
    cfgs = [hg.make_config(p) for p, _ in ens]
    cfgs[1].gamma = 0.5
    with pytest.raises(hg.HGKSError) as e:
        hg.hgks_batch_workspace_size(cfgs)
    assert e.value.status == hg.HGKS_E_INVALID
