"""The single-instance step captured in a HIP graph (hgks_step on a created
stream) against the same steps launched kernel by kernel (profiling on, so
no graph), through the C ABI: bit-identical states after every block of
replays, with the program's own eager work (statistics, reads, a residual)
between the replays, for every precision, a fixed and a CFL time step, and
the mass-flux controller."""
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


CASES = {
    "tgv_fp64": (lambda: W.tgv_params((20, 16, 12), ma=0.3, re=800.0), "tgv", "FP64"),
    "tgv_mixed": (lambda: W.tgv_params((20, 16, 12), ma=0.3, re=800.0), "tgv", "MIXED"),
    "tgv_fp32": (lambda: W.tgv_params((20, 16, 12), ma=0.3, re=800.0), "tgv", "FP32"),
    "channel_mass_flux": (lambda: dict(W.channel_params((16, 24, 12), ma_b=0.5, re_b=3000.0),
                                       mass_flux_control=True), "channel", "FP64"),
}


@pytest.mark.parametrize("case", list(CASES))
def test_graph_step_matches_plain_launches(hg, case):
    import torch

    make, kind, prec_name = CASES[case]
    p = make()
    q0 = W.tgv_initial(p) if kind == "tgv" else W.channel_initial(p, seed=2207)
    prec = getattr(hg, prec_name)
    sg = hg.Solver(p, q0, precision=prec, stream=torch.cuda.Stream())  # created stream: graph replays
    sp = hg.Solver(p, q0, precision=prec, stream=torch.cuda.Stream())
    hg.hgks_profile(sp.ctx, True)  # events between launches: kernel by kernel
    dt = 0.5 * sg.dt()
    for block, (k, dtf) in enumerate([(3, 0.0), (2, dt), (1, 0.0), (4, 0.0), (2, dt)]):
        sg.step(k, dtf)
        sp.step(k, dtf)
        hg.hgks_profile_read(sp.ctx)
        a, b = sg.state(), sp.state()
        sa, sb = sg.stats(), sp.stats()
        say(f"{case} block {block}: {k} steps dt_fixed {dtf:.3e}: max |diff| {np.abs(a - b).max():.3e} "
            f"t {sa['t']:.6e} {sb['t']:.6e}")
        np.testing.assert_array_equal(a, b)
        assert (sa["t"], sa["steps"], sa["dt_last"], sa["body_force_x"]) == \
               (sb["t"], sb["steps"], sb["dt_last"], sb["body_force_x"])
        # eager work on the graph solver's stream between replays
        L, dL = sg.residual(sg.q, dt)
        assert torch.isfinite(L).all() and torch.isfinite(dL).all()
    sg.close()
    sp.close()
