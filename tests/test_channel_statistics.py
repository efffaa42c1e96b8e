"""The channel statistics (paper_2207_01173_amd.channel) on a manufactured
field with closed-form answers (CPU, torch)."""
import math

import numpy as np
import pytest

from paper_2207_01173_amd import workloads as W


def test_channel_statistics_manufactured_field():
    torch = pytest.importorskip("torch")
    from paper_2207_01173_amd.channel import channel_statistics

    p = W.channel_params((16, 12, 8), ma_b=0.5, re_b=3000.0, y_stretch=0.0)
    nx, ny, nz = p["n"]
    x = (np.arange(nx) + 0.5) / nx * p["hi"][0]
    y = W.channel_y_centres(p)
    z = (np.arange(nz) + 0.5) / nz * p["hi"][2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    a, b, rho0, T0 = 0.1, 0.05, 1.3, p["T_wall"]
    kx = 2.0 * math.pi / p["hi"][0]
    U = 1.0 - Y * Y + a * np.sin(kx * X)       # laminar profile + a streamwise wave
    V = b * np.sin(kx * X)                      # in phase: <u'v'> = a b / 2
    Wv = np.zeros_like(U)
    rho = np.full_like(U, rho0)
    q = torch.as_tensor(np.ascontiguousarray(W.conserved(rho, U, V, Wv, rho0 * T0, p["gamma"])))
    st = channel_statistics(q, p, y)
    half = len(st["y"])
    assert half == ny // 2
    np.testing.assert_allclose(st["u_rms"], a / math.sqrt(2.0), rtol=1e-12)
    np.testing.assert_allclose(st["v_rms"], b / math.sqrt(2.0), rtol=1e-12)
    np.testing.assert_allclose(st["w_rms"], 0.0, atol=1e-15)
    np.testing.assert_allclose(st["uv"], a * b / 2.0, rtol=1e-12)
    np.testing.assert_allclose(st["T"], T0, rtol=1e-12)
    np.testing.assert_allclose(st["T_rms"], 0.0, atol=1e-10)
    c = math.sqrt(p["gamma"] * T0)
    np.testing.assert_allclose(st["M_t"], math.sqrt((a * a + b * b) / 2.0) / c, rtol=1e-12)
    # U = 1 - y^2 near y = -1 is 2 d - d^2: the one-sided quadratic is exact, dU/dy = 2
    assert st["tau_w"] == pytest.approx(2.0 * p["mu_ref"], rel=1e-10)
    assert st["rho_w"] == pytest.approx(rho0, rel=1e-12)
    u_tau = math.sqrt(2.0 * p["mu_ref"] / rho0)
    assert st["u_tau"] == pytest.approx(u_tau, rel=1e-10)
    assert st["Re_tau"] == pytest.approx(rho0 * u_tau / p["mu_ref"], rel=1e-10)
    # uniform density: the van Driest velocity is U+ itself
    np.testing.assert_allclose(st["U_vd_plus"], st["U_plus"], rtol=1e-12)
    np.testing.assert_allclose(st["y_plus"], (y[:half] + 1.0) * u_tau * rho0 / p["mu_ref"], rtol=1e-10)
