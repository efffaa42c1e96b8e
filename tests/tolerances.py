"""Error bounds of the GPU-vs-oracle comparisons derived from the arithmetic."""
import numpy as np


def residual_tolerances(p, q, dt, K=1000.0):
    """Absolute bounds for |GPU - oracle| in L and dL/dt from the arithmetic.

    Both sides compute the face integrals I(dt) ~ dt |F| to relative rounding
    error of order eps, in different operation orders (FMA contraction,
    summation order, libm).  L = -sum dF/h then differs by ~eps |F| / h, and
    dF/dt = 4 (I(dt) - 2 I(dt/2)) / dt^2 cancels to O(dt^2), so its difference
    is ~12 eps |F| / dt and dL/dt's is that over h.  K (a few hundred to a
    thousand rounding steps per face) is the margin; any real defect shows up
    many orders of magnitude above these bounds."""
    eps = np.finfo(np.float64).eps
    rho = q[0]
    u2 = (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho
    pres = (p["gamma"] - 1.0) * (q[4] - 0.5 * u2)
    speed = np.sqrt(u2 / rho)
    fscale = float((pres + u2).max() + (speed * (q[4] + pres)).max() + np.abs(q[1:4]).max())
    hmin = min((p["hi"][d] - p["lo"][d]) / p["n"][d] for d in range(3))
    return K * eps * fscale / hmin, 12.0 * K * eps * fscale / (dt * hmin)
