"""Seeded synthetic workloads of the paper (Sec. 4): initial conditions and
their gas parameters.

This module holds no arithmetic of the scheme itself (no reconstruction, flux
or update): only analytic initial fields, the equation of state that turns
primitive fields into conserved variables, and seeded random draws.  Both the
HIP path's tests and the oracle's tests take their inputs from here.

Layout of every field: float64 SoA array q[5, nz, ny, nx] of
(rho, rho U, rho V, rho W, rho E), x fastest.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4


def conserved(rho, U, V, W, p, gamma=GAMMA):
    """Primitive -> conserved for a perfect gas: rho E = p/(gamma-1) + rho|U|^2/2."""
    q = np.empty((5,) + np.shape(rho), dtype=np.float64)
    q[0] = rho
    q[1] = rho * U
    q[2] = rho * V
    q[3] = rho * W
    q[4] = p / (gamma - 1.0) + 0.5 * rho * (U * U + V * V + W * W)
    return q


def cell_centres(n, lo, hi):
    h = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * h


# ---------------------------------------------------------------------------
# Taylor-Green vortex (Sec. 4.1)
# ---------------------------------------------------------------------------

def tgv_params(n, ma=0.1, re=1600.0, pr=0.72, lo=0.0, hi=2.0 * math.pi, cfl=0.5, rho0=1.0, v0=1.0, L=1.0):
    """Gas and grid parameters of a TGV case.  p0 from Ma = V0/c0 with
    c0 = sqrt(gamma p0/rho0); constant viscosity mu = rho0 V0 L / Re; T = p/rho."""
    if np.isscalar(n):
        n = (int(n),) * 3
    p0 = rho0 * v0 * v0 / (GAMMA * ma * ma)
    return {
        "n": tuple(int(x) for x in n),
        "lo": (lo,) * 3,
        "hi": (hi,) * 3,
        "bc": (0, 0, 0),
        "y_stretch": 0.0,
        "gamma": GAMMA,
        "prandtl": pr,
        "mu_ref": rho0 * v0 * L / re,
        "T_ref": p0 / rho0,
        "mu_exp": 0.0,
        "T_wall": p0 / rho0,
        "body_force": (0.0, 0.0, 0.0),
        "cfl": cfl,
        # workload metadata (not read by the solvers)
        "p0": p0,
        "rho0": rho0,
        "v0": v0,
        "ma": ma,
        "re": re,
    }


def tgv_initial(p):
    """Point values at cell centres (uniform temperature T0 = p0/rho0):
    U = V0 sin x cos y cos z, V = -V0 cos x sin y cos z, W = 0,
    p = p0 + rho0 V0^2/16 (cos 2x + cos 2y)(cos 2z + 2), rho = p / T0."""
    nx, ny, nz = p["n"]
    # separable factors on 1-D axes (broadcast to [z][y][x] by the products)
    x = cell_centres(nx, p["lo"][0], p["hi"][0])[None, None, :]
    y = cell_centres(ny, p["lo"][1], p["hi"][1])[None, :, None]
    z = cell_centres(nz, p["lo"][2], p["hi"][2])[:, None, None]
    v0, rho0, p0 = p["v0"], p["rho0"], p["p0"]
    U = v0 * np.sin(x) * np.cos(y) * np.cos(z)
    V = -v0 * np.cos(x) * np.sin(y) * np.cos(z)
    W = np.zeros_like(U)
    pr = p0 + rho0 * v0 * v0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    rho = pr / (p0 / rho0)
    return np.ascontiguousarray(conserved(rho, U, V, W, pr, p["gamma"]))


# ---------------------------------------------------------------------------
# Advected density wave (Euler, tau = 0): exact solution for convergence
# ---------------------------------------------------------------------------

def density_wave_params(n, cfl=0.5):
    if np.isscalar(n):
        n = (int(n),) * 3
    return {
        "n": tuple(int(x) for x in n), "lo": (0.0,) * 3, "hi": (2.0,) * 3, "bc": (0, 0, 0),
        "y_stretch": 0.0, "gamma": GAMMA, "prandtl": 1.0, "mu_ref": 0.0, "T_ref": 1.0,
        "mu_exp": 0.0, "T_wall": 1.0, "body_force": (0.0, 0.0, 0.0), "cfl": cfl,
    }


def density_wave_cell_average(p, t):
    """Exact cell averages of rho = 1 + 0.2 sin(pi (x + y + z - 3t)) with
    U = V = W = 1, p = 1 on a uniform grid: each axis contributes the factor
    sin(pi h/2)/(pi h/2) to the average of the sine."""
    nx, ny, nz = p["n"]
    x = cell_centres(nx, p["lo"][0], p["hi"][0])
    y = cell_centres(ny, p["lo"][1], p["hi"][1])
    z = cell_centres(nz, p["lo"][2], p["hi"][2])
    h = [(p["hi"][d] - p["lo"][d]) / p["n"][d] for d in range(3)]
    fac = 1.0
    for hd in h:
        a = math.pi * hd / 2.0
        fac *= math.sin(a) / a
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return 1.0 + 0.2 * fac * np.sin(math.pi * (X + Y + Z - 3.0 * t))


def density_wave_initial(p, t=0.0):
    rho = density_wave_cell_average(p, t)
    one = np.ones_like(rho)
    return np.ascontiguousarray(conserved(rho, one, one, one, one, p["gamma"]))


# ---------------------------------------------------------------------------
# Compressible channel (Sec. 4.2), constant body force
# ---------------------------------------------------------------------------

def channel_params(n=(128, 128, 128), ma_b=0.5, re_b=3000.0, pr=0.7, y_stretch=2.0, force=None, cfl=0.5):
    """Domain 2 pi x 2 x pi, walls at y = -1, 1, U_b = rho_b = h = 1.
    mu_w = rho_b U_b h / Re_b, T_w from Ma_b = U_b / sqrt(gamma T_w),
    mu = mu_w (T/T_w)^0.7.  Constant streamwise force f (default from Dean's
    skin-friction correlation C_f = 0.073 Re_2h^-1/4: f = tau_w/(rho_b h))."""
    if np.isscalar(n):
        n = (int(n),) * 3
    T_w = 1.0 / (GAMMA * ma_b * ma_b)
    if force is None:
        cf = 0.073 * (2.0 * re_b) ** (-0.25)
        force = 0.5 * cf  # tau_w = Cf rho_b U_b^2 / 2, f = tau_w / (rho_b h)
    return {
        "n": tuple(int(x) for x in n), "lo": (0.0, -1.0, 0.0), "hi": (2.0 * math.pi, 1.0, math.pi),
        "bc": (0, 1, 0), "y_stretch": y_stretch, "gamma": GAMMA, "prandtl": pr,
        "mu_ref": 1.0 / re_b, "T_ref": T_w, "mu_exp": 0.7, "T_wall": T_w,
        "body_force": (force, 0.0, 0.0), "cfl": cfl, "rho0": 1.0, "ma": ma_b, "re": re_b,
    }


def channel_y_centres(p):
    """Cell-centre y of the tanh-stretched wall-normal axis (Sec. 4.2 map)."""
    ny = p["n"][1]
    lo, hi, b = p["lo"][1], p["hi"][1], p["y_stretch"]
    xi = (np.arange(ny) + 0.5) / ny
    if b > 0:
        return lo + 0.5 * (hi - lo) * (1.0 + np.tanh(b * (2.0 * xi - 1.0)) / math.tanh(b))
    return lo + (hi - lo) * xi


def channel_initial(p, seed=2207, amp=0.1):
    """Laminar Poiseuille U = 1.5 U_b (1 - y^2) plus uniform noise in
    [-amp, amp] U_b on U, V, W per cell (numpy PCG64), rho = 1, T = T_w."""
    nx, ny, nz = p["n"]
    y = channel_y_centres(p)
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.uniform(-amp, amp, size=(3, nz, ny, nx))
    U = 1.5 * (1.0 - y * y)[None, :, None] + noise[0]
    V = noise[1]
    W = noise[2]
    rho = np.ones((nz, ny, nx))
    pr = rho * p["T_wall"]
    return np.ascontiguousarray(conserved(rho, U, V, W, pr, p["gamma"]))


# ---------------------------------------------------------------------------
# Random smooth fields for kernel parity tests
# ---------------------------------------------------------------------------

def smooth_random(p, seed=1, modes=3, amp=0.05, rho_mean=1.0, p_mean=1.0, u_amp=0.3):
    """A smooth periodic random state: a few low Fourier modes per variable."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = p["n"]
    x = cell_centres(nx, p["lo"][0], p["hi"][0])
    y = cell_centres(ny, p["lo"][1], p["hi"][1])
    z = cell_centres(nz, p["lo"][2], p["hi"][2])
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    L = [p["hi"][d] - p["lo"][d] for d in range(3)]

    def field():
        f = np.zeros_like(X)
        for _ in range(modes):
            k = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            a = rng.uniform(-1, 1)
            f += a * np.sin(2 * math.pi * (k[0] * X / L[0] + k[1] * Y / L[1] + k[2] * Z / L[2]) + ph)
        return f

    rho = rho_mean * (1.0 + amp * field())
    U = u_amp * field()
    V = u_amp * field()
    W = u_amp * field()
    pr = p_mean * (1.0 + amp * field())
    return np.ascontiguousarray(conserved(rho, U, V, W, pr, p.get("gamma", GAMMA)))


# ---------------------------------------------------------------------------
# Batched ensemble of TGV instances
# ---------------------------------------------------------------------------

def tgv_ensemble(count=64, sizes=(24, 32, 48, 64, 96), seed=20220703, ma=(0.1, 0.5), re=(400.0, 3000.0)):
    """Instances with grid N drawn from sizes, Ma ~ U[ma], Re ~ U[re] (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        m = float(rng.uniform(*ma))
        r = float(rng.uniform(*re))
        out.append(tgv_params(n, ma=m, re=r))
    return out
