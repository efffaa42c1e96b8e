"""Independent reference pieces for pinning the oracle's kinetic arithmetic.

Nothing here calls the oracle.  One-dimensional Maxwellian moments come from
adaptive numerical quadrature (scipy), the internal degrees of freedom from K
independent one-dimensional Gaussians, and moments of polynomials from an
explicit monomial expansion; linear systems are solved with numpy.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from scipy import integrate


def _quad(f, a, b):
    v, _ = integrate.quad(f, a, b, epsabs=0.0, epsrel=2e-14, limit=400)
    return v


@functools.lru_cache(maxsize=None)
def gauss_moments_1d(mean: float, lam: float, side: int, nmax: int = 8):
    """<c^n> for the normalised 1D Gaussian sqrt(lam/pi) exp(-lam (c-mean)^2),
    over the whole line (side 0), c > 0 (side +1) or c < 0 (side -1)."""
    norm = math.sqrt(lam / math.pi)
    width = 12.0 / math.sqrt(lam)
    out = []
    for n in range(nmax + 1):
        f = lambda c, n=n: c ** n * norm * math.exp(-lam * (c - mean) ** 2)
        lo, hi = mean - width, mean + width
        if side == 0:
            pts = sorted({lo, mean, hi})
            v = sum(_quad(f, pts[i], pts[i + 1]) for i in range(len(pts) - 1))
        elif side > 0:
            a = max(0.0, lo)
            v = _quad(f, 0.0, a) if a > 0 else 0.0
            v += _quad(f, a, max(a, hi)) if hi > a else 0.0
        else:
            b = min(0.0, hi)
            v = _quad(f, b, 0.0) if b < 0 else 0.0
            v += _quad(f, min(lo, b), b) if lo < b else 0.0
        out.append(v)
    return tuple(out)


@functools.lru_cache(maxsize=None)
def xi_moments(lam: float, K: int):
    """<(xi^2)^e>, e = 0, 1, 2, with xi^2 the sum of K independent squares."""
    m = gauss_moments_1d(0.0, lam, 0, 4)
    m2, m4 = m[2], m[4]
    return (1.0, K * m2, K * m4 + K * (K - 1) * m2 * m2)


class Table:
    """Moments of one Maxwellian (normalised by density); side applies to u."""

    def __init__(self, rho, U, V, W, lam, K=2, side=0):
        self.rho, self.U, self.V, self.W, self.lam, self.K = rho, U, V, W, lam, K
        self.mu = gauss_moments_1d(float(U), float(lam), side)
        self.mv = gauss_moments_1d(float(V), float(lam), 0)
        self.mw = gauss_moments_1d(float(W), float(lam), 0)
        self.mx = xi_moments(float(lam), int(K))

    def mono(self, a, b, c, e):
        return self.mu[a] * self.mv[b] * self.mw[c] * self.mx[e]

    def of(self, poly: dict) -> float:
        return sum(cf * self.mono(*k) for k, cf in poly.items())


# polynomials in (u, v, w, xi^2): dict {(a, b, c, e): coefficient}

def pmul(p, q):
    r = {}
    for k1, c1 in p.items():
        for k2, c2 in q.items():
            k = tuple(x + y for x, y in zip(k1, k2))
            r[k] = r.get(k, 0.0) + c1 * c2
    return r


def padd(*ps):
    r = {}
    for p in ps:
        for k, c in p.items():
            r[k] = r.get(k, 0.0) + c
    return r


def pscale(p, s):
    return {k: c * s for k, c in p.items()}


ONE = {(0, 0, 0, 0): 1.0}
U_ = {(1, 0, 0, 0): 1.0}
V_ = {(0, 1, 0, 0): 1.0}
W_ = {(0, 0, 1, 0): 1.0}
XI2 = {(0, 0, 0, 1): 1.0}
PSI = [ONE, U_, V_, W_, {(2, 0, 0, 0): 0.5, (0, 2, 0, 0): 0.5, (0, 0, 2, 0): 0.5, (0, 0, 0, 1): 0.5}]
S_DIR = [U_, V_, W_]


def dot_psi(a):
    return padd(*[pscale(PSI[i], float(a[i])) for i in range(5)])


def vec(tab: Table, poly: dict) -> np.ndarray:
    """<poly psi> as a 5-vector."""
    return np.array([tab.of(pmul(poly, PSI[m])) for m in range(5)])


def gram(tab: Table) -> np.ndarray:
    return np.array([[tab.of(pmul(PSI[i], PSI[j])) for j in range(5)] for i in range(5)])


def primitive(q, gamma=1.4):
    rho = q[0]
    U, V, W = q[1] / rho, q[2] / rho, q[3] / rho
    p = (gamma - 1.0) * (q[4] - 0.5 * rho * (U * U + V * V + W * W))
    return rho, U, V, W, rho / (2.0 * p)


def euler_flux(q, gamma=1.4):
    rho, U, V, W, lam = primitive(q, gamma)
    p = rho / (2 * lam)
    return np.array([rho * U, rho * U * U + p, rho * U * V, rho * U * W, U * (q[4] + p)])


def time_factor_integrals(tau, delta):
    """Integrals over [0, delta] of the six time factors of the BGK solution,
    by quadrature (tau > 0)."""
    fs = [
        lambda t: 1.0 - math.exp(-t / tau),
        lambda t: (t + tau) * math.exp(-t / tau) - tau,
        lambda t: t - tau + tau * math.exp(-t / tau),
        lambda t: math.exp(-t / tau),
        lambda t: -(t + tau) * math.exp(-t / tau),
        lambda t: -tau * math.exp(-t / tau),
    ]
    return np.array([_quad(f, 0.0, delta) for f in fs])
