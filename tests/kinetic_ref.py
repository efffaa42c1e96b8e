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


def equilibrium_and_slopes(ql, qr, dql, dqr, dq0n, K=2, gamma=1.4):
    """Interface equilibrium and every micro-slope of the BGK solution at one
    Gauss point, by quadrature tables and dense solves only:
    Q0 from the compatibility condition (half-space integrals of the left and
    right Maxwellians), spatial slopes a from <(a . psi) psi> = dQ / rho,
    tangential slopes of Q0 as the derivative of the compatibility map,
    time slopes A from <a_n u + a_t1 v + a_t2 w + A> = 0 (full moments)."""
    pl, pr = primitive(ql, gamma), primitive(qr, gamma)
    tl_h, tr_h = Table(*pl, K=K, side=1), Table(*pr, K=K, side=-1)
    tl_f, tr_f = Table(*pl, K=K, side=0), Table(*pr, K=K, side=0)
    q0 = pl[0] * vec(tl_h, ONE) + pr[0] * vec(tr_h, ONE)
    p0 = primitive(q0, gamma)
    t0 = Table(*p0, K=K, side=0)
    al = [np.linalg.solve(gram(tl_f), np.asarray(dql[d], float) / pl[0]) for d in range(3)]
    ar = [np.linalg.solve(gram(tr_f), np.asarray(dqr[d], float) / pr[0]) for d in range(3)]
    dq0 = [np.asarray(dq0n, float)]
    for d in (1, 2):
        dq0.append(pl[0] * vec(tl_h, dot_psi(al[d])) + pr[0] * vec(tr_h, dot_psi(ar[d])))
    a0 = [np.linalg.solve(gram(t0), dq0[d] / p0[0]) for d in range(3)]

    def time_slope(tab, a):
        rhs = -vec(tab, padd(*[pmul(S_DIR[d], dot_psi(a[d])) for d in range(3)]))
        return np.linalg.solve(gram(tab), rhs)

    return {
        "q0": q0, "p0": p0, "pl": pl, "pr": pr,
        "t0": t0, "tl_h": tl_h, "tr_h": tr_h,
        "a0": a0, "al": al, "ar": ar,
        "A0": time_slope(t0, a0), "Al": time_slope(tl_f, al), "Ar": time_slope(tr_f, ar),
    }


def bgk_flux(ql, qr, dql, dqr, dq0n, delta, mu_ref, T_ref=1.0, mu_exp=0.0, Pr=1.0, K=2, gamma=1.4):
    """Time-integrated flux int_0^delta int u psi f at one Gauss point of the
    BGK solution of Sec. 2, Eq. (flux), evaluated term by term:

      f = (1 - e) g0 + ((t + tau) e - tau) (sum_d s_d a0_d . psi) g0 + (t - tau + tau e) (A0 . psi) g0
        + e [1 - (t + tau) (sum_d s_d al_d . psi) - tau (Al . psi)] g_l H(u)
        + e [1 - (t + tau) (sum_d s_d ar_d . psi) - tau (Ar . psi)] g_r (1 - H(u)),

    e = exp(-t / tau), s = (u, v, w), each time factor integrated over
    [0, delta] by quadrature and each velocity moment an explicit polynomial
    expansion on quadrature moment tables.  tau = mu(T0) / p0 from the
    equilibrium state.  With Pr != 1 the energy flux gains (1/Pr - 1) q, q
    the same time integral of int c_n (|c|^2 + xi^2)/2 f, c = (u, v, w) - U0
    (the heat flux in the frame of the equilibrium velocity).  Shares nothing
    with the oracle."""
    s = equilibrium_and_slopes(ql, qr, dql, dqr, dq0n, K=K, gamma=gamma)
    rho0, U0, lam0 = s["p0"][0], s["p0"][1:4], s["p0"][4]
    T0 = 1.0 / (2.0 * lam0)
    mu = mu_ref * (T0 / T_ref) ** mu_exp if mu_exp != 0.0 else mu_ref
    tau = mu / (rho0 * T0)
    C = time_factor_integrals(tau, delta)

    def transport(a):
        return padd(*[pmul(S_DIR[d], dot_psi(a[d])) for d in range(3)])

    terms = []
    for rho, tab, a, A, c in ((rho0, s["t0"], s["a0"], s["A0"], C[0:3]),
                              (s["pl"][0], s["tl_h"], s["al"], s["Al"], C[3:6]),
                              (s["pr"][0], s["tr_h"], s["ar"], s["Ar"], C[3:6])):
        terms += [(rho * c[0], tab, ONE), (rho * c[1], tab, transport(a)), (rho * c[2], tab, dot_psi(A))]
    F = sum(w * vec(tab, pmul(U_, poly)) for w, tab, poly in terms)
    cv = [padd(S_DIR[d], pscale(ONE, -U0[d])) for d in range(3)]
    energy = pscale(padd(pmul(cv[0], cv[0]), pmul(cv[1], cv[1]), pmul(cv[2], cv[2]), XI2), 0.5)
    heat = pmul(cv[0], energy)
    q = sum(w * tab.of(pmul(heat, poly)) for w, tab, poly in terms)
    F = np.array(F, dtype=float)
    F[4] += (1.0 / Pr - 1.0) * q
    return F, tau
