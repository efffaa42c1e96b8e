"""ctypes binding of the HGKS oracle (plain FP64 CPU implementation).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark import this module; the product library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hgks_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

CXXFLAGS = ["-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-std=c++17"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", *CXXFLAGS, "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class Config(ctypes.Structure):
    """Mirror of the oracle's own configuration struct."""

    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", ctypes.c_int32 * 3),
        ("y_stretch", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu_ref", ctypes.c_double),
        ("T_ref", ctypes.c_double),
        ("mu_exp", ctypes.c_double),
        ("T_wall", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("cfl", ctypes.c_double),
        ("flags", ctypes.c_int32),
    ]


def make_config(p: dict) -> Config:
    c = Config()
    for k in range(3):
        c.n[k] = int(p["n"][k])
        c.lo[k] = float(p["lo"][k])
        c.hi[k] = float(p["hi"][k])
        c.bc[k] = int(p.get("bc", (0, 0, 0))[k])
        c.body_force[k] = float(p.get("body_force", (0.0, 0.0, 0.0))[k])
    c.y_stretch = float(p.get("y_stretch", 0.0))
    c.gamma = float(p.get("gamma", 1.4))
    c.prandtl = float(p.get("prandtl", 1.0))
    c.mu_ref = float(p.get("mu_ref", 0.0))
    c.T_ref = float(p.get("T_ref", 1.0))
    c.mu_exp = float(p.get("mu_exp", 0.0))
    c.T_wall = float(p.get("T_wall", 1.0))
    c.cfl = float(p.get("cfl", 0.5))
    c.flags = 1 if p.get("mass_flux_control") else 0
    return c


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        d, i, P = ctypes.c_double, ctypes.c_int, ctypes.POINTER(Config)
        L.hgo_set_threads.argtypes = [i]
        L.hgo_get_threads.restype = i
        L.hgo_moments.argtypes = [_D, d, i, _D]
        L.hgo_mom_apsi.argtypes = [_D, d, i, _D, i, i, i, _D]
        L.hgo_mom_psi.argtypes = [_D, d, i, i, i, i, i, _D]
        L.hgo_slope_solve.argtypes = [_D, d, _D, _D]
        L.hgo_time_slope.argtypes = [_D, d, _D, _D]
        L.hgo_time_coefficients.argtypes = [d, d, _D]
        L.hgo_q0.argtypes = [_D, _D, d, _D]
        L.hgo_gp_flux.argtypes = [_D, _D, _D, _D, _D, d, d, _D, _D]
        L.hgo_wenoz.argtypes = [_D, i, _D]
        L.hgo_linear_value.argtypes = [_D, i]
        L.hgo_linear_value.restype = d
        L.hgo_linear_weights.argtypes = [i, _D]
        L.hgo_derivative_linear_weights.argtypes = [i, _D]
        L.hgo_candidates.argtypes = [_D, d, _D, _D]
        L.hgo_weno_linear.argtypes = [_D, i, _D]
        L.hgo_normal_sweep.argtypes = [_D, _D]
        L.hgo_residual.argtypes = [P, _D, d, _D, _D]
        L.hgo_residual_at.argtypes = [P, _D, d, i, ctypes.POINTER(ctypes.c_int), _D, _D]
        L.hgo_face_flux.argtypes = [P, _D, d, i, i, i, i, _D]
        L.hgo_cfl_dt.argtypes = [P, _D]
        L.hgo_cfl_dt.restype = d
        L.hgo_step.argtypes = [P, _D, i, d]
        L.hgo_step.restype = d
        L.hgo_step_force.argtypes = [P, _D, i, d, _D]
        L.hgo_step_force.restype = d
        L.hgo_s2o4_scalar.argtypes = [d, d, d]
        L.hgo_s2o4_scalar.restype = d
        L.hgo_stats.argtypes = [P, _D, d, _D]
        L.hgo_geometry.argtypes = [P, i, _D, _D, _D, _D]
        L.hgo_count_flops.argtypes = [_D]
        _lib = L
    return _lib


def _a(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


# ---- unit-level entry points -------------------------------------------------

def set_threads(n: int) -> None:
    lib().hgo_set_threads(int(n))


def get_threads() -> int:
    return int(lib().hgo_get_threads())


def moments(prim, K, side):
    """Return (u[7], v[7], w[7], xi[3]) normalised Maxwellian moments."""
    out = np.zeros(24)
    lib().hgo_moments(_ptr(_a(prim, 5)), float(K), int(side), _ptr(out))
    return out[0:7], out[7:14], out[14:21], out[21:24]


def mom_psi(prim, K, side, a, b, c, e=0):
    out = np.zeros(5)
    lib().hgo_mom_psi(_ptr(_a(prim, 5)), float(K), int(side), a, b, c, e, _ptr(out))
    return out


def mom_apsi(prim, K, side, coef, a, b, c):
    out = np.zeros(5)
    lib().hgo_mom_apsi(_ptr(_a(prim, 5)), float(K), int(side), _ptr(_a(coef, 5)), a, b, c, _ptr(out))
    return out


def slope_solve(prim, K, b):
    out = np.zeros(5)
    lib().hgo_slope_solve(_ptr(_a(prim, 5)), float(K), _ptr(_a(b, 5)), _ptr(out))
    return out


def time_slope(prim, K, a3x5):
    out = np.zeros(5)
    lib().hgo_time_slope(_ptr(_a(prim, 5)), float(K), _ptr(_a(a3x5, 15)), _ptr(out))
    return out


def time_coefficients(tau, delta):
    out = np.zeros(6)
    lib().hgo_time_coefficients(float(tau), float(delta), _ptr(out))
    return out


def q0(ql, qr, gamma=1.4):
    out = np.zeros(5)
    lib().hgo_q0(_ptr(_a(ql, 5)), _ptr(_a(qr, 5)), float(gamma), _ptr(out))
    return out


def gp_flux(ql, qr, dql, dqr, dq0n, gamma=1.4, mu_ref=0.0, T_ref=1.0, mu_exp=0.0, Pr=1.0, dt1=1e-3, dt2=5e-4):
    """Gauss-point flux in the local frame; dql, dqr are 3x5 (n, t1, t2)."""
    d = np.concatenate([_a(dql, 15), _a(dqr, 15)])
    gas = _a([gamma, mu_ref, T_ref, mu_exp, Pr, 0.0], 6)
    F1, F2 = np.zeros(5), np.zeros(5)
    lib().hgo_gp_flux(_ptr(_a(ql, 5)), _ptr(_a(qr, 5)), _ptr(d), _ptr(_a(dq0n, 5)), _ptr(gas),
                      float(dt1), float(dt2), _ptr(F1), _ptr(F2))
    return F1, F2


WHERE_FACE, WHERE_GM, WHERE_GP = 0, 1, 2


def wenoz(v, where):
    out = np.zeros(2)
    lib().hgo_wenoz(_ptr(_a(v, 5)), int(where), _ptr(out))
    return out[0], out[1]


def weno_linear(v, where):
    out = np.zeros(2)
    lib().hgo_weno_linear(_ptr(_a(v, 5)), int(where), _ptr(out))
    return out[0], out[1]


def linear_value(v, where):
    return float(lib().hgo_linear_value(_ptr(_a(v, 5)), int(where)))


def linear_weights(where):
    out = np.zeros(3)
    lib().hgo_linear_weights(int(where), _ptr(out))
    return out


def derivative_linear_weights(where):
    out = np.zeros(3)
    lib().hgo_derivative_linear_weights(int(where), _ptr(out))
    return out


def candidates(v, s):
    val, der = np.zeros(3), np.zeros(3)
    lib().hgo_candidates(_ptr(_a(v, 5)), float(s), _ptr(val), _ptr(der))
    return val, der


def normal_sweep(c6):
    out = np.zeros(5)
    lib().hgo_normal_sweep(_ptr(_a(c6, 6)), _ptr(out))
    return out  # ql, qr, dl, dr, d0


# ---- whole-grid entry points ----------------------------------------------

def _q(q, cfg):
    n = cfg.n
    assert q.shape == (5, n[2], n[1], n[0]), q.shape
    assert q.dtype == np.float64 and q.flags["C_CONTIGUOUS"]
    return q


def residual(p: dict, q: np.ndarray, dt: float):
    cfg = make_config(p)
    q = _q(np.ascontiguousarray(q), cfg)
    L, dL = np.zeros_like(q), np.zeros_like(q)
    lib().hgo_residual(ctypes.byref(cfg), _ptr(q), float(dt), _ptr(L), _ptr(dL))
    return L, dL


def residual_at(p: dict, q: np.ndarray, dt: float, cells):
    """L and dL/dt at the given cells [(i, j, k), ...] only; returns arrays [n, 5]."""
    cfg = make_config(p)
    q = _q(np.ascontiguousarray(q), cfg)
    ijk = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, 3))
    n = ijk.shape[0]
    L, dL = np.zeros((n, 5)), np.zeros((n, 5))
    lib().hgo_residual_at(ctypes.byref(cfg), _ptr(q), float(dt), int(n),
                          ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(L), _ptr(dL))
    return L, dL


def face_flux(p: dict, q: np.ndarray, dt: float, d: int, f: int, a: int, b: int):
    """F^n and dF^n/dt (10 values) of one face of direction d."""
    cfg = make_config(p)
    q = _q(np.ascontiguousarray(q), cfg)
    out = np.zeros(10)
    lib().hgo_face_flux(ctypes.byref(cfg), _ptr(q), float(dt), int(d), int(f), int(a), int(b), _ptr(out))
    return out


def cfl_dt(p: dict, q: np.ndarray) -> float:
    cfg = make_config(p)
    q = _q(np.ascontiguousarray(q), cfg)
    return float(lib().hgo_cfl_dt(ctypes.byref(cfg), _ptr(q)))


def step(p: dict, q: np.ndarray, nsteps: int, dt_fixed: float = 0.0):
    """Advance a copy of q by nsteps S2O4 steps; returns (q_new, last_dt)."""
    q, dt, _ = step_force(p, q, nsteps, dt_fixed)
    return q, dt


def step_force(p: dict, q: np.ndarray, nsteps: int, dt_fixed: float = 0.0):
    """As step, also returning the streamwise force in effect after the last
    step (changed by the constant-mass-flux controller when
    p["mass_flux_control"] is set)."""
    cfg = make_config(p)
    q = _q(np.array(q, dtype=np.float64, order="C", copy=True), cfg)
    f = ctypes.c_double(0.0)
    dt = lib().hgo_step_force(ctypes.byref(cfg), _ptr(q), int(nsteps), float(dt_fixed), ctypes.byref(f))
    return q, float(dt), float(f.value)


def s2o4_scalar(q, lam, dt):
    return float(lib().hgo_s2o4_scalar(float(q), float(lam), float(dt)))


STAT_KEYS = ["Ek", "eps_sol", "eps_dil", "eps_com"]


def stats(p: dict, q: np.ndarray, rho0: float = 1.0) -> dict:
    cfg = make_config(p)
    q = _q(np.ascontiguousarray(q), cfg)
    out = np.zeros(17)
    lib().hgo_stats(ctypes.byref(cfg), _ptr(q), float(rho0), _ptr(out))
    return {
        "Ek": out[0], "eps_sol": out[1], "eps_dil": out[2], "eps_com": out[3],
        "total": out[4:9].copy(), "max_abs": out[9:14].copy(),
        "min_p": out[14], "min_rho": out[15], "nonfinite": int(out[16]),
    }


def geometry(p: dict, axis: int):
    cfg = make_config(p)
    n = cfg.n[axis]
    h, xc, df, dg = np.zeros(n), np.zeros(n), np.zeros(n + 1), np.zeros(2 * n)
    lib().hgo_geometry(ctypes.byref(cfg), int(axis), _ptr(h), _ptr(xc), _ptr(df), _ptr(dg))
    return h, xc, df, dg


def count_flops() -> dict:
    """Operations of the plain (fully expanded) evaluation, counted by the
    oracle's counting scalar: every add, multiply, divide, square root and
    transcendental counts one."""
    out = np.zeros(12)
    lib().hgo_count_flops(_ptr(out))
    return {
        "normal_sweep_per_face": out[0],
        "tangential_1_per_face_gp_line": out[1],
        "tangential_2_per_gp": out[2],
        "flux_per_gp": out[3],
        "face_assembly": out[4],
        "flux_breakdown": dict(zip(["add", "mul", "div", "sqrt", "exp", "erfc", "pow"], out[5:12].tolist())),
    }
