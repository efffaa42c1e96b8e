"""Pins of the oracle's fifth-order WENO-Z reconstruction (Sec. 2, last
paragraph; readings R1-R5).  Expected values come from exact cell averages of
polynomials (antiderivatives), not from the oracle."""
import math

import numpy as np
import pytest

R3 = math.sqrt(3.0)
WHERES = {0: 0.5, 1: -R3 / 6, 2: R3 / 6}


def cell_averages(coef, centres=(-2, -1, 0, 1, 2)):
    """Exact averages of sum_k coef[k] x^k over unit cells centred at 'centres'."""
    P = np.polynomial.Polynomial(coef)
    I = P.integ()
    return np.array([I(c + 0.5) - I(c - 0.5) for c in centres])


def test_gauss_linear_weights_sum_to_one(oracle):
    for where in (0, 1, 2):
        d = oracle.linear_weights(where)
        assert abs(d.sum() - 1.0) <= 1e-15 and (d > 0).all()
    np.testing.assert_array_equal(oracle.linear_weights(1), oracle.linear_weights(2)[::-1])


@pytest.mark.parametrize("where", [0, 1, 2])
def test_linear_weights_reproduce_quartics(oracle, where):
    """P9: with the nonlinear weights replaced by the linear ones, the value at
    s reproduces any quartic from its five cell averages."""
    rng = np.random.default_rng(where)
    for _ in range(5):
        coef = rng.uniform(-1, 1, 5)
        v = cell_averages(coef)
        val, _ = oracle.weno_linear(v, where)
        s = WHERES[where]
        assert abs(val - np.polynomial.Polynomial(coef)(s)) <= 1e-14
        assert abs(oracle.linear_value(v, where) - val) <= 1e-15


@pytest.mark.parametrize("s", [0.5, -R3 / 6, R3 / 6, 0.1])
def test_candidates_exact_for_quadratics(oracle, s):
    """Each candidate is the quadratic through its three averages: value and
    derivative are exact for quadratic data."""
    rng = np.random.default_rng(1)
    coef = rng.uniform(-1, 1, 3)
    P = np.polynomial.Polynomial(coef)
    v = cell_averages(coef)
    val, der = oracle.candidates(v, s)
    np.testing.assert_allclose(val, P(s), atol=1e-14)
    np.testing.assert_allclose(der, P.deriv()(s), atol=1e-14)


@pytest.mark.parametrize("where", [0, 1, 2])
def test_constant_data(oracle, where):
    """Constant data: the value is the constant (to the rounding of the weight
    normalisation) and the slope vanishes."""
    val, der = oracle.wenoz([2.5] * 5, where)
    assert abs(val - 2.5) <= 2.5 * 4e-16 and der == 0.0


@pytest.mark.parametrize("where", [0, 1, 2])
def test_wenoz_smooth_convergence(oracle, where):
    """On smooth data WENO-Z approaches the linear (fifth-order) value; the
    value error against the point value decreases at high order."""
    errs = []
    hs = [0.2, 0.1, 0.05]
    for h in hs:
        # f(x) = sin(1 + x) sampled as cell averages on cells of width h
        centres = np.array([-2, -1, 0, 1, 2]) * h
        v = np.array([(math.cos(1 + c - h / 2) - math.cos(1 + c + h / 2)) / h for c in centres])
        val, der = oracle.wenoz(v, where)
        s = WHERES[where] * h
        errs.append(abs(val - math.sin(1 + s)))
    orders = [math.log(errs[i] / errs[i + 1], 2) for i in range(2)]
    assert orders[-1] > 4.5, orders


def test_wenoz_discontinuity_uses_smooth_stencil(oracle):
    val, der = oracle.wenoz([0.0, 0.0, 0.0, 1.0, 1.0], 0)
    assert abs(val) < 1e-12 and abs(der) < 1e-12


def test_normal_sweep_mirror_symmetry(oracle):
    """Reversing the six cells swaps left and right states and flips slopes."""
    rng = np.random.default_rng(2)
    c = rng.uniform(0.5, 1.5, 6)
    a = oracle.normal_sweep(c)
    b = oracle.normal_sweep(c[::-1].copy())
    assert a[0] == b[1] and a[1] == b[0]
    assert a[2] == -b[3] and a[3] == -b[2]
    assert abs(a[4] + b[4]) <= 1e-15


def test_normal_sweep_quartic(oracle):
    """Left/right values at the face agree for smooth quartics up to the WENO
    deviation; the equilibrium slope (R4) is the exact derivative of a quartic."""
    rng = np.random.default_rng(4)
    coef = rng.uniform(-1, 1, 5)
    P = np.polynomial.Polynomial(coef)
    # face at x = 0 between cells centred at -1/2 and +1/2
    v = cell_averages(coef, centres=(-2.5, -1.5, -0.5, 0.5, 1.5, 2.5))
    ql, qr, dl, dr, d0 = oracle.normal_sweep(v)
    assert abs(d0 - P.deriv()(0.0)) <= 1e-14
    # with linear weights, both sides are exact for quartics
    vl, _ = oracle.weno_linear(v[0:5], 0)
    vr, _ = oracle.weno_linear(v[5:0:-1].copy(), 0)
    assert abs(vl - P(0.0)) <= 1e-14 and abs(vr - P(0.0)) <= 1e-14


@pytest.mark.parametrize("where", [1, 2])
def test_derivative_weights_reproduce_quartic_slopes(oracle, where):
    """R3: at the Gauss points the derivative linear weights reproduce the
    derivative of any quartic from its five cell averages."""
    d = oracle.derivative_linear_weights(where)
    assert abs(d.sum() - 1.0) <= 1e-15 and (d > 0).all()
    rng = np.random.default_rng(10 + where)
    for _ in range(5):
        coef = rng.uniform(-1, 1, 5)
        _, der = oracle.weno_linear(cell_averages(coef), where)
        assert abs(der - np.polynomial.Polynomial(coef).deriv()(WHERES[where])) <= 1e-14


@pytest.mark.parametrize("where", [1, 2])
def test_wenoz_slope_convergence_at_gauss_points(oracle, where):
    """The WENO-Z slope at a Gauss point converges at fourth order on smooth data."""
    errs = []
    for h in (0.2, 0.1, 0.05):
        centres = np.array([-2, -1, 0, 1, 2]) * h
        v = np.array([(math.cos(1 + c - h / 2) - math.cos(1 + c + h / 2)) / h for c in centres])
        _, der = oracle.wenoz(v, where)
        errs.append(abs(der / h - math.cos(1 + WHERES[where] * h)))
    assert math.log(errs[1] / errs[2], 2) > 3.7, errs
