"""Pins of the oracle's SHWENO reconstruction (sec. 2.3 of the paper and the
reading documented in oracle/recon.c) against facts fixed by mathematics:
polynomial reproduction, a symbolic derivation of the smoothness indicator,
and the limits of the nonlinear weights."""
import numpy as np
import pytest
import sympy as sp

import oracle as O

CFG = O.Config(eq=O.ADVECTION)


def exact_data_of_quartic(c):
    """Averages of p over cells -1, 0, +1 and the jumps p(l+1/2)-p(l-1/2) over
    cells -1, +1, computed from numpy's antiderivative (independent route)."""
    p = np.polynomial.Polynomial(c)
    P = p.integ()
    a = [P(l + 0.5) - P(l - 0.5) for l in (-1, 0, 1)]
    b = [p(l + 0.5) - p(l - 0.5) for l in (-1, 1)]
    return np.array(a), np.array(b)


def test_big_stencil_reproduces_quartics():
    rng = np.random.default_rng(1)
    for _ in range(20):
        c = rng.normal(size=5)
        a, b = exact_data_of_quartic(c)
        got = O.big_quartic(a, b)
        np.testing.assert_allclose(got, c, rtol=0, atol=1e-13)


def test_interface_value_is_hweno5():
    """Value at xi = +1/2 of the big-stencil quartic: the classical fifth-order
    Hermite interface formula, derived here symbolically from the five
    conditions (independent of the oracle's numeric inverse)."""
    x = sp.symbols("x")
    cs = sp.symbols("c0:5")
    am, a0, ap, bm, bp = sp.symbols("am a0 ap bm bp")
    p = sum(cs[k] * x ** k for k in range(5))
    h = sp.Rational(1, 2)
    eqs = [sp.integrate(p, (x, l - h, l + h)) - v for l, v in ((-1, am), (0, a0), (1, ap))]
    eqs += [p.subs(x, l + h) - p.subs(x, l - h) - v for l, v in ((-1, bm), (1, bp))]
    sol = sp.solve(eqs, cs)
    val = sp.expand(p.subs(sol).subs(x, h))
    coef = [val.coeff(s) for s in (am, a0, ap, bm, bp)]
    assert coef == [sp.Rational(-23, 120), sp.Rational(19, 30), sp.Rational(67, 120),
                    sp.Rational(-3, 40), sp.Rational(-7, 40)]
    rng = np.random.default_rng(2)
    for _ in range(10):
        d = rng.normal(size=5)
        c = O.big_quartic(d[:3], d[3:])
        got = np.polynomial.Polynomial(c)(0.5)
        want = sum(float(k) * v for k, v in zip(coef, d))
        assert abs(got - want) < 1e-13


def test_smoothness_indicator_matches_symbolic_integral():
    x = sp.symbols("x")
    cs = sp.symbols("c0:5")
    p = sum(cs[k] * x ** k for k in range(5))
    beta = sum(sp.integrate(sp.diff(p, x, k) ** 2, (x, -sp.Rational(1, 2), sp.Rational(1, 2)))
               for k in range(1, 5))
    f = sp.lambdify(cs, beta)
    rng = np.random.default_rng(3)
    for _ in range(20):
        c = rng.normal(size=5)
        assert O.smoothness(c) == pytest.approx(f(*c), rel=1e-13, abs=1e-14)


def test_weights_equal_linear_weights_on_linear_data():
    # linear data: all three candidate polynomials coincide, so tau = 0
    for slope, off in ((0.0, 1.3), (0.7, -2.0), (-3.0, 0.1)):
        a = np.array([off - slope, off, off + slope])
        b = np.array([slope, slope])
        w = O.weights(CFG, a, b)
        np.testing.assert_allclose(w, CFG.lin_w, rtol=0, atol=1e-15)


def test_nonlinear_recon_equals_quartic_on_smooth_linear_data():
    a = np.array([0.3, 0.5, 0.7])
    b = np.array([0.2, 0.2])
    np.testing.assert_allclose(O.recon_scalar(CFG, a, b), O.big_quartic(a, b), atol=1e-15)


def test_combine_with_linear_weights_is_big_quartic():
    rng = np.random.default_rng(4)
    for _ in range(10):
        d = rng.normal(size=5)
        np.testing.assert_allclose(O.combine(CFG, d[:3], d[3:], CFG.lin_w),
                                   O.big_quartic(d[:3], d[3:]), atol=1e-13)


def test_weights_pick_the_smooth_side_at_a_jump():
    # a step between cells 0 and +1: the left linear stencil is smooth
    a = np.array([1.0, 1.0, 0.0])
    b = np.array([0.0, 0.0])
    w = O.weights(CFG, a, b)
    assert w[1] > 0.9 and w[0] < 0.05 and w[2] < 1e-3
    # mirror image: the right stencil wins
    w2 = O.weights(CFG, a[::-1].copy(), b)
    assert w2[2] > 0.9 and w2[0] < 0.05


def test_weights_sum_to_one_and_are_positive():
    rng = np.random.default_rng(5)
    for _ in range(50):
        d = rng.normal(size=5) * 10 ** rng.uniform(-6, 2)
        w = O.weights(CFG, d[:3], d[3:])
        assert np.all(w > 0) and abs(w.sum() - 1) < 1e-14


def test_reconstruction_preserves_cell_average():
    """Every candidate has the centre cell's average, so the combination does."""
    rng = np.random.default_rng(6)
    for _ in range(20):
        d = rng.normal(size=5)
        c = O.recon_scalar(CFG, d[:3], d[3:])
        P = np.polynomial.Polynomial(c).integ()
        assert P(0.5) - P(-0.5) == pytest.approx(d[1], abs=1e-13)
