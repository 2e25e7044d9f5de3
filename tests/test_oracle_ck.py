"""Pins of the oracle's GRP / Lax-Wendroff procedure (sec. 2.1.2, eq. (ck);
sec. 3.1): time Taylor coefficients of exact smooth solutions (Euler and
Burgers) differentiated in 40-digit arithmetic, and the closed form of the
linear-advection interface state."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O

def taylor_coeffs(fun, m, point, dims=3):
    """Taylor coefficients (m, 5, 5, 5) [c][a][b][k] about (x0, y0, t=0),
    total degree <= 4, of a smooth function fun(x, y, t, c) evaluated in
    40-digit arithmetic (mpmath's extrapolated numerical differentiation)."""
    mp.mp.dps = 40
    out = np.zeros((m, 5, 5, 5))
    p0 = (mp.mpf(point[0]), mp.mpf(point[1]), mp.mpf(0))
    for c in range(m):
        f = lambda x, y, t, c=c: fun(x, y, t, c)
        for a in range(5):
            for b in range(5 if dims == 3 else 1):
                for k in range(5 - a - b):
                    d = mp.diff(f, p0, (a, b, k))
                    out[c, a, b, k] = float(d) / (
                        math.factorial(a) * math.factorial(b) * math.factorial(k))
    return out


def check_ck(cfg, dim, exact, rtol=1e-11):
    w0 = exact.copy()
    w0[..., 1:] = 0.0
    got = O.ck_fill(cfg, dim, w0)
    scale = np.abs(exact).max()
    np.testing.assert_allclose(got, exact, rtol=0, atol=rtol * scale)


def mp_euler_cons(rho, u, v, p, c):
    g = mp.mpf(7) / 5
    return [rho, rho * u, rho * v, p / (g - 1) + rho * (u * u + v * v) / 2][c]


def test_ck_isentropic_vortex_exact_solution():
    """The isentropic vortex translating with (1,1) (sec. 5) is an exact Euler
    solution with non-trivial u, v, p: its time derivatives must come out of
    its spatial derivatives."""
    def fun(x, y, t, c):
        g = mp.mpf(7) / 5
        X, Y = x - t - 5, y - t - 5
        r2 = X * X + Y * Y
        T = 1 - 25 * (g - 1) / (8 * g * mp.pi ** 2) * mp.exp(1 - r2)
        rho = T ** (1 / (g - 1))
        e = mp.exp((1 - r2) / 2)
        u = 1 - 5 / (2 * mp.pi) * e * Y
        v = 1 + 5 / (2 * mp.pi) * e * X
        return mp_euler_cons(rho, u, v, rho ** g, c)

    exact = taylor_coeffs(fun, 4, ("5.4", "4.3"))
    check_ck(O.Config(eq=O.EULER), 2, exact)


def density_wave(x, y, t, c):
    rho = 1 + mp.mpf(1) / 5 * mp.sin(mp.pi * (x + y - 2 * t))
    return mp_euler_cons(rho, 1, 1, 1, c)


def test_ck_2d_density_wave():
    exact = taylor_coeffs(density_wave, 4, ("0.3", "1.1"))
    check_ck(O.Config(eq=O.EULER), 2, exact)


def test_ck_burgers_exact_implicit_solution():
    """Burgers' equation (sec. 5, the Burgers example): the smooth solution is
    u = u0(x - u t), here solved to 40 digits by mpmath before it is
    differentiated."""
    def fun(x, y, t, c):
        u0 = lambda s: mp.mpf(1) / 2 + mp.sin(mp.pi * s)
        if t == 0:
            return u0(x)
        return mp.findroot(lambda u: u - u0(x - u * t), u0(x))

    exact = taylor_coeffs(fun, 1, ("0.37", "0"), dims=1)
    check_ck(O.Config(eq=O.BURGERS), 1, exact, rtol=1e-10)


def test_ck_1d_density_wave():
    def fun(x, y, t, c):
        rho = 1 + mp.mpf(1) / 5 * mp.sin(mp.pi * (x - t))
        g = mp.mpf(7) / 5
        return [rho, rho, 1 / (g - 1) + rho / 2][c]

    exact = taylor_coeffs(fun, 3, ("0.61", "0"), dims=1)
    check_ck(O.Config(eq=O.EULER), 1, exact)


def test_ck_1d_euler_is_2d_euler_without_y():
    """1D Euler is 2D Euler with v = 0 and no y-dependence; the 2D procedure is
    pinned by exact solutions above, so the 1D one must agree with it."""
    rng = np.random.default_rng(10)
    for _ in range(5):
        w1 = np.zeros((3, 5, 5, 5))
        w1[0, 0, 0, 0] = rng.uniform(0.5, 2)
        w1[1, 0, 0, 0] = rng.uniform(-1, 1)
        w1[2, 0, 0, 0] = rng.uniform(3, 5)
        w1[:, 1:, 0, 0] = rng.normal(size=(3, 4)) * 0.3
        w2 = np.zeros((4, 5, 5, 5))
        w2[[0, 1, 3]] = w1
        cfg = O.Config(eq=O.EULER)
        g1 = O.ck_fill(cfg, 1, w1)
        g2 = O.ck_fill(cfg, 2, w2)
        np.testing.assert_allclose(g1, g2[[0, 1, 3]], rtol=1e-13, atol=1e-13)
        assert np.all(g2[2] == 0.0)


@pytest.mark.parametrize("a_speed", [1.0, -0.6])
def test_grp_linear_advection_is_exact_shift(a_speed):
    """For W_t + a W_x = 0 the interface state is the upwind polynomial shifted
    by a*tau: W(x_{j+1/2}, tau) = p(x_{j+1/2} - a tau), exactly for quartics."""
    rng = np.random.default_rng(9)
    pL = np.polynomial.Polynomial(rng.normal(size=5))
    pR = np.polynomial.Polynomial(rng.normal(size=5))
    JL = np.zeros((5, 5, 1))
    JR = np.zeros((5, 5, 1))
    for a in range(5):
        JL[a, 0, 0] = pL.deriv(a)(0.5) if a else pL(0.5)
        JR[a, 0, 0] = pR.deriv(a)(-0.5) if a else pR(-0.5)
    cfg = O.Config(eq=O.ADVECTION, adv_a=a_speed)
    w = O.grp_face(cfg, 1, JL, JR)
    for tau in (0.0, 0.13, 0.4):
        got = sum(w[0, 0, 0, k] * tau ** k for k in range(5))
        want = pL(0.5 - a_speed * tau) if a_speed > 0 else pR(-0.5 - a_speed * tau)
        assert got == pytest.approx(want, abs=1e-13)


def test_grp_euler_smooth_data_matches_exact_series():
    """With identical smooth jets on both sides the GRP must return the exact
    Taylor series of the solution (the Riemann problems are trivial)."""
    exact = taylor_coeffs(density_wave, 4, ("0.7", "0.2"))
    J = np.zeros((5, 5, 4))
    for a in range(5):
        for b in range(5 - a):
            J[a, b] = exact[:, a, b, 0] * math.factorial(a) * math.factorial(b)
    w = O.grp_face(O.Config(eq=O.EULER), 2, J, J)
    np.testing.assert_allclose(w, exact, atol=1e-11 * np.abs(exact).max())
