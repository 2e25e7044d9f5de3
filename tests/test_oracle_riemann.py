"""Pins of the oracle's Euler building blocks: the Jacobian eigensystem against
a complex-step Jacobian, the HLLC state on cases it must resolve exactly, and
the exact Riemann solver against Rankine-Hugoniot / Riemann-invariant
relations and textbook star states."""
import numpy as np
import pytest

import oracle as O
from paper_2304_09724_amd.workloads import prim_to_cons

G = 1.4


def flux(W, direction=0, g=G):
    """Euler flux written out from its definition, for any (complex) W."""
    if W.size == 3:
        rho, m, E = W
        u = m / rho
        p = (g - 1) * (E - 0.5 * rho * u * u)
        return np.array([m, m * u + p, (E + p) * u])
    rho, mx, my, E = W
    u, v = mx / rho, my / rho
    p = (g - 1) * (E - 0.5 * rho * (u * u + v * v))
    if direction == 0:
        return np.array([mx, mx * u + p, my * u, (E + p) * u])
    return np.array([my, mx * v, my * v + p, (E + p) * v])


def jacobian(W, direction=0):
    m = W.size
    J = np.zeros((m, m))
    h = 1e-30
    for k in range(m):
        d = W.astype(complex)
        d[k] += 1j * h
        J[:, k] = flux(d, direction).imag / h
    return J


@pytest.mark.parametrize("dim,direction", [(1, 0), (2, 0), (2, 1)])
def test_eigensystem_diagonalises_the_jacobian(dim, direction):
    rng = np.random.default_rng(7)
    for _ in range(10):
        rho, p = rng.uniform(0.1, 3, 2)
        u, v = rng.uniform(-2, 2, 2)
        W = prim_to_cons(rho, u, p) if dim == 1 else prim_to_cons(rho, u, p, v)
        lam, R, L = O.euler_eigen(G, W, direction)
        np.testing.assert_allclose(L @ R, np.eye(W.size), atol=1e-12)
        A = jacobian(W, direction)
        np.testing.assert_allclose(R @ np.diag(lam) @ L, A, atol=1e-11 * np.abs(A).max())
        c = np.sqrt(G * p / rho)
        un = u if direction == 0 else v
        assert lam[0] == pytest.approx(un - c) and lam[-1] == pytest.approx(un + c)


def test_hllc_resolves_a_contact_exactly():
    for u in (0.7, -0.4):
        WL = prim_to_cons(1.0, u, 1.0, 0.3)
        WR = prim_to_cons(0.2, u, 1.0, -0.5)
        Ws = O.hllc_state(G, WL, WR)
        np.testing.assert_allclose(Ws, WL if u > 0 else WR, rtol=1e-13)


def test_hllc_supersonic_takes_upwind_state():
    WL = prim_to_cons(1.0, 5.0, 1.0)
    WR = prim_to_cons(0.5, 4.0, 0.4)
    np.testing.assert_allclose(O.hllc_state(G, WL, WR), WL)
    WL = prim_to_cons(1.0, -5.0, 1.0)
    WR = prim_to_cons(0.5, -4.0, 0.4)
    np.testing.assert_allclose(O.hllc_state(G, WL, WR), WR)


def test_hllc_symmetric_collision_has_zero_velocity():
    WL = prim_to_cons(1.0, 0.8, 1.0)
    WR = prim_to_cons(1.0, -0.8, 1.0)
    Ws = O.hllc_state(G, WL, WR)
    assert abs(Ws[1]) < 1e-14


def test_hllc_state_consistency():
    """HLLC of a state with itself is that state."""
    W = prim_to_cons(0.7, -0.2, 2.0, 0.4)
    np.testing.assert_allclose(O.hllc_state(G, W, W), W, rtol=1e-14)


def prim(W, g=G):
    """(rho, u, v, p) of a conservative state (v = 0 in 1D)."""
    rho, E = W[0], W[-1]
    u = W[1] / rho
    v = W[2] / rho if W.size == 4 else 0.0
    return rho, u, v, (g - 1) * (E - 0.5 * rho * (u * u + v * v))


@pytest.mark.parametrize("dim", [1, 2])
def test_hllc_star_state_meets_the_jump_conditions(dim):
    """The HLLC state of the leading term (sec. 2.1, Toro ch. 10) on random
    data, both star regions: with S* = (rho u)*/rho* and Davis' speeds S_L,
    S_R, the state U*_K on the side K of the contact satisfies the
    Rankine-Hugoniot condition across S_K with the flux of a state moving at
    S* under the pressure p*_K = p_K + rho_K (S_K - u_K)(S* - u_K):
    F(U_K) + S_K (U*_K - U_K) = S* U*_K + p*_K (0, 1, [0,] S*); the pressures
    p*_L and p*_R agree (the condition that fixes S*); the transverse velocity
    is side K's; the energy term (S* - u_K), which vanishes at a contact, is
    exercised because S* != u_K on this data."""
    rng = np.random.default_rng(31 + dim)
    seen = {"L": 0, "R": 0}
    for _ in range(400):
        rl, rr, pl, pr = rng.uniform(0.1, 2.0, 4)
        ul, ur, vl, vr = rng.uniform(-2.0, 2.0, 4)
        if dim == 1:
            WL, WR = prim_to_cons(rl, ul, pl), prim_to_cons(rr, ur, pr)
        else:
            WL, WR = prim_to_cons(rl, ul, pl, vl), prim_to_cons(rr, ur, pr, vr)
        Ws = O.hllc_state(G, WL, WR)
        cl, cr = np.sqrt(G * pl / rl), np.sqrt(G * pr / rr)
        SL, SR = min(ul - cl, ur - cr), max(ul + cl, ur + cr)
        if SL >= 0:
            np.testing.assert_array_equal(Ws, WL)
            continue
        if SR < 0:
            np.testing.assert_array_equal(Ws, WR)
            continue
        Ss = Ws[1] / Ws[0]
        K = "L" if Ss >= 0 else "R"
        seen[K] += 1
        WK, SK = (WL, SL) if K == "L" else (WR, SR)
        rk, uk, vk, pk = prim(WK)
        p_star = {k: p + r * (S - u) * (Ss - u)
                  for k, (r, u, p, S) in {"L": (rl, ul, pl, SL), "R": (rr, ur, pr, SR)}.items()}
        assert p_star["L"] == pytest.approx(p_star["R"], rel=1e-11, abs=1e-12)
        ps = p_star[K]
        D = np.zeros(WK.size)
        D[1], D[-1] = 1.0, Ss
        lhs = flux(WK) + SK * (Ws - WK)
        rhs = Ss * Ws + ps * D
        np.testing.assert_allclose(lhs, rhs, rtol=1e-11, atol=1e-11 * np.abs(flux(WK)).max())
        assert Ws[0] == pytest.approx(rk * (SK - uk) / (SK - Ss), rel=1e-13)
        if dim == 2:
            assert Ws[2] / Ws[0] == pytest.approx(vk, rel=1e-12, abs=1e-14)
    assert seen["L"] > 50 and seen["R"] > 50


# ---- HLLE (the positivity safeguard's first-order flux) ----------------------

def einfeldt_bounds(WL, WR, g=G):
    """Wave-speed bounds of Einfeldt (1988): the sides' acoustic speeds and the
    Roe-averaged ones."""
    def prim(W):
        rho, m, E = W
        u = m / rho
        return rho, u, (g - 1) * (E - 0.5 * rho * u * u)
    (rl, ul, pl), (rr, ur, pr) = prim(WL), prim(WR)
    hl, hr = (WL[2] + pl) / rl, (WR[2] + pr) / rr
    a, b = np.sqrt(rl), np.sqrt(rr)
    ut, ht = (a * ul + b * ur) / (a + b), (a * hl + b * hr) / (a + b)
    ct = np.sqrt((g - 1) * (ht - 0.5 * ut * ut))
    return min(ul - np.sqrt(g * pl / rl), ut - ct), max(ur + np.sqrt(g * pr / rr), ut + ct)


@pytest.mark.parametrize("left,right", [((1.0, -2.0, 0.4), (1.0, 2.0, 0.4)),
                                        ((1.0, -0.5, 1.0), (0.4, 1.5, 0.3)),
                                        ((2.0, -1.5, 3.0), (0.8, 1.2, 0.7))])
def test_hlle_state_is_the_exact_fan_average(left, right):
    """Double rarefactions, whose exact fan runs from u_L - c_L to u_R + c_R,
    speeds among Einfeldt's bounds: the bounds contain the fan, and the HLLE
    state is the mean of the exact Riemann solution over it (the integral
    form of the conservation law over [S_L t, S_R t]); its flux meets the jump
    condition across the left bound.  (With a shock the bounds may fall inside
    the fan, which the scheme allows: its positivity rests on the bounds
    covering the Roe-averaged wave speeds.)"""
    WL, WR = prim_to_cons(*left), prim_to_cons(*right)
    assert O.exact_riemann(G, left, right, 0.0)[1] < min(left[2], right[2])   # two rarefactions
    SL, SR = einfeldt_bounds(WL, WR)
    assert SL < 0 < SR
    outside = [O.exact_riemann(G, left, right, s)[0] for s in (SL - 1e-9, SR + 1e-9)]
    np.testing.assert_allclose(outside[0], left, rtol=1e-12)
    np.testing.assert_allclose(outside[1], right, rtol=1e-12)
    s = SL + (np.arange(20000) + 0.5) / 20000 * (SR - SL)
    mean = np.mean([prim_to_cons(*O.exact_riemann(G, left, right, x)[0]) for x in s], axis=0)
    F, Ws = O.hlle(G, WL, WR)
    # midpoint rule over 20000 points: first order at the kinks of the fan's edges
    np.testing.assert_allclose(Ws, mean, rtol=2e-5, atol=1e-9)
    np.testing.assert_allclose(F, flux(WL) + SL * (Ws - WL), rtol=1e-12, atol=1e-12)


def test_hlle_consistency_and_upwinding():
    W = prim_to_cons(0.7, -0.2, 2.0)
    F, Ws = O.hlle(G, W, W)
    np.testing.assert_allclose(F, flux(W), rtol=1e-14)
    np.testing.assert_allclose(Ws, W, rtol=1e-14)
    WL, WR = prim_to_cons(1.0, 5.0, 1.0), prim_to_cons(0.5, 4.0, 0.4)
    F, Ws = O.hlle(G, WL, WR)
    np.testing.assert_allclose(F, flux(WL), rtol=1e-14)
    np.testing.assert_array_equal(Ws, WL)
    F, Ws = O.hlle(G, prim_to_cons(1.0, 0.8, 1.0), prim_to_cons(1.0, -0.8, 1.0))
    assert abs(F[0]) < 1e-14 and abs(Ws[1]) < 1e-14


# Star states of the classical shock-tube tests (Toro, Riemann Solvers and
# Numerical Methods for Fluid Dynamics, ch. 4, table of exact solutions).
TORO = [
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.30313, 0.92745),
    ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 0.00189, 0.0),
    ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01), 460.894, 19.5975),
    ((1.0, 0.0, 0.01), (1.0, 0.0, 100.0), 46.0950, -6.19633),
    ((5.99924, 19.5975, 460.894), (5.99242, -6.19633, 46.0950), 1691.64, 8.68975),
]


@pytest.mark.parametrize("left,right,pstar,ustar", TORO)
def test_exact_riemann_star_state(left, right, pstar, ustar):
    out, ps = O.exact_riemann(G, left, right, 0.0)
    assert ps == pytest.approx(pstar, rel=2e-5, abs=1e-5)
    # velocity just left of the contact is u*
    lo, _ = O.exact_riemann(G, left, right, ustar - 1e-9)
    assert lo[1] == pytest.approx(ustar, rel=2e-5, abs=1e-5)


def _shock_jump_residual(a, b, s):
    """Rankine-Hugoniot residual F(b) - F(a) - s (b - a) of a 1D shock."""
    Wa, Wb = prim_to_cons(*a), prim_to_cons(*b)
    return flux(Wb) - flux(Wa) - s * (Wb - Wa)


def test_exact_riemann_rankine_hugoniot_and_isentropic_fan():
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)        # rarefaction + contact + shock
    # sample finely, locate the shock as the largest density jump right of the contact
    s = np.linspace(-2, 2, 40001)
    sol = np.array([O.exact_riemann(G, left, right, si)[0] for si in s])
    jumps = np.abs(np.diff(sol[:, 0]))
    k = np.argsort(jumps)[-1]
    a, b = sol[k + 1], sol[k]                                # a: ahead (right), b: behind
    shock_speed = s[k]
    res = _shock_jump_residual(tuple(a), tuple(b), shock_speed)
    assert np.abs(res).max() < 2e-4 * np.abs(prim_to_cons(*b)).max()
    # isentropic inside the fan: p / rho^gamma constant, u + 2c/(g-1) constant
    fan = (s > -np.sqrt(G) + 1e-3) & (s < -0.1)
    r, u, p = sol[fan].T
    ent = p / r ** G
    np.testing.assert_allclose(ent, ent[0], rtol=1e-12)
    inv = u + 2 * np.sqrt(G * p / r) / (G - 1)
    np.testing.assert_allclose(inv, inv[0], rtol=1e-12)


def test_exact_riemann_pressure_equation_residual():
    rng = np.random.default_rng(8)
    for _ in range(20):
        rl, rr, pl, pr = rng.uniform(0.1, 2, 4)
        ul, ur = rng.uniform(-1, 1, 2)
        out, ps = O.exact_riemann(G, (rl, ul, pl), (rr, ur, pr), 0.0)

        def f(p, rk, pk):
            ck = np.sqrt(G * pk / rk)
            if p > pk:
                A, B = 2 / ((G + 1) * rk), (G - 1) / (G + 1) * pk
                return (p - pk) * np.sqrt(A / (p + B))
            return 2 * ck / (G - 1) * ((p / pk) ** ((G - 1) / (2 * G)) - 1)

        assert abs(f(ps, rl, pl) + f(ps, rr, pr) + ur - ul) < 1e-12


def test_exact_riemann_symmetric_data():
    out, ps = O.exact_riemann(G, (1.0, 1.0, 1.0), (1.0, -1.0, 1.0), 0.0)
    assert abs(out[1]) < 1e-14 and ps > 1.0
