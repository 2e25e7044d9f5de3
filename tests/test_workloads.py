"""The seeded input generators: closed forms against Gauss-Legendre
quadrature of the same initial functions, one-sided data at a shock on a cell
edge, and the recipes' shapes and ranges."""
import numpy as np
import pytest

from paper_2304_09724_amd import workloads as WL

POST = (3.857143, 2.629369, 0.0, 10.333333)


def shock_sine_fun(x, y, side):
    left = np.asarray(side) < 0
    rho = np.where(left, POST[0], 1.0 + 0.2 * np.sin(5 * x) * np.sin(3 * y))
    u = np.where(left, POST[1], 0.0)
    p = np.where(left, POST[3], 1.0)
    return WL.prim_to_cons(rho, u, p, np.zeros_like(rho))


@pytest.mark.parametrize("nx,ny", [(64, 24), (100, 30), (40, 8)])
def test_shock_sine_2d_closed_form_matches_quadrature(nx, ny):
    """(40, 8) puts the shock on a cell edge, (64, 24) and (100, 30) inside a cell."""
    ref = WL.averages_2d(shock_sine_fun, -5.0, 5.0, 0.0, 2 * np.pi / 3, nx, ny, xbreak=-4.0)
    got = WL.shock_sine_2d(nx, ny)
    for q in range(4):
        scale = np.abs(ref[q]).max()
        assert np.abs(got[q] - ref[q]).max() <= 1e-13 * scale, q


def test_2d_averages_by_row_blocks_equal_the_whole():
    f = lambda x, y: WL.prim_to_cons(1 + 0.2 * np.sin(5 * x) * np.sin(3 * y), 0.1 + 0 * x,
                                     1 + 0 * x, 0 * x)
    whole = WL.averages_2d(f, -5, 5, 0, 2, 64, 40)
    blocks = WL.averages_2d(f, -5, 5, 0, 2, 64, 40, max_points=64 * 100 * 7)
    assert np.array_equal(whole, blocks)


@pytest.mark.parametrize("u,amp,k", [(1.0, 0.2, 1), (0.0, 0.2, 4), (-1.0, 0.1, 3)])
def test_density_wave_1d_closed_form(u, amp, k):
    n, t = 40, 0.3
    got = WL.density_wave_1d(n, t=t, u=u, amp=amp, k=k)
    ref = WL.averages_1d(lambda x: WL.prim_to_cons(1 + amp * np.sin(k * np.pi * (x - u * t)),
                                                   u + 0 * x, 1 + 0 * x), 0.0, 2.0, n)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_shock_sine_1d_one_sided_at_the_shock():
    n = 100
    st = WL.shock_sine_1d(n)
    post = WL.prim_to_cons(3.857143, 2.629369, 10.333333)
    j = 10                                  # x = -4 is the left edge of cell 10
    np.testing.assert_allclose(st[0, :, :j], np.repeat(post[:, None], j, axis=1), rtol=1e-15)
    assert np.abs(st[1, :, :j]).max() == 0.0        # no jump inside the left cells
    x = np.linspace(-5, 5, n + 1)
    want = 0.2 * (np.sin(5 * x[j + 1]) - np.sin(5 * x[j])) / 0.1
    assert st[1, 0, j] == pytest.approx(want, rel=1e-12)
    assert np.abs(st[0, 1, j:]).max() == 0.0        # at rest ahead of the shock


def test_riemann_batch_recipe():
    insts = WL.riemann_batch_1d(count=64)
    ns = np.array([d.n for d in insts])
    assert np.all(ns % 2 == 0) and ns.min() >= 200 and ns.max() <= 2000
    for d in insts:
        for side in (d.left, d.right):
            assert 0.1 <= side[0] <= 2 and -1 <= side[1] <= 1 and 0.1 <= side[2] <= 2
    again = WL.riemann_batch_1d(count=64)
    assert all(a.n == b.n and a.left == b.left for a, b in zip(insts, again))


def test_four_quadrant_batch_recipe():
    insts = WL.four_quadrant_batch(count=32)
    ns = np.array([d.n for d in insts])
    assert np.all(ns % 128 == 0) and ns.min() >= 128 and ns.max() <= 1024
    for d in insts:
        for rho, u, v, p in d.quads:
            assert 0.1 <= rho <= 1.5 and 0.1 <= p <= 1.5 and abs(u) <= 1 and abs(v) <= 1


def test_density_wave_2d_exact_average_matches_quadrature():
    for n in (12, 64):
        rho = WL.density_wave_2d(n, t=0.37)[0, 0]
        np.testing.assert_allclose(WL.density_wave_2d_exact_rho(n, t=0.37), rho, rtol=0,
                                   atol=1e-14)


def test_burgers_exact_averages():
    """At t = 0 the exact averages equal the closed-form initial ones; later,
    on the periodic domain, they keep the initial mean (conservation) and the
    initial range (the solution is constant along characteristics)."""
    n = 64
    np.testing.assert_allclose(WL.burgers_sine_exact(n, 0.0), WL.burgers_sine(n)[0, 0],
                               rtol=0, atol=1e-14)
    w = WL.burgers_sine_exact(n, 0.25)
    assert abs(w.mean() - 0.5) < 1e-14
    assert w.min() >= -0.5 - 1e-12 and w.max() <= 1.5 + 1e-12


def test_piecewise_data_matches_the_two_state_form():
    """One break: the piecewise form equals the two-state Riemann form, with the
    jump inside a cell (n = 25, up to rounding of the split cell's shares) and
    on a cell edge (n = 20)."""
    L, R = (0.445, 0.698, 3.528), (0.5, 0.0, 0.571)
    for n in (20, 25):
        np.testing.assert_allclose(WL.lax_tube(n),
                                   WL.riemann_1d(n, L, R, x0=-5.0, x1=5.0, xd=0.0),
                                   rtol=1e-15, atol=1e-14)


def test_blast_wave_data():
    st = WL.blast_waves(400)                       # breaks on cell edges
    p = (0.4 * st[0, 2])                           # u = 0: p = (gamma - 1) E
    assert np.allclose(p[:40], 1000.0) and np.allclose(p[40:360], 0.01)
    assert np.allclose(p[360:], 100.0) and np.abs(st[1]).max() == 0.0
    st = WL.blast_waves(25)                        # 0.1 inside cell 2, 0.9 inside cell 22
    assert 0.4 * st[0, 2, 2] == pytest.approx(0.5 * 1000.0 + 0.5 * 0.01)
    assert st[1, 2, 2] == pytest.approx((0.01 - 1000.0) / 0.4 / 0.04)
