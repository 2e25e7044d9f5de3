"""Pins of the oracle's whole time step against the paper's printed error
tables (sec. 5), exact solutions, conservation, symmetries and the linear
stability of the scheme."""
import numpy as np
import pytest

import oracle as O
from paper_2304_09724_amd import workloads as WL
from tests.golden.load import table

EULER = O.Config(eq=O.EULER)


def errs(e):
    return np.abs(e).mean(), np.sqrt((e ** 2).mean()), np.abs(e).max()


# ---- the paper's tables --------------------------------------------------------

@pytest.mark.parametrize("n", [10, 20, 40, 80, 160])
def test_euler1d_density_wave_matches_paper_table(n):
    """Table ex4.21d (1D Euler density wave, T = 10, CFL 0.9).  The paper does
    not print its reconstruction; with the reading in oracle/recon.c the
    L1 and L2 errors agree within 2% for N >= 20 (the paper's fine-grid
    errors sit ~0.7% above, as a CFL of ~0.893 would give), Linf within 6% at
    N = 20 and 2% beyond, and all within 15% at N = 10."""
    st = WL.density_wave_1d(n)
    s, t, steps, bad = O.advance1d(EULER, st, 2.0 / n, 0.9, 10.0)
    assert not bad and t == 10.0
    e = errs(s[0, 0] - WL.density_wave_1d(n, t=10.0)[0, 0])
    ref = table("euler1d_density_wave")[n]
    if n == 10:
        np.testing.assert_allclose(e, ref, rtol=0.15)
    else:
        np.testing.assert_allclose(e[:2], ref[:2], rtol=0.02)          # L1, L2
        np.testing.assert_allclose(e[2], ref[2], rtol=0.06 if n == 20 else 0.02)


@pytest.mark.parametrize("mode", [O.W_LINEAR, O.W_NONLINEAR])
@pytest.mark.parametrize("n", [10, 20, 40])
def test_euler2d_density_wave_matches_paper_table(n, mode):
    """Table ex4.12d (2D Euler density wave, T = 1).  At 10^2 the paper's error
    is 3-5x the oracle's (coarse-grid effects of unprinted details); from
    20^2 on, L1 and L2 agree within 11% (6% at 40^2) and Linf within 25%
    (8%), converging together (an earlier run of the same reading found
    1.2% at 160^2)."""
    st = WL.density_wave_2d(n)
    cfg = O.Config(eq=O.EULER, weights=mode)
    s, t, steps, bad = O.advance2d(cfg, st, 2.0 / n, 2.0 / n, 0.9, 1.0)
    assert not bad
    e = errs(s[0, 0] - WL.density_wave_2d_exact_rho(n, t=1.0))
    ref = table("euler2d_density_wave")[n]
    if n == 10:
        assert np.all(e < ref) and np.all(e > ref / 10)
    else:
        np.testing.assert_allclose(e[:2], ref[:2], rtol=0.11 if n == 20 else 0.06)
        np.testing.assert_allclose(e[2], ref[2], rtol=0.25 if n == 20 else 0.08)


def test_burgers_orders_match_paper_table():
    """Table ex4.1 (Burgers from W0 = 0.5 + sin(pi x), periodic (0,2),
    T = 0.5/pi, CFL 0.9) against exact averages (Newton's iteration on the
    characteristics, then Gauss-Legendre).  The oracle's L1 errors lie
    3.6-4.9x under the paper's at every N, by the same factor at every CFL
    number from 0.2 to 1 (the error is spatial; the paper does not print what
    differs), so the pins are the orders: within 0.2 of the printed ones at
    80 -> 160 -> 320 and above 4.5 from 40 on; every error under the paper's,
    L1 above a sixth of it."""
    ref = table("burgers")
    cfg = O.Config(eq=O.BURGERS)
    T = 0.5 / np.pi
    ns = [40, 80, 160, 320]
    l1 = []
    for n in ns:
        s, t, steps, bad = O.advance1d(cfg, WL.burgers_sine(n), 2.0 / n, 0.9, T)
        assert not bad and t == T
        e = errs(s[0, 0] - WL.burgers_sine_exact(n, T))
        assert np.all(e < ref[n]) and e[0] > ref[n][0] / 6, (n, e, ref[n])
        l1.append(e[0])
    orders = np.log2(np.array(l1[:-1]) / np.array(l1[1:]))
    paper = np.log2(np.array([ref[n][0] for n in ns[:-1]]) / np.array([ref[n][0] for n in ns[1:]]))
    assert np.all(orders > 4.5), orders
    assert np.all(np.abs(orders[1:] - paper[1:]) < 0.2), (orders, paper)


@pytest.mark.parametrize("n", [10, 20])
def test_isentropic_vortex_matches_paper_table(n):
    """Table isotro (2D isentropic vortex on periodic (0,10)^2, T = 10, CFL 0.9;
    the vortex is back at its start, so the exact averages are the initial
    ones): the nonlinear smooth case, with density, both velocities and
    pressure all varying, that drives every term of the 2D Lax-Wendroff
    procedure.  The oracle's L1 and L2 lie 4-12% under the paper's at 10^2
    and within 5% at 20^2 (4.8% and 2.7% at 40^2), Linf within a factor 2 at
    10^2 and 25% at 20^2."""
    st = WL.isentropic_vortex(n)
    s, t, steps, bad = O.advance2d(EULER, st, 10.0 / n, 10.0 / n, 0.9, 10.0)
    assert not bad and t == 10.0
    e = errs(s[0, 0] - st[0, 0])
    ref = table("isentropic_vortex")[n]
    if n == 10:
        np.testing.assert_allclose(e[:2], ref[:2], rtol=0.15)
        assert ref[2] / 2 < e[2] < ref[2]
    else:
        np.testing.assert_allclose(e[:2], ref[:2], rtol=0.05)
        np.testing.assert_allclose(e[2], ref[2], rtol=0.25)


def test_euler2d_order_from_paper_grids():
    e = {}
    for n in (20, 40):
        s, *_ = O.advance2d(EULER, WL.density_wave_2d(n), 2.0 / n, 2.0 / n, 0.9, 1.0)
        e[n] = np.abs(s[0, 0] - WL.density_wave_2d_exact_rho(n, t=1.0)).mean()
    order = np.log2(e[20] / e[40])
    ref = table("euler2d_density_wave")
    paper = np.log2(ref[20][0] / ref[40][0])
    assert abs(order - paper) < 0.1 and order > 4.9


# ---- linear advection (order of accuracy, closed forms) ------------------------

def test_advection_fifth_order_under_refinement():
    """u_t + u_x = 0, u0 = sin(pi x) on periodic [0,2], t = 2, CFL 0.3: the
    error against the exact averages falls by 2^5 per refinement."""
    cfg = O.Config(eq=O.ADVECTION, adv_a=1.0)
    e = []
    for n in (100, 200, 400):
        s, t, steps, bad = O.advance1d(cfg, WL.sine_advection(n), 2.0 / n, 0.3, 2.0)
        e.append(np.abs(s[0, 0] - WL.sine_advection_exact(n, 2.0)).mean())
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(np.abs(orders - 5.0) < 0.1), orders


def _amplification(nu, theta, n=64):
    """2x2 amplification matrix of the linear scheme (linear weights, a = 1)
    on the Fourier mode exp(i k x), from one oracle step applied to the real
    and imaginary parts of the mode in W and in V."""
    cfg = O.Config(eq=O.ADVECTION, adv_a=1.0, weights=O.W_LINEAR)
    dx = 1.0
    j = np.arange(n)
    k = int(round(theta * n / (2 * np.pi)))
    th = 2 * np.pi * k / n
    cols = []
    for q in range(2):
        resp = []
        for part in (np.cos, np.sin):
            st = np.zeros((2, 1, n))
            st[q, 0] = part(th * j)
            out, _ = O.step1d(cfg, st, dx, nu * dx)
            resp.append(out[:, 0, :])
        # complex response to exp(i th j) = cos + i sin
        z = resp[0] + 1j * resp[1]
        cols.append(z[:, 0])             # value at cell 0 (mode amplitude)
    return th, np.array(cols).T


@pytest.mark.parametrize("nu", [0.3, 0.6, 0.9, 1.0])
def test_linear_scheme_is_stable_up_to_cfl_one(nu):
    for theta in np.linspace(0.1, np.pi, 16):
        th, A = _amplification(nu, theta)
        rho = np.abs(np.linalg.eigvals(A)).max()
        assert rho <= 1.0 + 1e-12, (nu, th, rho)


def test_linear_scheme_unstable_beyond_cfl_one():
    worst = max(np.abs(np.linalg.eigvals(_amplification(1.05, th)[1])).max()
                for th in np.linspace(0.1, np.pi, 32))
    assert worst > 1.0 + 1e-3


def test_linear_scheme_physical_mode_is_fifth_order():
    """The physical eigenvalue approximates exp(-i nu theta) with a local error
    O(theta^6) (fifth order in space and time)."""
    errs_ = []
    for theta in (0.4, 0.2):
        th, A = _amplification(0.3, theta, n=int(round(2 * np.pi / theta)) * 4)
        ev = np.linalg.eigvals(A)
        exact = np.exp(-1j * 0.3 * th)
        errs_.append(np.abs(ev - exact).min())
    assert 5.5 < np.log2(errs_[0] / errs_[1]) < 6.5


# ---- conservation, invariants, symmetry ------------------------------------

def _smooth_random_1d(n, rng):
    x = (np.arange(n) + 0.5) / n
    rho = 1 + 0.3 * np.sin(2 * np.pi * x + rng.uniform(0, 6))
    u = 0.4 * np.cos(2 * np.pi * x)
    p = 1 + 0.2 * np.sin(4 * np.pi * x)
    W = WL.prim_to_cons(rho, u, p)
    V = np.gradient(W, 1.0 / n, axis=1)
    return np.stack([W, V])


def test_conservation_and_derivative_sums_1d_periodic():
    rng = np.random.default_rng(11)
    st = _smooth_random_1d(64, rng)
    dx = 1.0 / 64
    mass0 = st[0].sum(axis=1)
    for _ in range(20):
        dt = O.dt1d(EULER, st, dx, 0.9)
        st, bad = O.step1d(EULER, st, dx, dt)
        assert not bad
    scale = np.abs(st[0]).sum(axis=1)
    assert np.all(np.abs(st[0].sum(axis=1) - mass0) < 1e-14 * scale)
    assert np.abs(st[1].sum(axis=1)).max() * dx < 1e-12


def test_free_stream_is_preserved():
    W = WL.prim_to_cons(np.full(32, 0.7), np.full(32, -0.3), np.full(32, 2.0))
    st = np.stack([W, np.zeros_like(W)])
    out, bad = O.step1d(EULER, st, 1 / 32, 0.01)
    np.testing.assert_allclose(out, st, rtol=0, atol=1e-14)
    W2 = WL.prim_to_cons(np.full((8, 12), 0.7), 0.3, 2.0, np.full((8, 12), -0.4))
    z = np.zeros_like(W2)
    st2 = np.stack([W2, z, z, z])
    out2, bad = O.step2d(EULER, st2, 0.1, 0.07, 0.01)
    np.testing.assert_allclose(out2, st2, rtol=0, atol=1e-13)


def test_mirror_symmetry_1d():
    """x -> -x: mirrored data (momentum negated) gives the mirrored result."""
    rng = np.random.default_rng(12)
    st = _smooth_random_1d(40, rng)
    mir = st[:, :, ::-1].copy()
    mir[0, 1] *= -1          # momentum is odd
    mir[1, [0, 2]] *= -1     # x-derivatives of even quantities are odd
    a, _ = O.step1d(EULER, st, 1 / 40, 0.004)
    b, _ = O.step1d(EULER, mir, 1 / 40, 0.004)
    bm = b[:, :, ::-1].copy()
    bm[0, 1] *= -1
    bm[1, [0, 2]] *= -1
    np.testing.assert_allclose(a, bm, rtol=0, atol=1e-12)


def _smooth_random_2d(nx, ny, rng):
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    ph = rng.uniform(0, 6, 3)
    rho = 1 + 0.3 * np.sin(2 * np.pi * (X + ph[0])) * np.cos(2 * np.pi * (Y + ph[1]))
    u = 0.3 * np.cos(2 * np.pi * (Y + ph[2]))
    v = -0.2 * np.sin(2 * np.pi * X)
    p = 1 + 0.1 * np.cos(2 * np.pi * (X - Y))
    W = WL.prim_to_cons(rho, u, p, v)
    V = np.gradient(W, 1.0 / nx, axis=2)
    Yd = np.gradient(W, 1.0 / ny, axis=1)
    Z = np.gradient(V, 1.0 / ny, axis=1)
    return np.ascontiguousarray(np.stack([W, V, Yd, Z]))


def test_conservation_and_derivative_sums_2d_periodic():
    rng = np.random.default_rng(13)
    st = _smooth_random_2d(16, 12, rng)
    dx, dy = 1 / 16, 1 / 12
    mass0 = st[0].sum(axis=(1, 2))
    for _ in range(3):
        dt = O.dt2d(EULER, st, dx, dy, 0.9)
        st, bad = O.step2d(EULER, st, dx, dy, dt)
        assert not bad
    scale = np.abs(st[0]).sum(axis=(1, 2))
    assert np.all(np.abs(st[0].sum(axis=(1, 2)) - mass0) < 1e-14 * scale)
    for q in (1, 2, 3):
        assert np.abs(st[q].sum(axis=(1, 2))).max() < 1e-10 * np.abs(st[q]).max() * st[q][0].size


def test_transpose_symmetry_2d():
    rng = np.random.default_rng(14)
    st = _smooth_random_2d(10, 14, rng)
    tr = np.ascontiguousarray(st[[0, 2, 1, 3]][:, [0, 2, 1, 3]].transpose(0, 1, 3, 2))
    a, _ = O.step2d(EULER, st, 0.1, 0.07, 0.01)
    b, _ = O.step2d(EULER, tr, 0.07, 0.1, 0.01)
    bt = b[[0, 2, 1, 3]][:, [0, 2, 1, 3]].transpose(0, 1, 3, 2)
    np.testing.assert_allclose(a, bt, rtol=0, atol=1e-12)


def test_2d_step_on_y_independent_data_is_the_1d_step():
    """2D Euler data that does not depend on y and has v = 0 evolves exactly as
    1D Euler data (the scheme reduces dimension by dimension)."""
    rng = np.random.default_rng(15)
    s1 = _smooth_random_1d(24, rng)
    W = np.zeros((4, 4, 5, 24))
    W[0][[0, 1, 3]] = s1[0][:, None, :]
    W[1][[0, 1, 3]] = s1[1][:, None, :]
    dt = 0.005
    o1, _ = O.step1d(EULER, s1, 1 / 24, dt)
    o2, _ = O.step2d(EULER, W, 1 / 24, 0.3, dt)
    for j in range(5):
        np.testing.assert_allclose(o2[0][[0, 1, 3]][:, j], o1[0], rtol=0, atol=1e-13)
        np.testing.assert_allclose(o2[1][[0, 1, 3]][:, j], o1[1], rtol=0, atol=1e-11)
    assert np.abs(o2[2]).max() < 1e-12 and np.abs(o2[3]).max() < 1e-10


# ---- shocks: exact Riemann solutions ------------------------------------------

def exact_riemann_averages(left, right, n, t, x0=0.0, x1=1.0, xd=0.5, sub=64):
    e = np.linspace(x0, x1, n + 1)
    xs = (e[:-1, None] + (np.arange(sub) + 0.5) / sub * (x1 - x0) / n)
    rho = np.array([[O.exact_riemann(1.4, left, right, (xx - xd) / t)[0][0] for xx in row]
                    for row in xs])
    return rho.mean(axis=1)


@pytest.mark.parametrize("left,right", [((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),
                                        ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))])
def test_riemann_problem_converges_to_exact_solution(left, right):
    """Sod and Lax data on [0,1], transmissive ends, t = 0.14: the L1 error
    against the exact Riemann solution falls under refinement and stays
    non-oscillatory (densities inside the data's range, up to small
    overshoots)."""
    cfg = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4)
    e = []
    for n in (50, 100, 200):
        st = WL.riemann_1d(n, left, right)
        s, t, steps, bad = O.advance1d(cfg, st, 1.0 / n, 0.9, 0.14)
        assert not bad
        ex = exact_riemann_averages(left, right, n, 0.14)
        e.append(np.abs(s[0, 0] - ex).mean())
        lo, hi = min(left[0], right[0], ex.min()), max(left[0], right[0], ex.max())
        assert s[0, 0].min() > lo - 0.05 * (hi - lo) and s[0, 0].max() < hi + 0.05 * (hi - lo)
    assert e[1] < 0.75 * e[0] and e[2] < 0.75 * e[1], e


def test_blast_waves_conserve_at_reflective_walls():
    """The interacting blast waves (sec. 5) at 400 cells to T = 0.038 with
    reflective walls: the run stays physical, and mass and energy, whose wall
    fluxes vanish, are conserved to rounding."""
    cfg = O.Config(eq=O.EULER, bc=(O.BC_REFLECTIVE,) * 4)
    st = WL.blast_waves(400)
    s, t, steps, bad = O.advance1d(cfg, st, 1.0 / 400, 0.9, 0.038)
    assert not bad and t == 0.038
    for c in (0, 2):
        assert abs(s[0, c].sum() - st[0, c].sum()) <= 1e-14 * st[0, c].sum()
    assert s[0, 0].min() > 0.1 and s[0, 0].max() < 7.0


# ---- the positivity safeguard (an addition, off by default) ------------------

def test_positivity_safeguard_changes_nothing_where_it_is_not_needed():
    """Runs that never meet a non-physical update are bit for bit the same
    with the safeguard on."""
    for st, dx, T, bc in ((WL.density_wave_1d(40), 2.0 / 40, 0.5, O.BC_PERIODIC),
                          (WL.lax_tube(200), 10.0 / 200, 1.3, O.BC_TRANSMISSIVE)):
        runs = [O.advance1d(O.Config(eq=O.EULER, bc=(bc,) * 4, positivity=p), st, dx, 0.9, T)
                for p in (False, True)]
        assert not runs[0][3] and not runs[1][3]
        np.testing.assert_array_equal(runs[0][0], runs[1][0])


def test_positivity_safeguard_is_local_and_conservative():
    """Blast waves at 200 cells (which fail without the safeguard at step 262):
    at every step where the unguarded update would be non-physical, the guarded
    one is physical, equals the unguarded one bit for bit in every cell with
    no troubled cell next to it, and has the same total mass and energy (the
    walls' fluxes of both vanish); the whole guarded run reaches T."""
    n = 200
    on = O.Config(eq=O.EULER, bc=(O.BC_REFLECTIVE,) * 4, positivity=True)
    off = O.Config(eq=O.EULER, bc=(O.BC_REFLECTIVE,) * 4)
    st, t, hits = WL.blast_waves(n), 0.0, 0
    while t < 0.038:
        dt = min(O.dt1d(on, st, 1.0 / n, 0.9), 0.038 - t)
        a, bad_off = O.step1d(off, st, 1.0 / n, dt)
        b, bad_on = O.step1d(on, st, 1.0 / n, dt)
        assert not bad_on
        if bad_off:
            hits += 1
            rho, m, E = a[0]
            with np.errstate(all="ignore"):
                trouble = ~((rho > 0) & (0.4 * (E - 0.5 * m * m / rho) > 0))
            near = trouble | np.roll(trouble, 1) | np.roll(trouble, -1)
            near[0] |= trouble[0]                      # mirror ghosts
            near[-1] |= trouble[-1]
            np.testing.assert_array_equal(a[:, :, ~near], b[:, :, ~near])
            for c in (0, 2):
                assert abs(b[0, c].sum() - st[0, c].sum()) <= 1e-13 * st[0, c].sum()
        st, t = b, t + dt
    assert hits > 0


def test_positivity_safeguard_2d_is_local_and_conservative():
    """2D: four-quadrant data of the batch (instance 75) on a periodic 16^2
    grid fail at step 4 without the safeguard.  With it, 12 steps run; at
    every step where the unguarded update would be non-physical, cells with no
    troubled cell among themselves and their four edge neighbours are the
    unguarded values bit for bit, and the totals of mass, both momenta and
    energy hold (periodic faces cancel); a smooth run is unchanged."""
    n = 16
    quads = WL.four_quadrant_batch(count=256)[75].quads
    on = O.Config(eq=O.EULER, positivity=True)
    off = O.Config(eq=O.EULER)
    st, hits = WL.four_quadrant(n, quads), 0
    for _ in range(12):
        dt = O.dt2d(on, st, 1.0 / n, 1.0 / n, 0.9)
        a, bad_off = O.step2d(off, st, 1.0 / n, 1.0 / n, dt)
        b, bad_on = O.step2d(on, st, 1.0 / n, 1.0 / n, dt)
        assert not bad_on
        if bad_off:
            hits += 1
            rho, mx, my, E = a[0]
            with np.errstate(all="ignore"):
                trouble = ~((rho > 0) & (0.4 * (E - 0.5 * (mx * mx + my * my) / rho) > 0))
            near = trouble.copy()
            for ax in (0, 1):
                near |= np.roll(trouble, 1, ax) | np.roll(trouble, -1, ax)
            np.testing.assert_array_equal(a[:, :, ~near], b[:, :, ~near])
            for c in range(4):
                scale = max(np.abs(st[0, c]).sum(), 1.0)
                assert abs(b[0, c].sum() - st[0, c].sum()) <= 1e-13 * scale, c
        st = b
    assert hits > 0
    smooth = WL.density_wave_2d(12)
    x = O.step2d(off, smooth, 2 / 12, 2 / 12, 0.01)[0]
    y = O.step2d(on, smooth, 2 / 12, 2 / 12, 0.01)[0]
    np.testing.assert_array_equal(x, y)


def test_transmissive_boundary_keeps_constant_state():
    cfg = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4)
    W = WL.prim_to_cons(np.full(20, 1.3), np.full(20, 0.4), np.full(20, 0.8))
    st = np.stack([W, np.zeros_like(W)])
    out, _ = O.step1d(cfg, st, 0.05, 0.01)
    np.testing.assert_allclose(out, st, atol=1e-14)


def test_reflective_wall_has_zero_mass_flux():
    """Reflective ends: the total mass in the domain is conserved exactly."""
    cfg = O.Config(eq=O.EULER, bc=(O.BC_REFLECTIVE,) * 4)
    st = WL.riemann_1d(60, (1.0, 0.5, 1.0), (0.5, -0.5, 0.5))
    m0 = st[0, 0].sum()
    s, t, steps, bad = O.advance1d(cfg, st, 1 / 60, 0.9, 0.3)
    assert not bad
    assert abs(s[0, 0].sum() - m0) < 1e-13 * m0
