"""Seeded synthetic inputs: initial states of the paper's test problems and of
the batched workloads, as exact cell averages and exact derivative averages.

This module holds no arithmetic of the scheme.  It only evaluates initial
conditions and their exact averages, so both the GPU library's tests and the
CPU oracle's tests draw the same inputs from it.

Layout: 1D state (2, m, n) = [W, V][component][cell]; 2D state (4, m, ny, nx)
= [W, V, Y, Z][component][y][x].  Components are conservative
(rho, rho u[, rho v], E).

Initial averages (the scheme's state, sec. 2.4 eq. (vv) and sec. 3.2):
  W = (1/|I|) int_I W0,  V = average of dW0/dx over the open cell, i.e.
  (W0(x_{j+1/2}^-) - W0(x_{j-1/2}^+))/dx; Y likewise in y; Z from the four
  corner values.  A jump lying exactly on a cell edge therefore contributes
  nothing to any derivative average (a reading: the paper does not say).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED = 230409724
GAMMA = 1.4

_GL_X, _GL_W = np.polynomial.legendre.leggauss(10)   # on [-1, 1]


def _gl_nodes(a, b):
    """Gauss-Legendre nodes/weights (normalised to sum 1) on each [a_k, b_k]."""
    a = np.asarray(a, float)[..., None]
    b = np.asarray(b, float)[..., None]
    x = 0.5 * (a + b) + 0.5 * (b - a) * _GL_X
    return x, 0.5 * _GL_W


def prim_to_cons(rho, u, p, v=None, gamma=GAMMA):
    """Conservative variables from primitive ones (1D if v is None)."""
    rho = np.asarray(rho, float)
    if v is None:
        return np.stack([rho, rho * u, p / (gamma - 1) + 0.5 * rho * u * u])
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1) + 0.5 * rho * (u * u + v * v)])


def cons_to_prim(W, gamma=GAMMA):
    W = np.asarray(W, float)
    if W.shape[0] == 3:
        rho, m, E = W
        u = m / rho
        return rho, u, (gamma - 1) * (E - 0.5 * rho * u * u)
    rho, mx, my, E = W
    u, v = mx / rho, my / rho
    return rho, u, v, (gamma - 1) * (E - 0.5 * rho * (u * u + v * v))


# ---------------------------------------------------------------------------
# 1D
# ---------------------------------------------------------------------------

def averages_1d(fun, x0, x1, n):
    """Exact-quadrature averages of a smooth pointwise function fun(x) ->
    (m, ...) over n uniform cells of [x0, x1]; returns state (2, m, n)."""
    e = np.linspace(x0, x1, n + 1)
    dx = (x1 - x0) / n
    xq, wq = _gl_nodes(e[:-1], e[1:])
    Wq = np.asarray(fun(xq))
    Wbar = (Wq * wq).sum(-1)
    We = np.asarray(fun(e))
    V = (We[..., 1:] - We[..., :-1]) / dx
    return np.ascontiguousarray(np.stack([Wbar, V]))


def sine_advection(n: int = 200, x0: float = 0.0, x1: float = 2.0):
    """u0 = sin(pi x) on periodic [0, 2] (the linear-advection workload)."""
    e = np.linspace(x0, x1, n + 1)
    dx = (x1 - x0) / n
    Wbar = -(np.cos(np.pi * e[1:]) - np.cos(np.pi * e[:-1])) / (np.pi * dx)
    V = (np.sin(np.pi * e[1:]) - np.sin(np.pi * e[:-1])) / dx
    return np.ascontiguousarray(np.stack([Wbar[None], V[None]]))


def sine_advection_exact(n, t, x0=0.0, x1=2.0, a=1.0):
    e = np.linspace(x0, x1, n + 1) - a * t
    dx = (x1 - x0) / n
    return -(np.cos(np.pi * e[1:]) - np.cos(np.pi * e[:-1])) / (np.pi * dx)


def burgers_sine(n: int, x0=0.0, x1=2.0):
    """W0 = 0.5 + sin(pi x) on periodic (0, 2) (sec. 5, Burgers example)."""
    e = np.linspace(x0, x1, n + 1)
    dx = (x1 - x0) / n
    Wbar = 0.5 - (np.cos(np.pi * e[1:]) - np.cos(np.pi * e[:-1])) / (np.pi * dx)
    V = (np.sin(np.pi * e[1:]) - np.sin(np.pi * e[:-1])) / dx
    return np.ascontiguousarray(np.stack([Wbar[None], V[None]]))


def burgers_sine_exact(n: int, t: float, x0=0.0, x1=2.0):
    """Exact cell averages at time t < 1/pi (before the shock forms) of
    Burgers' equation from W0 = 0.5 + sin(pi x): the value at x is the root of
    w = 0.5 + sin(pi (x - w t)) (the characteristic through x), found by
    Newton's iteration (its derivative 1 + pi t cos(.) stays positive), then
    averaged by Gauss-Legendre quadrature."""
    assert 0.0 <= t < 1.0 / np.pi

    def point(x):
        w = 0.5 + np.sin(np.pi * x)
        for _ in range(60):
            ph = np.pi * (x - w * t)
            step = (w - 0.5 - np.sin(ph)) / (1.0 + np.pi * t * np.cos(ph))
            w = w - step
            if np.abs(step).max() < 1e-16:
                break
        return w[None]
    return averages_1d(point, x0, x1, n)[0, 0]


def density_wave_1d(n: int, t: float = 0.0, gamma=GAMMA, x0=0.0, x1=2.0, u=1.0, amp=0.2,
                    k=1):
    """rho = 1 + amp sin(k pi (x - u t)), velocity u, p = 1 on periodic (0, 2)
    (sec. 5, the 1D Euler accuracy example has u = 1, amp = 0.2, k = 1).
    Exact averages at time t."""
    e = np.linspace(x0, x1, n + 1) - u * t
    dx = (x1 - x0) / n
    w = k * np.pi
    rbar = 1.0 - amp * (np.cos(w * e[1:]) - np.cos(w * e[:-1])) / (w * dx)
    rv = amp * (np.sin(w * e[1:]) - np.sin(w * e[:-1])) / dx
    Wbar = np.stack([rbar, u * rbar, 1.0 / (gamma - 1) + 0.5 * u * u * rbar])
    V = np.stack([rv, u * rv, 0.5 * u * u * rv])
    return np.ascontiguousarray(np.stack([Wbar, V]))


def shock_sine_1d(n: int, gamma=GAMMA):
    """Mach-3 shock at x = -4 moving right into rho = 1 + 0.2 sin(5x) at rest,
    p = 1, on (-5, 5) (sec. 5, the Shu-Osher example).  n a multiple of 10
    puts the shock on a cell edge; each cell's averages come from its own
    side (derivative averages over the open cell)."""
    assert n % 10 == 0
    post = (3.857143, 2.629369, 10.333333)
    x0, x1 = -5.0, 5.0
    e = np.linspace(x0, x1, n + 1)
    dx = (x1 - x0) / n

    def fun(x, left):
        rho = np.where(left, post[0], 1.0 + 0.2 * np.sin(5 * x))
        u = np.where(left, post[1], 0.0)
        p = np.where(left, post[2], 1.0)
        return prim_to_cons(rho, u, p, gamma=gamma)

    left = (0.5 * (e[:-1] + e[1:]) < -4.0)
    xq, wq = _gl_nodes(e[:-1], e[1:])
    Wbar = (np.asarray(fun(xq, left[:, None])) * wq).sum(-1)
    V = (np.asarray(fun(e[1:], left)) - np.asarray(fun(e[:-1], left))) / dx
    return np.ascontiguousarray(np.stack([Wbar, V]))


def riemann_1d(n: int, left, right, x0=0.0, x1=1.0, xd=0.5, gamma=GAMMA):
    """Piecewise-constant Euler data, left/right = (rho, u, p), jump at xd."""
    e = np.linspace(x0, x1, n + 1)
    dx = (x1 - x0) / n
    WL = prim_to_cons(*left, gamma=gamma)
    WR = prim_to_cons(*right, gamma=gamma)
    frac_left = np.clip((xd - e[:-1]) / dx, 0.0, 1.0)          # share of cell left of xd
    Wbar = WL[:, None] * frac_left + WR[:, None] * (1.0 - frac_left)
    V = np.zeros_like(Wbar)
    inside = (e[:-1] < xd) & (e[1:] > xd)                       # jump strictly inside
    V[:, inside] = ((WR - WL) / dx)[:, None]
    return np.ascontiguousarray(np.stack([Wbar, V]))


def piecewise_1d(n: int, states, breaks, x0, x1, gamma=GAMMA):
    """Piecewise-constant Euler data: states[k] = (rho, u, p) on the k-th
    interval between x0, the sorted breaks and x1.  Averages by covered
    length; the derivative average of a cell is the sum of the jumps strictly
    inside it over dx (a jump on a cell edge contributes nothing)."""
    e = np.linspace(x0, x1, n + 1)
    dx = (x1 - x0) / n
    Ws = [prim_to_cons(*s, gamma=gamma) for s in states]
    bounds = [x0, *breaks, x1]
    Wbar = np.zeros((3, n))
    for W, a, b in zip(Ws, bounds[:-1], bounds[1:]):
        share = np.clip((np.minimum(e[1:], b) - np.maximum(e[:-1], a)) / dx, 0.0, 1.0)
        share[(e[:-1] >= a) & (e[1:] <= b)] = 1.0          # whole cells exactly
        Wbar += W[:, None] * share
    V = np.zeros_like(Wbar)
    for k, xb in enumerate(breaks):
        inside = (e[:-1] < xb) & (e[1:] > xb)
        V[:, inside] += ((Ws[k + 1] - Ws[k]) / dx)[:, None]
    return np.ascontiguousarray(np.stack([Wbar, V]))


def lax_tube(n: int, gamma=GAMMA):
    """Lax's shock tube (sec. 5): (0.445, 0.698, 3.528) for x < 0 and
    (0.5, 0, 0.571) for x > 0 on (-5, 5); inflow/outflow (transmissive) ends,
    T = 1.3."""
    return piecewise_1d(n, [(0.445, 0.698, 3.528), (0.5, 0.0, 0.571)], [0.0], -5.0, 5.0, gamma)


def blast_waves(n: int, gamma=GAMMA):
    """Interacting blast waves of Woodward and Colella (sec. 5): rho = 1, u = 0
    and p = 1000 on [0, 0.1), 0.01 on [0.1, 0.9), 100 on [0.9, 1]; reflective
    walls, T = 0.038."""
    return piecewise_1d(n, [(1.0, 0.0, 1000.0), (1.0, 0.0, 0.01), (1.0, 0.0, 100.0)],
                        [0.1, 0.9], 0.0, 1.0, gamma)


# ---------------------------------------------------------------------------
# 2D
# ---------------------------------------------------------------------------

def averages_2d(fun, x0, x1, y0, y1, nx, ny, xbreak=None, max_points=1 << 24):
    """Exact-quadrature averages (W, V, Y, Z) of fun -> (m, ...) on a uniform
    nx x ny grid.  Without xbreak, fun(x, y) must be smooth.  With xbreak, fun
    may jump across the vertical line x = xbreak and is called as
    fun(x, y, side), side = -1 / +1 selecting the piece left / right of it
    (so points on the line are unambiguous).  Large grids go by blocks of
    rows of at most max_points quadrature points."""
    ey = np.linspace(y0, y1, ny + 1)
    rows = max(1, max_points // (nx * len(_GL_W) ** 2))
    if ny > rows:
        parts = [_averages_2d_rows(fun, x0, x1, ey[r:min(r + rows, ny) + 1], nx, (y1 - y0) / ny,
                                   xbreak) for r in range(0, ny, rows)]
        return np.ascontiguousarray(np.concatenate(parts, axis=-2))
    return _averages_2d_rows(fun, x0, x1, ey, nx, (y1 - y0) / ny, xbreak)


def _averages_2d_rows(fun, x0, x1, ey, nx, dy, xbreak):
    """averages_2d on the rows between the edges ey."""
    ex = np.linspace(x0, x1, nx + 1)
    ny = len(ey) - 1
    dx = (x1 - x0) / nx
    a, b = ex[:-1], ex[1:]
    if xbreak is None:
        pieces = [(a, b, np.zeros(nx))]
        f = lambda x, y, s: np.asarray(fun(x, y))
    else:
        cut = np.clip(xbreak, a, b)                  # per cell: split point
        pieces = [(a, cut, -np.ones(nx)), (cut, b, np.ones(nx))]
        f = lambda x, y, s: np.asarray(fun(x, y, s))
    edge_l = np.where(a < xbreak, -1.0, 1.0) if xbreak is not None else np.zeros(nx)
    edge_r = np.where(b <= xbreak, -1.0, 1.0) if xbreak is not None else np.zeros(nx)
    gy, wy = _gl_nodes(ey[:-1], ey[1:])              # (ny, q), (q,)
    q = gy.shape[1]
    Wbar = 0.0
    Yacc = 0.0
    for pa, pb, side in pieces:
        gx, wx = _gl_nodes(pa, pb)                   # (nx, q)
        frac = (pb - pa) / dx                        # (nx,)
        X = np.broadcast_to(gx[None, :, None, :], (ny, nx, q, q))
        Y = np.broadcast_to(gy[:, None, :, None], (ny, nx, q, q))
        S = np.broadcast_to(side[None, :, None, None], (ny, nx, q, q))
        w2 = wy[None, None, :, None] * wx[None, None, None, :] * frac[None, :, None, None]
        Wbar = Wbar + (f(X, Y, S) * w2).sum((-1, -2))
        Xe = np.broadcast_to(gx[None, :, :], (ny, nx, q))
        Se = np.broadcast_to(side[None, :, None], (ny, nx, q))
        Yh = np.broadcast_to(ey[1:, None, None], (ny, nx, q))
        Yl = np.broadcast_to(ey[:-1, None, None], (ny, nx, q))
        w1 = wx[None, None, :] * frac[None, :, None]
        Yacc = Yacc + ((f(Xe, Yh, Se) - f(Xe, Yl, Se)) * w1).sum(-1)
    Yq = np.broadcast_to(gy[:, None, :], (ny, nx, q))
    XL = np.broadcast_to(a[None, :, None], (ny, nx, q))
    XR = np.broadcast_to(b[None, :, None], (ny, nx, q))
    SL = np.broadcast_to(edge_l[None, :, None], (ny, nx, q))
    SR = np.broadcast_to(edge_r[None, :, None], (ny, nx, q))
    V = ((f(XR, Yq, SR) - f(XL, Yq, SL)) * wy).sum(-1) / dx
    Xl = np.broadcast_to(a[None, :], (ny, nx))
    Xr = np.broadcast_to(b[None, :], (ny, nx))
    Ylo = np.broadcast_to(ey[:-1, None], (ny, nx))
    Yhi = np.broadcast_to(ey[1:, None], (ny, nx))
    sl = np.broadcast_to(edge_l[None, :], (ny, nx))
    sr = np.broadcast_to(edge_r[None, :], (ny, nx))
    Z = (f(Xr, Yhi, sr) - f(Xl, Yhi, sl) - f(Xr, Ylo, sr) + f(Xl, Ylo, sl)) / (dx * dy)
    return np.ascontiguousarray(np.stack([Wbar, V, Yacc / dy, Z]))


def density_wave_2d(nx: int, ny: int | None = None, t: float = 0.0, gamma=GAMMA,
                    L: float = 2.0):
    """rho = 1 + 0.2 sin(pi (x + y - 2t)), u = v = 1, p = 1 on periodic
    (0, 2)^2 (sec. 5, the 2D accuracy example).  Exact averages at time t."""
    ny = nx if ny is None else ny

    def fun(x, y):
        r = 1.0 + 0.2 * np.sin(np.pi * (x + y - 2.0 * t))
        return prim_to_cons(r, 1.0, 1.0, 1.0, gamma)

    return averages_2d(fun, 0.0, L, 0.0, L, nx, ny)


def density_wave_2d_exact_rho(nx, ny=None, t=0.0, L=2.0):
    """Exact density cell averages (closed form) of the 2D density wave: the
    average of sin(pi (x + y)) over a cell is
    4 sin(pi dx/2) sin(pi dy/2) sin(pi (xc + yc)) / (pi^2 dx dy), free of the
    cancellation of a corner difference on fine meshes."""
    ny = nx if ny is None else ny
    dx, dy = L / nx, L / ny
    xc = (np.arange(nx) + 0.5) * dx - t
    yc = (np.arange(ny) + 0.5) * dy - t
    k = 4.0 * np.sin(np.pi * dx / 2) * np.sin(np.pi * dy / 2) / (np.pi ** 2 * dx * dy)
    return 1.0 + 0.2 * k * np.sin(np.pi * (xc[None, :] + yc[:, None]))


def isentropic_vortex(n: int, t: float = 0.0, gamma=GAMMA, L=10.0):
    """Isentropic vortex on periodic (0,10)^2 moving with (1,1) (sec. 5)."""
    def fun(x, y):
        xs = np.mod(x - t - 0.0, L)
        ys = np.mod(y - t - 0.0, L)
        # nearest periodic image of the centre (5,5)
        dxc = xs - 5.0
        dyc = ys - 5.0
        r2 = dxc ** 2 + dyc ** 2
        T = 1.0 - 25.0 * (gamma - 1.0) / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
        rho = T ** (1.0 / (gamma - 1.0))
        u = 1.0 - 5.0 / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2)) * dyc
        v = 1.0 + 5.0 / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2)) * dxc
        p = rho ** gamma
        return prim_to_cons(rho, u, p, v, gamma)
    return averages_2d(fun, 0.0, L, 0.0, L, n, n)


def four_quadrant(n: int, quads, gamma=GAMMA):
    """Four-quadrant Riemann data on (0,1)^2 split at (0.5, 0.5); quads =
    primitive (rho, u, v, p) for the quadrants (x>.5,y>.5), (x<.5,y>.5),
    (x<.5,y<.5), (x>.5,y<.5).  n even puts the splits on cell edges."""
    assert n % 2 == 0
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc)
    rho, u, v, p = (np.empty((n, n)) for _ in range(4))
    masks = [(X > .5) & (Y > .5), (X < .5) & (Y > .5), (X < .5) & (Y < .5), (X > .5) & (Y < .5)]
    for msk, q in zip(masks, quads):
        rho[msk], u[msk], v[msk], p[msk] = q
    W = prim_to_cons(rho, u, p, v, gamma)
    z = np.zeros_like(W)
    return np.ascontiguousarray(np.stack([W, z, z.copy(), z.copy()]))


def shock_sine_2d(nx: int, ny: int, gamma=GAMMA):
    """Mach-3 shock moving right into rho = 1 + 0.2 sin(5x) sin(3y) at rest,
    p = 1, on (-5,5) x (0, 2pi/3) (the 2D shock/sine workload; post-shock
    state of sec. 5, Shu-Osher example).  Exact averages in closed form (the
    field is separable): W, and V, Y, Z as differences of edge and corner
    values; the cell holding x = -4 splits into its post-shock and its
    sine part, and its V carries the jump."""
    post = prim_to_cons(3.857143, 2.629369, 10.333333, 0.0, gamma)
    x0, x1, y0, y1, xs = -5.0, 5.0, 0.0, 2.0 * np.pi / 3.0, -4.0
    ex, ey = np.linspace(x0, x1, nx + 1), np.linspace(y0, y1, ny + 1)
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    a, b = ex[:-1], ex[1:]
    lo = np.clip(xs, a, b)                            # start of the sine part
    f_sine = (b - lo) / dx                            # its share of the cell
    # x integrals of the sine part over [lo, b] / dx, and edge values
    Sx = (np.cos(5 * lo) - np.cos(5 * b)) / (5 * dx)
    # edge values: an edge left of the shock (or on it, for the cell to its
    # left) belongs to the post-shock part
    sin_b = np.where(b > xs, np.sin(5 * b), 0.0)
    sin_a = np.where(a >= xs, np.sin(5 * a), 0.0)
    Sy = (np.cos(3 * ey[:-1]) - np.cos(3 * ey[1:])) / (3 * dy)
    Dy = (np.sin(3 * ey[1:]) - np.sin(3 * ey[:-1])) / dy
    rest = prim_to_cons(1.0, 0.0, 1.0, 0.0, gamma)    # the field without its density wave
    W = np.empty((4, ny, nx))
    V, Y, Z = (np.zeros((4, ny, nx)) for _ in range(3))
    for c in range(4):
        W[c] = (1.0 - f_sine)[None, :] * post[c] + f_sine[None, :] * rest[c]
    W[0] += 0.2 * Sx[None, :] * Sy[:, None]
    # x-derivative averages: (value at b - value at a) / dx, with the jump
    for c in range(4):
        va = np.where(a < xs, post[c], rest[c])
        vb = np.where(b > xs, rest[c], post[c])
        V[c] = ((vb - va) / dx)[None, :] + np.zeros((ny, 1))
    V[0] += 0.2 * ((sin_b - sin_a) / dx)[None, :] * Sy[:, None]
    Y[0] = 0.2 * Sx[None, :] * Dy[:, None]
    Z[0] = 0.2 * ((sin_b - sin_a) / dx)[None, :] * Dy[:, None]
    return np.ascontiguousarray(np.stack([W, V, Y, Z]))


# ---------------------------------------------------------------------------
# batched workloads
# ---------------------------------------------------------------------------

@dataclass
class Instance1D:
    n: int
    x0: float
    x1: float
    left: tuple      # (rho, u, p)
    right: tuple
    T: float

    @property
    def dx(self):
        return (self.x1 - self.x0) / self.n

    def state(self, gamma=GAMMA):
        return riemann_1d(self.n, self.left, self.right, self.x0, self.x1, 0.5 * (self.x0 + self.x1), gamma)


def riemann_batch_1d(count: int = 4096, seed: int = SEED, nmin: int = 200, nmax: int = 2000,
                     T: float = 0.14):
    """Independent 1D Euler Riemann problems on [0,1]: N even, uniform in
    {nmin..nmax}; rho, p ~ U[0.1, 2], u ~ U[-1, 1] on each side; jump at 0.5."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 2 * rng.integers(nmin // 2, nmax // 2 + 1, size=count)
    rho = rng.uniform(0.1, 2.0, size=(count, 2))
    u = rng.uniform(-1.0, 1.0, size=(count, 2))
    p = rng.uniform(0.1, 2.0, size=(count, 2))
    return [Instance1D(int(n[i]), 0.0, 1.0, (rho[i, 0], u[i, 0], p[i, 0]),
                       (rho[i, 1], u[i, 1], p[i, 1]), T) for i in range(count)]


@dataclass
class Instance2D:
    n: int
    quads: list
    T: float

    def state(self, gamma=GAMMA):
        return four_quadrant(self.n, self.quads, gamma)


def four_quadrant_batch(count: int = 256, seed: int = SEED + 5, T: float = 0.25,
                        nmin: int = 128, nmax: int = 1024):
    """Four-quadrant problems on (0,1)^2 with n = 128 * U{1..8} (square),
    per-quadrant rho, p ~ U[0.1, 1.5], u, v ~ U[-1, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(nmin // 128, nmax // 128 + 1, size=count)
    out = []
    for i in range(count):
        q = [(rng.uniform(0.1, 1.5), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.1, 1.5))
             for _ in range(4)]
        out.append(Instance2D(int(128 * k[i]), q, T))
    return out
