"""Pins of the oracle's gate network: the FP64 gradient against central
finite differences of its own loss (an independent route to the derivative)
and the loss against a direct numpy evaluation of the network."""
import numpy as np

import oracle as O


NF = 16


def numpy_logits(p, X):
    o = 32 * NF
    W1 = p[:o].reshape(32, NF)
    b1 = p[o:o + 32]
    W2 = p[o + 32:o + 1056].reshape(32, 32)
    b2 = p[o + 1056:o + 1088]
    w3 = p[o + 1088:o + 1120]
    b3 = p[o + 1120]
    h1 = np.maximum(X @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    return h2 @ w3 + b3


def test_forward_matches_numpy():
    rng = np.random.default_rng(0)
    p = rng.normal(size=O.N_PARAMS) * 0.3
    X = rng.normal(size=(50, NF))
    np.testing.assert_allclose(O.mlp_forward(p, X), numpy_logits(p, X), rtol=1e-12, atol=1e-12)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = rng.normal(size=O.N_PARAMS) * 0.3
    X = rng.normal(size=(40, NF))
    y = (rng.uniform(size=40) < 0.3).astype(float)
    loss, g = O.mlp_backward(p, X, y, pos_weight=4.0)
    z = numpy_logits(p, X)
    w = np.where(y > 0.5, 4.0, 1.0)
    direct = np.mean(w * (np.logaddexp(0, z) - y * z))
    assert abs(loss - direct) < 1e-12
    idx = rng.choice(O.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(O.N_PARAMS)
        e[i] = h
        lp, _ = O.mlp_backward(p + e, X, y, 4.0)
        lm, _ = O.mlp_backward(p - e, X, y, 4.0)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_parameter_count():
    assert O.N_PARAMS == 32 * NF + 32 + 32 * 32 + 32 + 32 + 1 == 1633


TR = (O.BC_TRANSMISSIVE,) * 4
RF = (O.BC_REFLECTIVE,) * 4


def euler_state(rho, u, p, V=None, gamma=1.4):
    """(2, 3, n) state from primitive cell values; derivative averages V
    (3, n) or zero."""
    rho, u, p = (np.asarray(a, dtype=float) for a in (rho, u, p))
    W = np.stack([rho, rho * u, p / (gamma - 1) + 0.5 * rho * u * u])
    return np.stack([W, np.zeros_like(W) if V is None else np.asarray(V, dtype=float)])


def test_features_of_a_linear_density_profile():
    """rho = 1 + 0.1 x, u = 0, p = 1: averages are the centre values and every
    derivative average is 0.1, so dl = dr = gm = gp = 0.1 dx for density and
    momentum/energy are flat."""
    n, dx = 12, 0.05
    x = (np.arange(n) + 0.5) * dx
    V = np.zeros((3, n))
    V[0] = 0.1
    st = euler_state(1 + 0.1 * x, np.zeros(n), np.ones(n), V)
    f = O.gate_features1d(O.Config(eq=O.EULER, bc=TR), st, dx)
    floor = np.log2(1e-12) / 32
    for j in range(2, n - 2):
        np.testing.assert_allclose(f[j, 0:4], 0.25, rtol=1e-12)
        np.testing.assert_allclose(f[j, 4], np.log2((0.4 * dx) ** 2 + 1e-12) / 32, rtol=1e-12)
        np.testing.assert_array_equal(f[j, 5:9], 0.0)
        np.testing.assert_array_equal(f[j, 10:14], 0.0)
        np.testing.assert_allclose(f[j, [9, 14]], floor, rtol=1e-12)
        assert f[j, 15] == 0.0


def test_features_order_and_signs():
    """A density step (dl = 0, dr = -0.5 at the cell left of it), hand-set
    neighbour derivatives (gm = 3 dx, gp = -dx) and u = c on the left (last
    feature 1/2; on the right c = sqrt(2) u, so 1 / (1 + sqrt(2)))."""
    n, dx = 10, 0.1
    rho = np.where(np.arange(n) < 5, 1.0, 0.5)
    V = np.zeros((3, n))
    V[2, 1], V[2, 3] = 3.0, -1.0
    c = np.sqrt(1.4)
    st = euler_state(rho, np.full(n, c), np.ones(n), V)
    f = O.gate_features1d(O.Config(eq=O.EULER, bc=TR), st, dx)
    np.testing.assert_allclose(f[4, 0:4], [0.0, -1.0, 0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(f[4, 4], np.log2(0.25 + 1e-12) / 32, rtol=1e-12)
    # energy of cell 2: flat averages, derivative averages 3 (left), -1 (right)
    np.testing.assert_allclose(f[2, 10:14], [0.0, 0.0, 0.75, -0.25], atol=1e-15)
    np.testing.assert_allclose(f[2, 14], np.log2((4 * dx) ** 2 + 1e-12) / 32, rtol=1e-12)
    np.testing.assert_allclose(f[:5, 15], 0.5, rtol=1e-12)
    np.testing.assert_allclose(f[5:, 15], 1 / (1 + np.sqrt(2)), rtol=1e-12)


def test_features_see_the_reflective_ghost():
    """Constant rho, p and u > 0 next to a reflective wall: the ghost carries
    the opposite momentum, so the momentum jump to the left is 2 rho u."""
    n, dx = 8, 0.1
    st = euler_state(np.full(n, 2.0), np.full(n, 0.5), np.ones(n))
    f = O.gate_features1d(O.Config(eq=O.EULER, bc=RF), st, dx)
    np.testing.assert_allclose(f[0, 5:9], [1.0, 0.0, 0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(f[0, 9], np.log2(2.0 ** 2 + 1e-12) / 32, rtol=1e-12)
    np.testing.assert_allclose(f[n - 1, 5:9], [0.0, -1.0, 0.0, 0.0], atol=1e-15)
    np.testing.assert_array_equal(f[3, 5:9], 0.0)


def test_labels_flag_exactly_the_stencils_across_a_jump():
    """A flat stencil has zero smoothness indicators, hence exactly the linear
    weights; the two cells whose stencils straddle the jump get a quartic
    weight far below its linear one."""
    from paper_2304_09724_amd import workloads as WL
    cfg = O.Config(eq=O.EULER, bc=TR)
    st = WL.riemann_1d(100, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    for level in (0.5, 0.99, 0.999):
        lab = O.gate_labels1d(cfg, st, 0.01, level)
        assert list(np.nonzero(lab)[0]) == [49, 50]


def test_labels_of_ghost_cells_follow_the_boundary():
    n = 8
    st = euler_state(np.full(n, 2.0), np.full(n, 0.5), np.ones(n))
    lab = O.gate_labels1d(O.Config(eq=O.EULER, bc=RF), st, 0.1, 0.99, cells=range(-1, n + 1))
    assert list(lab) == [1, 1] + [0] * (n - 2) + [1, 1]
    lab = O.gate_labels1d(O.Config(eq=O.EULER, bc=TR), st, 0.1, 0.99, cells=range(-1, n + 1))
    assert not lab.any()


def test_labels_nest_with_the_level():
    """The label condition w0 < L * gamma0 can only gain cells as L grows."""
    from paper_2304_09724_amd import workloads as WL
    cfg = O.Config(eq=O.EULER, bc=TR)
    d = WL.riemann_batch_1d(count=1, seed=5, nmin=120, nmax=120)[0]
    st, _, _, bad = O.advance1d(cfg, d.state(), d.dx, 0.9, 0.05)
    assert not bad
    prev = None
    for level in (0.5, 0.9, 0.99, 0.999, 1.0):
        lab = O.gate_labels1d(cfg, st, d.dx, level)
        if prev is not None:
            assert np.all(lab >= prev)
        prev = lab
    assert 0 < prev.sum() < len(prev)


def test_smooth_data_have_no_labels():
    from paper_2304_09724_amd import workloads as WL
    for n in (40, 100):
        st = WL.density_wave_1d(n)
        assert not O.gate_labels1d(O.Config(eq=O.EULER), st, 2.0 / n, 0.999).any()


def test_2d_features_on_y_independent_data_are_the_1d_ones():
    """With v = 0 and nothing varying in y, the features along x of every row
    are the 1D features of (rho, m_x, E); along y every shape is zero."""
    from paper_2304_09724_amd import workloads as WL
    n, ny, dx, dy = 20, 4, 0.1, 0.3
    rho = 1 + 0.3 * np.sin(np.arange(n) * 0.7)
    u = 0.2 + 0.1 * np.cos(np.arange(n))
    p = 1 + 0.2 * np.sin(np.arange(n) * 1.3)
    V = np.random.default_rng(1).normal(size=(3, n))
    st1 = euler_state(rho, u, p, V)
    st2 = np.zeros((4, 4, ny, n))
    for qd in range(2):
        for k2, k1 in ((0, 0), (1, 1), (3, 2)):
            st2[qd, k2] = st1[qd, k1][None, :]
    cfg1 = O.Config(eq=O.EULER, bc=TR)
    cfg2 = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE, O.BC_TRANSMISSIVE, O.BC_PERIODIC,
                                    O.BC_PERIODIC))
    f1 = O.gate_features1d(cfg1, st1, dx)
    fx = O.gate_features2d(cfg2, st2, dx, dy, 0)
    fy = O.gate_features2d(cfg2, st2, dx, dy, 1)
    for j in range(ny):
        np.testing.assert_allclose(fx[j], f1, rtol=1e-13, atol=1e-15)
    shape = [0, 1, 2, 3, 5, 6, 7, 8, 10, 11, 12, 13]
    np.testing.assert_array_equal(fy[:, :, shape], 0.0)
    np.testing.assert_array_equal(fy[:, :, 15], 0.0)       # no normal velocity in y


def test_2d_features_transpose():
    """Features along y of a state equal the features along x of its
    transpose (x <-> y, m_x <-> m_y, V <-> Y), including ghost cells."""
    rng = np.random.default_rng(2)
    nx, ny = 7, 5
    st = rng.uniform(0.5, 1.5, size=(4, 4, ny, nx))
    st[0, 3] += 3.0                                       # keep the pressure positive
    tr = np.ascontiguousarray(st.transpose(0, 1, 3, 2))[[0, 2, 1, 3]][:, [0, 2, 1, 3]]
    bc = (O.BC_TRANSMISSIVE, O.BC_PERIODIC, O.BC_REFLECTIVE, O.BC_TRANSMISSIVE)
    bct = (bc[2], bc[3], bc[0], bc[1])
    fy = O.gate_features2d(O.Config(eq=O.EULER, bc=bc), st, 0.1, 0.2, 1)
    fxt = O.gate_features2d(O.Config(eq=O.EULER, bc=bct), tr, 0.2, 0.1, 0)
    np.testing.assert_allclose(fy, fxt.transpose(1, 0, 2), rtol=1e-13, atol=1e-15)
