"""Pins of the oracle's gate network: the FP64 gradient against central
finite differences of its own loss (an independent route to the derivative)
and the loss against a direct numpy evaluation of the network."""
import numpy as np

import oracle as O


def numpy_logits(p, X):
    W1 = p[:256].reshape(32, 8)
    b1 = p[256:288]
    W2 = p[288:1312].reshape(32, 32)
    b2 = p[1312:1344]
    w3 = p[1344:1376]
    b3 = p[1376]
    h1 = np.maximum(X @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    return h2 @ w3 + b3


def test_forward_matches_numpy():
    rng = np.random.default_rng(0)
    p = rng.normal(size=O.N_PARAMS) * 0.3
    X = rng.normal(size=(50, 8))
    np.testing.assert_allclose(O.mlp_forward(p, X), numpy_logits(p, X), rtol=1e-12, atol=1e-12)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = rng.normal(size=O.N_PARAMS) * 0.3
    X = rng.normal(size=(40, 8))
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


def test_labels_flag_jumps_not_smooth_data():
    from paper_2304_09724_amd import workloads as WL
    cfg = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4)
    st = WL.riemann_1d(100, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    lab = O.gate_labels1d(cfg, st, 0.01)
    assert lab[48:52].any() and not lab[:40].any() and not lab[60:].any()
    smooth = WL.density_wave_1d(100)
    assert not O.gate_labels1d(O.Config(eq=O.EULER), smooth, 0.02).any()


def test_features_of_constant_state_are_the_floor():
    from paper_2304_09724_amd import workloads as WL
    W = WL.prim_to_cons(np.full(10, 1.0), np.full(10, 0.5), np.full(10, 1.0))
    st = np.stack([W, np.zeros_like(W)])
    f = O.gate_features1d(st, 0.1)
    np.testing.assert_allclose(f, np.log2(1e-12) / 32, rtol=1e-12)
