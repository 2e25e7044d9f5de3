"""GPU tests of the learned troubled-cell gate: the BF16 matrix-core network
against the FP64 oracle network, the FP32 training gradient against the
oracle gradient, Adam, the features and labels the method generates, the
gate's limits (all-full = plain, all-linear = linear weights), and a trained
gate that keeps the plain method's error while passing smooth cells."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2304_09724_amd as S
from paper_2304_09724_amd import gate as GT
from paper_2304_09724_amd import workloads as WL

pytestmark = pytest.mark.gpu


def bf16(x):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32)
    u += np.uint32(0x7FFF) + ((u >> 16) & 1)
    u &= np.uint32(0xFFFF0000)
    return a.astype(np.float64)


def packed(params):
    return torch.from_numpy(S.gate_pack(params)).cuda()


def test_matrix_core_layout_is_exact():
    """Weights and inputs chosen so that every product and every hidden value
    is exact in BF16/FP32: the network must reproduce the FP64 oracle
    exactly, which pins the operand and accumulator layouts."""
    rng = np.random.default_rng(0)
    p = np.zeros(S.GATE_NPARAMS, dtype=np.float32)
    p[:256] = rng.choice([-1.0, 0.0, 1.0], size=256)
    p[256:288] = rng.choice([-0.5, 0.0, 0.5], size=32)
    p[288:1312] = rng.choice([-1.0, 0.0, 1.0], size=1024)
    p[1312:1344] = rng.choice([-1.0, 0.0, 1.0], size=32)
    p[1344:1376] = rng.choice([-0.25, 0.0, 0.5], size=32)
    p[1376] = 0.75
    X = rng.choice([0.0, 0.5, 1.0, 1.5, 2.0], size=(200, 8)).astype(np.float32)
    z = S.mlp_logits(torch.from_numpy(X).cuda(), packed(p)).cpu().numpy()
    want = O.mlp_forward(p.astype(np.float64), X.astype(np.float64))
    np.testing.assert_allclose(z, want, rtol=0, atol=1e-5)


def test_logits_match_oracle_within_bf16():
    rng = np.random.default_rng(1)
    p = GT.init_params(3)
    X = rng.normal(size=(1000, 8)).astype(np.float32)
    z = S.mlp_logits(torch.from_numpy(X).cuda(), packed(p)).cpu().numpy()
    pr = p.astype(np.float64).copy()
    pr[:256] = bf16(p[:256])
    pr[288:1312] = bf16(p[288:1312])
    want = O.mlp_forward(pr, bf16(X))
    # the only other rounding is the first hidden layer's BF16 input to layer 2
    assert np.abs(z - want).max() < 0.03 * (1 + np.abs(want).max())


def test_training_gradient_matches_oracle():
    rng = np.random.default_rng(2)
    p = GT.init_params(5)
    X = rng.normal(size=(2000, 8)).astype(np.float32)
    y = (rng.uniform(size=2000) < 0.2).astype(np.float32)
    loss, g = S.mlp_grad(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(),
                         torch.from_numpy(p).cuda(), pos_weight=4.0)
    lo, go = O.mlp_backward(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64), 4.0)
    assert abs(float(loss.item()) - lo) < 1e-5 * abs(lo)
    g = g.cpu().numpy()
    assert np.abs(g - go).max() < 1e-4 * np.abs(go).max()


def test_adam_step():
    rng = np.random.default_rng(3)
    p = rng.normal(size=S.GATE_NPARAMS).astype(np.float32)
    g = rng.normal(size=S.GATE_NPARAMS).astype(np.float32)
    pt, gt = torch.from_numpy(p.copy()).cuda(), torch.from_numpy(g).cuda()
    m, v = torch.zeros_like(pt), torch.zeros_like(pt)
    S.mlp_adam(pt, gt, m, v, 1, 1e-2)
    # step 1 of Adam moves every parameter by lr * g / (|g| + eps)
    want = p - 1e-2 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(pt.cpu().numpy(), want, rtol=1e-5, atol=1e-7)


def test_features_and_labels_match_oracle():
    insts = WL.riemann_batch_1d(count=4, seed=3, nmin=60, nmax=120)
    meshes = [S.Mesh.line(d.n, d.x0, d.x1, S.BC_TRANSMISSIVE) for d in insts]
    s = S.Solver(meshes, S.Params.make(eq=S.EULER))
    for i, d in enumerate(insts):
        s.set_state(i, d.state())
    s.advance_to(0.02)
    f, lab = s.gate_data()
    f, lab = f.cpu().numpy(), lab.cpu().numpy()
    cfg = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4)
    off = 0
    for i, d in enumerate(insts):
        st = s.get_state(i)
        fo = O.gate_features1d(st, d.dx, O.BC_TRANSMISSIVE)
        lo = O.gate_labels1d(cfg, st, d.dx)
        np.testing.assert_allclose(f[off:off + d.n], fo, rtol=0, atol=2e-6)
        assert np.array_equal(lab[off:off + d.n], lo)
        assert lo.any() and not lo.all()
        off += d.n


@pytest.mark.parametrize("b3,mode", [(40.0, S.W_NONLINEAR), (-40.0, S.W_LINEAR)])
def test_learned_gate_limits(b3, mode):
    """A gate that calls every cell troubled gives the plain method bit for
    bit (on a Riemann problem); one that calls every cell smooth gives the
    linear-weight scheme (on the smooth density wave, which linear weights
    can run)."""
    p = np.zeros(S.GATE_NPARAMS, dtype=np.float32)
    p[1376] = b3
    if b3 > 0:
        d = WL.riemann_batch_1d(count=1, seed=9, nmin=100, nmax=100)[0]
        m = [S.Mesh.line(d.n, d.x0, d.x1, S.BC_TRANSMISSIVE)]
        st = d.state()
    else:
        m = [S.Mesh.line(64, 0.0, 2.0, S.BC_PERIODIC)]
        st = WL.density_wave_1d(64)
    a = S.Solver(m, S.Params.make(eq=S.EULER, weights=S.W_LEARNED, gate_threshold=0.5))
    a.gate_load(p)
    a.set_state(0, st)
    a.advance_to(0.05, max_steps=20)
    b = S.Solver(m, S.Params.make(eq=S.EULER, weights=mode))
    b.set_state(0, st)
    b.advance_to(0.05, max_steps=20)
    assert np.array_equal(a.get_state(0), b.get_state(0))


def exact_rho(d, t, sub=16):
    e = np.linspace(d.x0, d.x1, d.n + 1)
    xs = e[:-1, None] + (np.arange(sub) + 0.5) / sub * d.dx
    out = np.empty(xs.shape)
    for j in range(d.n):
        for k in range(sub):
            out[j, k] = O.exact_riemann(1.4, d.left, d.right, (xs[j, k] - 0.5) / t)[0][0]
    return out.mean(axis=1)


def extrema(r, range_):
    d = np.diff(r)
    big = np.abs(d) > 1e-6 * range_
    s = np.sign(d[big])
    return int((s[1:] != s[:-1]).sum())


def test_trained_gate_keeps_the_error_of_the_plain_method():
    X, y = GT.collect(GT.training_problems(), times=[0.0, 0.02, 0.06, 0.1, 0.14])
    assert 0.01 < float(y.mean()) < 0.5
    params, hist = GT.train(X, y, steps=500)
    assert hist[-1] < 0.5 * hist[0]
    # held-out problems from the batched workload's distribution
    val = WL.riemann_batch_1d(count=12, seed=1234, nmin=100, nmax=400)
    meshes = [S.Mesh.line(d.n, d.x0, d.x1, S.BC_TRANSMISSIVE) for d in val]
    plain = S.Solver(meshes, S.Params.make(eq=S.EULER))
    gated = S.Solver(meshes, S.Params.make(eq=S.EULER, weights=S.W_LEARNED, gate_threshold=0.1))
    gated.gate_load(params)
    for i, d in enumerate(val):
        plain.set_state(i, d.state())
        gated.set_state(i, d.state())
    plain.advance_to(0.14, raise_nonphysical=False)
    gated.advance_to(0.14, raise_nonphysical=False)
    okp, okg = plain.instance_status() == 0, gated.instance_status() == 0
    l1p, l1g = [], []
    for i, d in enumerate(val):
        if not (okp[i] and okg[i]):
            continue
        ex = exact_rho(d, 0.14)
        rp, rg = plain.get_state(i)[0, 0], gated.get_state(i)[0, 0]
        l1p.append(np.abs(rp - ex).mean())
        l1g.append(np.abs(rg - ex).mean())
        rng_ = ex.max() - ex.min()
        assert extrema(rg, rng_) <= extrema(rp, rng_) + 2, i
    assert len(l1p) >= 8
    assert np.sum(l1g) <= 1.05 * np.sum(l1p)
    # the gate must actually pass most cells as smooth
    z = S.mlp_logits(X[:200000].contiguous(), packed(params)).cpu().numpy()
    assert (1.0 / (1.0 + np.exp(-z)) < 0.1).mean() > 0.5
