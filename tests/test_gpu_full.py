"""GPU parity at the workloads' full sizes.

1D: the 4096-problem Riemann batch in one persistent launch to t = 0.14 (the
benchmark's launch), 24 instances sampled across the deciles of the mesh size
plus the largest, the smallest and one that turns non-physical, each re-run
whole by the oracle.

2D: 20 CFL steps of the whole mesh or batch, in two ways: with the 8-step HIP
graphs the benchmark replays (advance_to), and step by step from the host
(the step sizes are read back and handed to the oracle); the two end bit for
bit alike.  The oracle then takes the same 20 steps on windows around sampled
cells: a cell's result after k steps depends only on cells within 2k of it
(each step reads two cells each way), so the centre of a window of radius
2k + 1 is the oracle's exact answer.  Tolerances (tests/tolerances.py) are
relative L-infinity per plane: 1e-11 on the cell averages W; on the derivative
averages V, Y, Z bounds set above the floor at which two valid rounding
orders of the oracle itself already differ (measured in
tests/test_oracle_rounding.py).  Every comparison prints its per-quantity
error."""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import torch

import oracle as O
import paper_2304_09724_amd as S
from paper_2304_09724_amd import gate as GT
from paper_2304_09724_amd import workloads as WL
from tests.tolerances import FULL_2D, TOL

pytestmark = pytest.mark.gpu
STEPS = 20
WORKERS = min(16, os.cpu_count() or 1)


def rel_err(g, o):
    errs = []
    for q in range(o.shape[0]):
        scale = max(np.abs(o[q]).max(), 1e-300)
        errs.append(np.abs(g[q] - o[q]).max() / scale)
    return max(errs)


@pytest.mark.timeout(900)
def test_bench_batch_sampled_instances():
    insts = WL.riemann_batch_1d(count=4096, T=0.14)
    meshes = [S.Mesh.line(d.n, d.x0, d.x1, S.BC_TRANSMISSIVE) for d in insts]
    s = S.Solver(meshes, S.Params.make(eq=S.EULER, cfl=0.9))
    init = torch.from_numpy(np.concatenate([d.state().reshape(-1) for d in insts])).cuda()
    s.state.copy_(init)
    s.set_times(np.zeros(len(insts)))
    steps = s.advance_to(np.full(len(insts), 0.14), raise_nonphysical=False)
    codes = s.instance_status()
    ns = np.array([d.n for d in insts])
    rng = np.random.default_rng(5)
    # three from each eighth of the instances ordered by mesh size
    order = np.argsort(ns, kind="stable")
    pick = set()
    for part in np.array_split(order, 8):
        pick |= {int(i) for i in rng.choice(part, 3, replace=False)}
    pick |= {int(np.argmax(ns)), int(np.argmin(ns)), int(np.nonzero(codes != 0)[0][0])}
    cfg = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4)

    def one(i):
        return O.advance1d(cfg, insts[i].state(), insts[i].dx, 0.9, 0.14)

    pick = sorted(pick, key=lambda i: -ns[i])          # longest first
    with cf.ThreadPoolExecutor(WORKERS) as ex:
        res = dict(zip(pick, ex.map(one, pick)))
    worst = 0.0
    for i, (o, t, osteps, bad) in res.items():
        assert (codes[i] != 0) == bool(bad), i
        assert steps[i] == osteps, i
        if not bad:
            e = rel_err(s.get_state(i), o)
            worst = max(worst, e)
            assert e < TOL, (i, e)
    print(f"{len(res)} instances (N {min(ns[list(res)])}..{max(ns[list(res)])}), worst {worst:.2e}")
    assert len(res) >= 24


def window(st, i, j, r, wrap_x, wrap_y):
    """Cells (j - r .. j + r, i - r .. i + r) of a (4, m, ny, nx) array (or of a
    (ny, nx) one)."""
    ny, nx = st.shape[-2:]
    ii = np.arange(i - r, i + r + 1)
    jj = np.arange(j - r, j + r + 1)
    ii = ii % nx if wrap_x else ii
    jj = jj % ny if wrap_y else jj
    assert ii.min() >= 0 and ii.max() < nx and jj.min() >= 0 and jj.max() < ny
    return np.ascontiguousarray(st[..., jj, :][..., ii]), ii, jj


def plane_scales(state):
    """Largest |value| of each plane (q, component) of a (4, 4, ny, nx) state;
    the momentum components share the largest momentum magnitude."""
    size = np.abs(state).max(axis=(-1, -2))
    size[:, 1:3] = np.sqrt(state[:, 1] ** 2 + state[:, 2] ** 2).max(axis=(-1, -2))[:, None]
    return size


def check_windows(label, init, gpu_state, cells, dx, dy, dts, wrap_x, wrap_y, flags=None):
    """Oracle steps (sizes dts) of windows around the cells against the GPU's
    values, per plane; flags: per step (ny, nx) gate decisions (GATED mode)."""
    r = 2 * len(dts) + 1
    weights = O.W_NONLINEAR if flags is None else O.W_GATED
    cfg = O.Config(eq=O.EULER, bc=(O.BC_PERIODIC,) * 4, weights=weights)
    scale = plane_scales(gpu_state)
    worst = np.zeros(4)
    for i, j in cells:
        w, ii, jj = window(init, i, j, r, wrap_x, wrap_y)
        for k, dt in enumerate(dts):
            fw = None
            if flags is not None:
                fw = window(flags[k], i, j, r, wrap_x, wrap_y)[0].reshape(-1)
            w, bad = O.step2d(cfg, w, dx, dy, dt, fw)
        err = np.abs(w[:, :, r, r] - gpu_state[:, :, j, i]) / np.maximum(scale, 1e-300)
        worst = np.maximum(worst, err.max(axis=1))
    print(f"{label}: {len(cells)} windows, {len(dts)} steps, per-plane error W V Y Z "
          + " ".join(f"{e:.2e}" for e in worst), flush=True)
    for q, name in enumerate("WVYZ"):
        assert worst[q] < FULL_2D[name], (label, name, worst[q])


def stepwise(s, nsteps, flags=False):
    """nsteps device-CFL steps one call at a time: returns per-step step sizes
    (n_inst,) and, if asked, the gate decisions each step used (instance 0)."""
    dts, fl = [], []
    t_prev = s.times()[0]
    for _ in range(nsteps):
        s.step_cfl(raise_nonphysical=False)
        t = s.times()[0]
        dts.append(t - t_prev)
        t_prev = t
        if flags:
            fl.append(s.get_flags(0))
    return np.array(dts), fl


def run_both(meshes, params, states, network=None, flags=False):
    """The 20 steps as the benchmark launches them (graph chunks) and step by
    step; asserts the two agree bit for bit and returns the second solver,
    its step sizes and flags."""
    out = []
    for mode in ("graph", "stepwise"):
        s = S.Solver(meshes, params)
        if network is not None:
            s.gate_load(network)
        for i, st in enumerate(states):
            s.set_state(i, st)
        if mode == "graph":
            steps = s.advance_to(np.full(len(meshes), 1e9), max_steps=STEPS,
                                 raise_nonphysical=False)
            codes = s.instance_status()
            assert np.all(steps[codes == 0] == STEPS)
            ref = [s.get_state(i) for i in range(len(meshes))]
            del s
            torch.cuda.empty_cache()
        else:
            dts, fl = stepwise(s, STEPS, flags)
            for i in range(len(meshes)):
                if codes[i] == 0:
                    assert np.array_equal(s.get_state(i), ref[i]), i
            assert np.array_equal(s.instance_status(), codes)
            return s, dts, fl, codes


@pytest.mark.timeout(900)
def test_density_wave_1024():
    n = 1024
    st = WL.density_wave_2d(n)
    s, dts, _, _ = run_both([S.Mesh.rect(n, n, 0.0, 2.0, 0.0, 2.0)], S.Params.make(eq=S.EULER),
                            [st])
    g = s.get_state(0)
    rng = np.random.default_rng(1)
    cells = [(0, 0), (n - 1, n - 1), (3, n - 2)] + [tuple(rng.integers(0, n, 2)) for _ in range(3)]
    check_windows("density wave 1024^2", st, g, cells, 2.0 / n, 2.0 / n, dts[:, 0], True, True)


@pytest.fixture(scope="module")
def network():
    X, y = GT.collect(GT.training_problems(), times=[0.0, 0.02, 0.06, 0.1, 0.14])
    return GT.train(X, y)[0]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("learned", [False, True])
def test_shock_sine_4096x1024(learned, network):
    """The shock/sine shape, plain and with the learned gate (the oracle
    takes the gate's decisions of each step as flags)."""
    nx, ny = 4096, 1024
    st = WL.shock_sine_2d(nx, ny)
    m = [S.Mesh.rect(nx, ny, -5.0, 5.0, 0.0, 2 * np.pi / 3, S.BC_TRANSMISSIVE, S.BC_PERIODIC)]
    if learned:
        p = S.Params.make(eq=S.EULER, weights=S.W_LEARNED, gate_threshold=0.05)
    else:
        p = S.Params.make(eq=S.EULER)
    s, dts, fl, _ = run_both(m, p, [st], network if learned else None, flags=learned)
    g = s.get_state(0)
    if learned:
        assert all(0 < f.mean() < 0.2 for f in fl)
    dx, dy = 10.0 / nx, (2 * np.pi / 3) / ny
    shock = int(round(1.0 / dx))                    # x = -4
    rng = np.random.default_rng(2)
    cells = [(shock, 5), (shock + 1, ny - 1), (shock - 2, 300), (shock + 30, 77), (2000, 0)]
    cells += [(int(rng.integers(50, nx - 50)), int(rng.integers(0, ny))) for _ in range(2)]
    check_windows(f"shock/sine 4096x1024 {'learned' if learned else 'plain'}", st, g, cells,
                  dx, dy, dts[:, 0], False, True, fl if learned else None)


@pytest.mark.timeout(1200)
def test_four_quadrant_batch_256():
    insts = WL.four_quadrant_batch(count=256)
    meshes = [S.Mesh.rect(d.n, d.n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE, S.BC_TRANSMISSIVE)
              for d in insts]
    s, dts, _, codes = run_both(meshes, S.Params.make(eq=S.EULER), [d.state() for d in insts])
    ns = np.array([d.n for d in insts])
    ok = np.nonzero(codes == 0)[0]
    rng = np.random.default_rng(3)
    pick = {int(ok[np.argmax(ns[ok])]), int(ok[np.argmin(ns[ok])])}
    pick |= {int(i) for i in rng.choice(ok, 3, replace=False)}
    for k in sorted(pick):
        n = insts[k].n
        g = s.get_state(k)
        h = n // 2
        cells = [(h, h), (h - 1, h + 2), (int(rng.integers(42, n - 42)), int(rng.integers(42, n - 42)))]
        check_windows(f"four-quadrant #{k} {n}^2", insts[k].state(), g, cells, 1.0 / n, 1.0 / n,
                      dts[:, k], False, False)


def test_density_wave_order_under_refinement():
    """The 2D density wave to t = 2 (CFL 0.9) at 128^2, 256^2, 512^2: the L1
    error of the density against the exact averages falls at the scheme's
    fifth order (1024^2 sits at the FP64 floor)."""
    errs = []
    for n in (128, 256, 512):
        s = S.Solver([S.Mesh.rect(n, n, 0.0, 2.0, 0.0, 2.0)], S.Params.make(eq=S.EULER))
        s.set_state(0, WL.density_wave_2d(n))
        s.advance_to(2.0)
        ex = WL.density_wave_2d_exact_rho(n, t=2.0)
        errs.append(np.abs(s.get_state(0)[0, 0] - ex).mean())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[0] < 1e-8
    assert np.all(orders > 4.5), (errs, orders)
