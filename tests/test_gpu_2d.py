"""GPU parity of the 2D path (x-sweep + y-sweep kernels, device-side time
loop) against the CPU oracle: relative L-infinity per quantity (W, V, Y, Z)
<= 1e-11."""
import numpy as np
import pytest

import oracle as O
import paper_2304_09724_amd as S
from paper_2304_09724_amd import workloads as WL
from tests.golden.load import table

pytestmark = pytest.mark.gpu
TOL = 1e-11


def rel_err(g, o):
    errs = []
    for q in range(o.shape[0]):
        scale = max(np.abs(o[q]).max(), 1e-300)
        errs.append(np.abs(g[q] - o[q]).max() / scale)
    return max(errs)


def smooth_state(nx, ny, seed, lx=1.0, ly=1.0):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx * lx
    y = (np.arange(ny) + 0.5) / ny * ly
    X, Y = np.meshgrid(x, y)
    ph = rng.uniform(0, 6, 4)
    rho = 1 + 0.3 * np.sin(2 * np.pi * X / lx + ph[0]) * np.cos(2 * np.pi * Y / ly + ph[1])
    u = 0.3 * np.cos(2 * np.pi * Y / ly + ph[2])
    v = -0.2 * np.sin(2 * np.pi * X / lx + ph[3])
    p = 1 + 0.1 * np.cos(2 * np.pi * (X / lx - Y / ly))
    W = WL.prim_to_cons(rho, u, p, v)
    # derivative averages: random but moderate (the step does not need them consistent)
    V = rng.normal(size=W.shape) * 0.2
    Yd = rng.normal(size=W.shape) * 0.2
    Z = rng.normal(size=W.shape) * 0.1
    return np.ascontiguousarray(np.stack([W, V, Yd, Z]))


def ocfg(bcx=O.BC_PERIODIC, bcy=O.BC_PERIODIC, weights=O.W_NONLINEAR, charwise=True,
         eq=O.EULER, a=1.0, b=0.0):
    return O.Config(eq=eq, bc=(bcx, bcx, bcy, bcy), weights=weights, charwise=charwise,
                    adv_a=a, adv_b=b)


def gparams(weights=S.W_NONLINEAR, charwise=True, eq=S.EULER, a=1.0, b=0.0, cfl=0.9):
    return S.Params.make(eq=eq, weights=weights, charwise=charwise, adv_a=a, adv_b=b, cfl=cfl)


def one_step(nx, ny, bcx, bcy, st, dt, weights=S.W_NONLINEAR, charwise=True, flags=None,
             eq=S.EULER, a=1.0, b=0.0):
    s = S.Solver([S.Mesh.rect(nx, ny, 0.0, 1.0, 0.0, 1.0, bcx, bcy)],
                 gparams(weights, charwise, eq, a, b))
    s.set_state(0, st)
    if flags is not None:
        s.set_flags(0, flags)
    s.step([dt])
    return s.get_state(0)


@pytest.mark.parametrize("nx,ny", [(3, 3), (4, 5), (59, 4), (60, 3), (61, 7), (64, 5),
                                   (121, 3), (5, 61), (7, 64)])
@pytest.mark.parametrize("bc", [S.BC_PERIODIC, S.BC_TRANSMISSIVE, S.BC_REFLECTIVE])
def test_single_step_tile_edges_and_boundaries(nx, ny, bc):
    st = smooth_state(nx, ny, nx * 100 + ny + bc)
    dt = 0.1 / max(nx, ny)
    g = one_step(nx, ny, bc, bc, st, dt)
    o, bad = O.step2d(ocfg(bc, bc), st, 1.0 / nx, 1.0 / ny, dt)
    assert not bad
    assert rel_err(g, o) < TOL


@pytest.mark.parametrize("scale", [1e-8, 1e8])
def test_scaled_states_steps(scale):
    """As in 1D: density, momenta and energy times one factor keep every
    velocity and sound speed, while the sweeps' reciprocals and square roots
    work at another exponent.  Five fixed steps on a 61 x 64 mesh (ragged in
    both tile directions), against the oracle on the same scaled data."""
    nx, ny = 61, 64
    st = smooth_state(nx, ny, 17) * scale
    dt = 0.2 / max(nx, ny)
    s = S.Solver([S.Mesh.rect(nx, ny, 0.0, 1.0, 0.0, 1.0, S.BC_PERIODIC, S.BC_TRANSMISSIVE)],
                 gparams())
    s.set_state(0, st)
    o = st
    for _ in range(5):
        s.step([dt])
        o, bad = O.step2d(ocfg(O.BC_PERIODIC, O.BC_TRANSMISSIVE), o, 1.0 / nx, 1.0 / ny, dt)
        assert not bad
    assert rel_err(s.get_state(0), o) < TOL


def test_mixed_boundaries():
    nx, ny = 23, 17
    st = smooth_state(nx, ny, 3)
    dt = 0.005
    g = one_step(nx, ny, S.BC_REFLECTIVE, S.BC_TRANSMISSIVE, st, dt)
    o, _ = O.step2d(ocfg(O.BC_REFLECTIVE, O.BC_TRANSMISSIVE), st, 1.0 / nx, 1.0 / ny, dt)
    assert rel_err(g, o) < TOL


@pytest.mark.parametrize("weights,charwise", [(S.W_LINEAR, True), (S.W_NONLINEAR, False),
                                              (S.W_GATED, True), (S.W_GATED, False)])
def test_weight_modes(weights, charwise):
    """Each compiled instance of the sweeps against the oracle on a
    four-quadrant problem, three steps: the paper's scheme with the
    characteristic path off, linear weights, and per-cell flags (40 % set)
    with the characteristic path on and off."""
    n = 24
    quads = [(1.1, 0.0, 0.0, 1.1), (0.5065, 0.8939, 0.0, 0.35), (1.1, 0.8939, 0.8939, 1.1),
             (0.5065, 0.0, 0.8939, 0.35)]
    st = WL.four_quadrant(n, quads)
    rng = np.random.default_rng(4)
    flags = (rng.uniform(size=n * n) < 0.4).astype(np.uint8)
    s = S.Solver([S.Mesh.rect(n, n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE, S.BC_TRANSMISSIVE)],
                 gparams(weights, charwise))
    s.set_state(0, st)
    if weights == S.W_GATED:
        s.set_flags(0, flags)
    dt = 0.2 / n
    for _ in range(3):
        s.step([dt])
    g = s.get_state(0)
    cfg = ocfg(O.BC_TRANSMISSIVE, O.BC_TRANSMISSIVE, weights, charwise)
    o = st
    for _ in range(3):
        o, bad = O.step2d(cfg, o, 1.0 / n, 1.0 / n, dt, flags if weights == S.W_GATED else None)
    assert rel_err(g, o) < TOL


@pytest.mark.parametrize("n", [10, 20])
def test_density_wave_full_run(n):
    """2D Euler density wave (sec. 5, first 2D example) to T = 1, CFL 0.9:
    GPU and oracle agree after the whole run, and the GPU error matches the
    paper's table entry within the oracle's own agreement."""
    st = WL.density_wave_2d(n)
    s = S.Solver([S.Mesh.rect(n, n, 0.0, 2.0, 0.0, 2.0)], gparams())
    s.set_state(0, st)
    steps = s.advance_to(1.0)
    g = s.get_state(0)
    o, t, osteps, bad = O.advance2d(ocfg(), st, 2.0 / n, 2.0 / n, 0.9, 1.0)
    assert steps[0] == osteps
    assert rel_err(g, o) < TOL
    tg, _ = s.times()
    assert tg[0] == 1.0


def test_isentropic_vortex_full_run_parity():
    """The isentropic vortex (sec. 5) at 20^2 to T = 10 (118 CFL steps): the
    GPU's whole run against the oracle's, on the nonlinear smooth case in
    which density, both velocities and pressure all vary."""
    n = 20
    st = WL.isentropic_vortex(n)
    s = S.Solver([S.Mesh.rect(n, n, 0.0, 10.0, 0.0, 10.0)], gparams())
    s.set_state(0, st)
    steps = s.advance_to(10.0)
    o, t, osteps, bad = O.advance2d(ocfg(), st, 10.0 / n, 10.0 / n, 0.9, 10.0)
    assert not bad and steps[0] == osteps
    assert rel_err(s.get_state(0), o) < TOL


def test_isentropic_vortex_paper_table():
    """Table isotro on the GPU at 40^2 .. 320^2 in one ragged batch (periodic
    (0,10)^2, T = 10, CFL 0.9; the exact averages at T are the initial ones):
    density L1 and L2 within 6% of the paper's (the oracle's own agreement at
    20^2 and 40^2 is 2.5-5%), Linf within 25%, and fifth order between
    successive meshes as the table prints it (4.8, 4.9, 4.8)."""
    ns = [40, 80, 160, 320]
    s = S.Solver([S.Mesh.rect(n, n, 0.0, 10.0, 0.0, 10.0) for n in ns], gparams())
    init = [WL.isentropic_vortex(n) for n in ns]
    for i, st in enumerate(init):
        s.set_state(i, st)
    s.advance_to(np.full(len(ns), 10.0))
    tg, _ = s.times()
    assert np.all(tg == 10.0)
    ref = table("isentropic_vortex")
    l1 = []
    for i, n in enumerate(ns):
        e = s.get_state(i)[0, 0] - init[i][0, 0]
        got = np.array([np.abs(e).mean(), np.sqrt((e ** 2).mean()), np.abs(e).max()])
        print(n, got, ref[n])
        np.testing.assert_allclose(got[:2], ref[n][:2], rtol=0.06)
        np.testing.assert_allclose(got[2], ref[n][2], rtol=0.25)
        l1.append(got[0])
    orders = np.log2(np.array(l1[:-1]) / np.array(l1[1:]))
    assert np.all(orders > 4.5), orders


def test_positivity_safeguard_2d_against_oracle():
    """The safeguard in 2D (not in the paper): the four-quadrant data of the
    batch's instance 75, which fail at step 4 under the paper's scheme, run 12
    steps on a periodic 16^2 grid and 8 steps on a transmissive 64^2 grid; the
    GPU matches the oracle's runs with the same safeguard step for step."""
    quads = WL.four_quadrant_batch(count=256)[75].quads
    for n, bc, steps in ((16, S.BC_PERIODIC, 12), (64, S.BC_TRANSMISSIVE, 8)):
        st = WL.four_quadrant(n, quads)
        s = S.Solver([S.Mesh.rect(n, n, 0.0, 1.0, 0.0, 1.0, bc, bc)],
                     S.Params.make(eq=S.EULER, positivity=True))
        s.set_state(0, st)
        k = s.advance_to(1.0, max_steps=steps)
        assert k[0] == steps and s.instance_status()[0] == 0
        obc = O.BC_PERIODIC if bc == S.BC_PERIODIC else O.BC_TRANSMISSIVE
        cfg = O.Config(eq=O.EULER, bc=(obc,) * 4, positivity=True)
        o, t, osteps, bad = O.advance2d(cfg, st, 1.0 / n, 1.0 / n, 0.9, 1.0, max_steps=steps)
        assert not bad and osteps == steps
        assert rel_err(s.get_state(0), o) < TOL, n


def test_positivity_safeguard_2d_unchanged_where_not_needed():
    """A ragged batch of smooth states runs bit for bit the same with the
    safeguard on and off."""
    sizes = [(12, 20), (70, 9), (33, 33)]
    runs = []
    for pos in (False, True):
        s = S.Solver([S.Mesh.rect(nx, ny, 0.0, 1.0, 0.0, 1.0) for nx, ny in sizes],
                     S.Params.make(eq=S.EULER, positivity=pos))
        for i, (nx, ny) in enumerate(sizes):
            s.set_state(i, smooth_state(nx, ny, seed=i))
        s.advance_to(np.full(len(sizes), 1.0), max_steps=5)
        runs.append([s.get_state(i) for i in range(len(sizes))])
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)


def test_positivity_safeguard_2d_batch_failures():
    """Four-quadrant problems of the batch (n <= 384), run to t = 0.25: three of
    the first 64 meet a non-physical state under the paper's scheme; with the
    safeguard two of them complete.  The third (instance 120, 384^2) still
    stops at step 3: next to the quadrants' corner a cell's update with the
    first-order HLLE flux on all four faces is itself non-physical at CFL 0.9
    (sum form), and the oracle with the same safeguard stops at the same step."""
    insts = WL.four_quadrant_batch(count=256)
    pick = [i for i, d in enumerate(insts) if d.n <= 384][:64]
    sub = [insts[i] for i in pick]
    meshes = [S.Mesh.rect(d.n, d.n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE, S.BC_TRANSMISSIVE)
              for d in sub]
    failed, steps = [], []
    for pos in (False, True):
        s = S.Solver(meshes, S.Params.make(eq=S.EULER, positivity=pos))
        for k, d in enumerate(sub):
            s.set_state(k, d.state())
        steps.append(s.advance_to(np.full(len(sub), 0.25), raise_nonphysical=False))
        failed.append({pick[k] for k in np.nonzero(s.instance_status())[0]})
    print(f"failures without the safeguard {sorted(failed[0])}, with it {sorted(failed[1])}")
    assert failed[0] == {75, 120, 126}
    assert failed[1] == {120}
    d = insts[120]
    cfg = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4, positivity=True)
    o, t, osteps, bad = O.advance2d(cfg, d.state(), 1.0 / d.n, 1.0 / d.n, 0.9, 0.25, max_steps=3)
    assert bad and osteps == 3 and steps[1][pick.index(120)] == 3


def test_advection_2d():
    n = 16
    st = smooth_state(n, n, 9)[:, :1].copy()          # one component
    g = one_step(n, n, S.BC_PERIODIC, S.BC_PERIODIC, st, 0.01, eq=S.ADVECTION, a=1.0, b=0.5)
    o, _ = O.step2d(ocfg(eq=O.ADVECTION, a=1.0, b=0.5), st, 1.0 / n, 1.0 / n, 0.01)
    assert rel_err(g, o) < TOL


def test_step_cfl_is_compute_dt_then_step():
    """2D: one device-sized CFL step equals shw_compute_dt followed by
    shw_step, bit for bit, on a ragged batch."""
    sizes = [(12, 20), (70, 9), (33, 33)]
    meshes = [S.Mesh.rect(nx, ny, 0.0, 1.0, 0.0, 1.0) for nx, ny in sizes]
    states = [smooth_state(nx, ny, seed=k) for k, (nx, ny) in enumerate(sizes)]
    a, b = (S.Solver(meshes, gparams()) for _ in range(2))
    for s in (a, b):
        for i, st in enumerate(states):
            s.set_state(i, st)
    dt = a.compute_dt()
    a.step(dt)
    b.step_cfl()
    for i in range(len(sizes)):
        np.testing.assert_array_equal(a.get_state(i), b.get_state(i))
    t, steps = b.times()
    np.testing.assert_array_equal(t, dt)
    assert np.all(steps == 1)


def test_compute_dt_matches_oracle():
    st = smooth_state(13, 9, 5, lx=2.0)
    s = S.Solver([S.Mesh.rect(13, 9, 0.0, 2.0, 0.0, 1.0)], gparams())
    s.set_state(0, st)
    dt = s.compute_dt()[0]
    want = O.dt2d(ocfg(), st, 2.0 / 13, 1.0 / 9, 0.9)
    assert dt == pytest.approx(want, rel=1e-14)


def test_ragged_batch_of_quadrant_problems():
    """Three four-quadrant problems of different sizes in one batch (the
    batched 2D workload's recipe, small meshes), each advanced with its own
    CFL steps to t = 0.05."""
    insts = WL.four_quadrant_batch(count=3, seed=11, nmin=128, nmax=128)
    sizes = [16, 24, 20]
    meshes = [S.Mesh.rect(n, n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE, S.BC_TRANSMISSIVE)
              for n in sizes]
    s = S.Solver(meshes, gparams())
    states = [WL.four_quadrant(n, d.quads) for n, d in zip(sizes, insts)]
    for i, st in enumerate(states):
        s.set_state(i, st)
    steps = s.advance_to(0.05, raise_nonphysical=False)
    codes = s.instance_status()
    cfg = ocfg(O.BC_TRANSMISSIVE, O.BC_TRANSMISSIVE)
    n_bad = 0
    for i, (n, st) in enumerate(zip(sizes, states)):
        o, t, osteps, bad = O.advance2d(cfg, st, 1.0 / n, 1.0 / n, 0.9, 0.05)
        # the unlimited scheme cannot continue some random problems: both sides
        # must stop on the same one at the same step
        assert (codes[i] != 0) == bad, i
        assert steps[i] == osteps, i
        n_bad += bad
        if not bad:
            assert rel_err(s.get_state(i), o) < TOL, i
    assert n_bad < len(sizes)


def test_transpose_symmetry_on_gpu():
    """x <-> y exchange of the data gives the exchanged result (both sweep
    kernels see the same arithmetic)."""
    nx, ny = 19, 26
    st = smooth_state(nx, ny, 21)
    tr = np.ascontiguousarray(st[[0, 2, 1, 3]][:, [0, 2, 1, 3]].transpose(0, 1, 3, 2))
    a = one_step(nx, ny, S.BC_PERIODIC, S.BC_PERIODIC, st, 0.004)
    s = S.Solver([S.Mesh.rect(ny, nx, 0.0, 1.0, 0.0, 1.0)], gparams())
    s.set_state(0, tr)
    s.step([0.004])
    b = s.get_state(0)
    bt = b[[0, 2, 1, 3]][:, [0, 2, 1, 3]].transpose(0, 1, 3, 2)
    assert rel_err(a, bt) < 1e-12


@pytest.mark.parametrize("weights", [S.W_NONLINEAR, S.W_LEARNED])
def test_graph_replays_match_eager_launches(weights):
    """The 2D time loop's captured chunk (8 steps as one HIP graph) against
    the same kernels launched one by one: each call below is exactly one
    replay, checked bit for bit, with eager work of the program (state round
    trips, a torch op, synchronisations) between the replays."""
    import torch
    from paper_2304_09724_amd import gate as GT
    sizes = [24, 40, 32]
    insts = WL.four_quadrant_batch(count=3, seed=11)
    meshes = [S.Mesh.rect(n, n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE, S.BC_TRANSMISSIVE)
              for n in sizes]
    prm = S.Params.make(eq=S.EULER, weights=weights, gate_threshold=0.3)
    a, b = S.Solver(meshes, prm), S.Solver(meshes, prm)
    b.set_graphs(False)
    for s in (a, b):
        if weights == S.W_LEARNED:
            s.gate_load(GT.init_params(3))
        for i, (n, d) in enumerate(zip(sizes, insts)):
            s.set_state(i, WL.four_quadrant(n, d.quads))
    for rep in range(6):
        ka = a.advance_to(1.0, max_steps=8, raise_nonphysical=False)
        kb = b.advance_to(1.0, max_steps=8, raise_nonphysical=False)
        assert np.array_equal(ka, kb), rep
        for i in range(len(sizes)):
            assert np.array_equal(a.get_state(i), b.get_state(i)), (rep, i)
        ta, sa = a.times()
        tb, sb = b.times()
        assert np.array_equal(ta, tb) and np.array_equal(sa, sb)
        # eager work between replays
        x = a.get_state(1)
        a.set_state(1, x)
        b.set_state(1, b.get_state(1))
        a.state.mul_(1.0)
        torch.cuda.synchronize()
    assert ka.sum() > 0


def test_tile_variants_and_autotuner():
    """Every tile variant (1, 2, 4 lines of 60 cells) gives the same result
    bit for bit, graphs on; the autotuner picks one and leaves state and times
    as they were."""
    sizes = [24, 70, 46]
    insts = WL.four_quadrant_batch(count=3, seed=11)
    meshes = [S.Mesh.rect(n, n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE, S.BC_TRANSMISSIVE)
              for n in sizes]
    ref = None
    for v in (0, 1, 2):
        s = S.Solver(meshes, gparams())
        assert s.get_tile() == 2
        s.set_tile(v)
        for i, (n, d) in enumerate(zip(sizes, insts)):
            s.set_state(i, WL.four_quadrant(n, d.quads))
        steps = s.advance_to(0.03, raise_nonphysical=False)
        got = [s.get_state(i) for i in range(len(sizes))]
        if ref is None:
            ref = (steps, got)
        else:
            assert np.array_equal(steps, ref[0])
            for a, b in zip(got, ref[1]):
                assert np.array_equal(a, b)
    before = [s.get_state(i) for i in range(len(sizes))]
    t0, k0 = s.times()
    best, ms = s.autotune(steps=8)
    assert best in (0, 1, 2) and s.get_tile() == best and min(ms) > 0
    t1, k1 = s.times()
    assert np.array_equal(t0, t1) and np.array_equal(k0, k1)
    for i in range(len(sizes)):
        assert np.array_equal(s.get_state(i), before[i])
    # and it keeps stepping as before
    s.advance_to(0.04, raise_nonphysical=False)


def test_autotuner_restores_nonphysical_flags():
    """An instance that turns non-physical during the autotuner's probe steps
    (a four-quadrant problem that fails at its fourth step on 24^2 cells) is
    restored with its state: afterwards the batch steps bit for bit as a
    fresh context with the same tile does, and nothing is reported."""
    bad_quads = WL.four_quadrant_batch(count=16, seed=11)[12].quads
    ok_quads = WL.four_quadrant_batch(count=3, seed=11)[1].quads
    sizes = [46, 24]
    meshes = [S.Mesh.rect(n, n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE, S.BC_TRANSMISSIVE)
              for n in sizes]
    states = [WL.four_quadrant(46, ok_quads), WL.four_quadrant(24, bad_quads)]
    o = O.advance2d(O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4), states[1], 1 / 24, 1 / 24,
                    0.9, 10.0, max_steps=8)
    assert o[3] and 2 < o[2] < 8                  # fails inside the probe, not before
    runs = []
    for tune in (True, False):
        s = S.Solver(meshes, gparams())
        for i, st in enumerate(states):
            s.set_state(i, st)
        if tune:
            best, _ = s.autotune(steps=8)
            assert np.all(s.instance_status() == 0)
        else:
            s.set_tile(best)
        steps = s.advance_to(10.0, max_steps=2, raise_nonphysical=False)
        assert np.array_equal(steps, [2, 2]) and np.all(s.instance_status() == 0)
        runs.append([s.get_state(i) for i in range(2)])
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_ragged_batch_matches_instances_run_alone():
    """Instances of a batch that finish at different times (own mesh sizes and
    end times): each step's sweeps run only the tiles of the instances still
    advancing, renumbered and spread over the XCDs.  Every instance's state
    and step count equal those of the same instance advanced alone, bit for
    bit, with graphs on."""
    insts = WL.four_quadrant_batch(count=6, seed=23)
    sizes = [64, 18, 130, 40, 96, 22]
    ends = [0.02, 0.05, 0.01, 0.04, 0.03, 0.005]
    meshes = [S.Mesh.rect(n, n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE, S.BC_TRANSMISSIVE)
              for n in sizes]
    states = [WL.four_quadrant(n, d.quads) for n, d in zip(sizes, insts)]
    b = S.Solver(meshes, gparams())
    for i, st in enumerate(states):
        b.set_state(i, st)
    steps = b.advance_to(np.array(ends), raise_nonphysical=False)
    codes = b.instance_status()
    assert len(set(steps.tolist())) > 3            # they do finish at different steps
    for i, (m, st) in enumerate(zip(meshes, states)):
        a = S.Solver([m], gparams())
        a.set_state(0, st)
        k = a.advance_to(ends[i], raise_nonphysical=False)
        assert k[0] == steps[i] and a.instance_status()[0] == codes[i], i
        assert np.array_equal(a.get_state(0), b.get_state(i)), i
