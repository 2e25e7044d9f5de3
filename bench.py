#!/usr/bin/env python3
"""Throughput of batched ADER-SHWENO time stepping on one MI355X.

Headline workload: 256 independent 2D Euler four-quadrant Riemann problems
on [0,1]^2 (the paper's 2D Riemann example, sec. 5, with seeded states),
meshes n x n with n = 128 * U{1..8} (1.16e8 cells in all), per-quadrant rho,
p ~ U[0.1, 1.5] and u, v ~ U[-1, 1], transmissive boundaries, gamma 1.4, CFL
0.9, the paper's scheme (nonlinear weights, characteristic reconstruction).
All instances advance together: per step the device computes each
instance's CFL step, the x- and y-sweep kernels run over every instance's
tiles, and the steps are replayed in chunks of 8 as captured HIP graphs.
One bench step = one CFL time step of every instance of the batch (one pass
of the whole hot path over the batch); W untimed warm-up steps from t = 0,
then K timed steps.  Inputs are resident in HBM before the timed region.

The same line carries the learned-gate run of the same batch and window
(with the gated-vs-plain L1 error on a seeded subset against 2x-refined
reference runs), the 1D batch (4096 Riemann problems to t = 0.14), the
1024^2 density wave, the 4096 x 1024 shock/sine problem (plain and gated),
the FP64 roofline of the sweeps and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/sec FP64 (plain vs learned-gated, batched) at fixed L1 error"
FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X, dense FP64 vector
HBM_PEAK_GBS = 8000.0
GATE_THRESHOLD = 0.05
C5_COUNT = 2 ** 8
C2_COUNT = 4096
C2_T = 0.14
C4_T = 1.8


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---- counted HBM traffic (profiles/) -----------------------------------------
# Bytes per launch from two counter runs (FETCH_SIZE and WRITE_SIZE scaled by a
# 1 GiB copy), valid only for the kernel code those runs measured: the sources
# compared without their comments and with whitespace collapsed.
KERNEL_SOURCES_1D = ["sweep1d.hip", "shw_kernels.h", "sweep1d_math.h", "shw_math.h",
                     "gate_math.h", "lanes.h"]
KERNEL_SOURCES_2D = ["sweep2d.hip", "shw_kernels.h", "sweep2d_math.h", "shw_math.h",
                     "gate_math.h", "lanes.h", "ck2d_gen.h"]


def kernel_fingerprint(sources):
    import hashlib
    import re
    # string literals kept, // and /* */ comments dropped, whitespace runs as one blank
    token = re.compile(r'"(?:\\.|[^"\\])*"|//[^\n]*|/\*.*?\*/', re.S)
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2304_09724_amd", "csrc", f)) as fh:
            text = token.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", fh.read())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(profile, sources, key="hbm_bytes_per_launch"):
    """Counted HBM bytes recorded in a profiles/ summary, or None if the
    kernel changed since the counters were taken."""
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("kernel_sources_sha256_16:", key + ":")))
    if fields.get("kernel_sources_sha256_16", "").strip() != kernel_fingerprint(sources):
        return None
    try:
        return float(fields[key])
    except (KeyError, ValueError):
        return None


def flops_2d(full=True):
    from paper_2304_09724_amd import flopcount
    return flopcount.euler2d_cell_update(full)["flops"]


def flops_1d():
    from paper_2304_09724_amd import flopcount
    return flopcount.euler1d_cell_update()["flops"]


def roofline_alu(flops_per_cu, cu, ms, kernel, traffic=None, algo_bytes=None):
    tf = flops_per_cu * cu / (ms * 1e-3) / 1e12
    out = {"bound": "alu", "achieved": round(tf, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4),
           "traffic": traffic, "kernel": kernel, "kernel_ms": round(ms, 3),
           "flops_per_cell_update": flops_per_cu}
    if algo_bytes is not None:
        gbs = algo_bytes * cu / (ms * 1e-3) / 1e9
        out["hbm_algorithmic_GBs"] = round(gbs, 1)
        out["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    return out


# ---- the learned gate ----------------------------------------------------------

def train_gate():
    from paper_2304_09724_amd import gate as GT
    log("gate: training data and training ...")
    t0 = time.perf_counter()
    X, y = GT.collect(GT.training_problems(), times=[0.0, 0.02, 0.06, 0.1, 0.14])
    params, hist = GT.train(X, y)
    return params, {"samples": int(X.shape[0]), "adam_steps": 800,
                    "loss_first_last": [hist[0], hist[-1]],
                    "seconds": round(time.perf_counter() - t0, 2)}


# ---- 2D batch of four-quadrant problems (headline) ------------------------------

def c5_meshes(S, insts):
    return [S.Mesh.rect(d.n, d.n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE, S.BC_TRANSMISSIVE)
            for d in insts]


def c5_window(S, insts, params, warmup, steps, gate=None, autotune_steps=2):
    """Warm-up steps from t = 0, then `steps` timed CFL steps of the whole
    batch; HIP events on the solver's stream bracket the timed advance."""
    import torch
    s = S.Solver(c5_meshes(S, insts), params, device="cuda:0")
    if gate is not None:
        s.gate_load(gate)
    for i, d in enumerate(insts):
        s.set_state(i, d.state())
    tile, tile_ms = s.autotune(steps=autotune_steps)
    ncell = np.array([d.n * d.n for d in insts], dtype=np.int64)
    s.advance_to(np.full(len(insts), 1e9), max_steps=warmup, raise_nonphysical=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s.stream)
    k = s.advance_to(np.full(len(insts), 1e9), max_steps=steps, raise_nonphysical=False)
    e1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    cu = int((ncell * k).sum())
    res = {"value": cu / wall, "cell_updates": cu, "wall_s": wall, "event_ms": ms,
           "tile_lines": [1, 2, 4][tile], "autotune_ms": [round(x, 2) for x in tile_ms],
           "nonphysical_instances": int((s.instance_status() != 0).sum()),
           "running_instances": int((k == steps).sum())}
    if gate is not None:
        res["cells_nonlinear_last_step"] = float(np.mean(
            [s.get_flags(i).mean() for i in range(0, len(insts), 16)]))
    del s
    torch.cuda.empty_cache()
    return res


def c5_full_job(S, insts, params, gate=None, t_end=0.25, autotune_steps=2):
    """The whole job: every instance from t = 0 to t_end (its own CFL steps,
    the last one clamped), with autotuned tiles; instances finish at
    different times and their tiles then return at once."""
    import torch
    s = S.Solver(c5_meshes(S, insts), params, device="cuda:0")
    if gate is not None:
        s.gate_load(gate)
    for i, d in enumerate(insts):
        s.set_state(i, d.state())
    tile, tile_ms = s.autotune(steps=autotune_steps)
    ncell = np.array([d.n * d.n for d in insts], dtype=np.int64)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s.stream)
    # in calls of 256 steps, each reporting its progress (a call ends with the
    # instances' states back in the caller's buffer: a copy of at most the
    # running instances' states, a few ms)
    k = np.zeros(len(insts), dtype=np.int64)
    while True:
        kk = s.advance_to(np.full(len(insts), t_end), max_steps=256, raise_nonphysical=False)
        k += kk
        log(f"    {int(k.max())} steps, {int((kk == 256).sum())} instances still running, "
            f"{time.perf_counter() - t0:.0f} s")
        if not (kk == 256).any():
            break
    e1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cu = int((ncell * k).sum())
    codes = s.instance_status()
    res = {"value": cu / wall, "cell_updates": cu, "wall_s": wall, "event_ms": e0.elapsed_time(e1),
           "tile_lines": [1, 2, 4][tile], "autotune_ms": [round(x, 2) for x in tile_ms],
           "steps_min_max": [int(k[codes == 0].min()), int(k.max())],
           "nonphysical_instances": int((codes != 0).sum()), "t_end": t_end}
    del s
    torch.cuda.empty_cache()
    return res


def extrema(r, rel):
    """Local extrema along rows and columns of a 2D field that stand out by
    more than rel times its range."""
    tol = rel * (r.max() - r.min())
    cnt = 0
    for a in (r, r.T):
        d1, d2 = a[:, 1:-1] - a[:, :-2], a[:, 2:] - a[:, 1:-1]
        cnt += int((((d1 > tol) & (d2 < -tol)) | ((d1 < -tol) & (d2 > tol))).sum())
    return cnt


def envelope_excess(g, p):
    """How far g leaves the 3x3 local min/max envelope of p (0 if inside)."""
    from numpy.lib.stride_tricks import sliding_window_view as win
    w = win(np.pad(p, 1, mode="edge"), (3, 3))
    return float(max((g - w.max(axis=(-1, -2))).max(), (w.min(axis=(-1, -2)) - g).max(), 0.0))


def c5_accuracy(S, insts, gate, t_end=0.05, count=8):
    """Gated vs plain at fixed L1 error: a seeded subset of the batch (meshes
    of at most 384^2) run to t_end plain and gated, and the reference of each
    by a plain run on the 2x-refined mesh, restricted by 2x2 averaging; L1 of
    the density against the reference, local extrema and the 3x3 envelope."""
    import torch
    rng = np.random.default_rng(230409724)
    cand = [i for i, d in enumerate(insts) if d.n <= 384]
    pick = sorted(int(i) for i in rng.choice(cand, count, replace=False))
    sub = [insts[i] for i in pick]
    runs = {}
    for name, refine, prm in (("plain", 1, S.Params.make(eq=S.EULER)),
                              ("gated", 1, S.Params.make(eq=S.EULER, weights=S.W_LEARNED,
                                                         gate_threshold=GATE_THRESHOLD)),
                              ("reference", 2, S.Params.make(eq=S.EULER))):
        from paper_2304_09724_amd import workloads as WL
        m = [S.Mesh.rect(refine * d.n, refine * d.n, 0.0, 1.0, 0.0, 1.0, S.BC_TRANSMISSIVE,
                         S.BC_TRANSMISSIVE) for d in sub]
        s = S.Solver(m, prm, device="cuda:0")
        if name == "gated":
            s.gate_load(gate)
        for i, d in enumerate(sub):
            s.set_state(i, WL.four_quadrant(refine * d.n, d.quads))
        s.advance_to(np.full(len(sub), t_end), raise_nonphysical=False)
        ok = s.instance_status() == 0
        rho = []
        for i in range(len(sub)):
            r = s.get_state(i)[0, 0]
            if refine == 2:
                n = sub[i].n
                r = r.reshape(n, 2, n, 2).mean(axis=(1, 3))
            rho.append(r)
        runs[name] = (ok, rho)
        del s
        torch.cuda.empty_cache()
    l1p = l1g = 0.0
    xp = xg = 0
    env = 0.0
    used = []
    for i in range(len(sub)):
        if not all(runs[k][0][i] for k in runs):
            continue
        ref, rp, rg = runs["reference"][1][i], runs["plain"][1][i], runs["gated"][1][i]
        l1p += float(np.abs(rp - ref).mean())
        l1g += float(np.abs(rg - ref).mean())
        xp += extrema(rp, 1e-6)
        xg += extrema(rg, 1e-6)
        env = max(env, envelope_excess(rg, rp) / float(rp.max() - rp.min()))
        used.append(pick[i])
    return {"instances": used, "t_end": t_end, "l1_plain": l1p, "l1_gated": l1g,
            "l1_ratio_gated_over_plain": l1g / l1p if l1p > 0 else None,
            "local_extrema_plain": xp, "local_extrema_gated": xg,
            "envelope_excess_over_range": env,
            "reference": "plain runs on the 2x-refined meshes, restricted by 2x2 averaging"}


def oracle_2d_rate(n, steps, threads=None):
    """Cell-updates/s of the CPU oracle's 2D step on one n x n four-quadrant
    instance of the batch (its own OpenMP over rows), in a child process so
    that the thread count can be set."""
    code = (
        "import sys, time, json; sys.path.insert(0, %r)\n"
        "import numpy as np, oracle as O\n"
        "from paper_2304_09724_amd import workloads as WL\n"
        "d = [x for x in WL.four_quadrant_batch(count=%d) if x.n == %d][0]\n"
        "st = d.state(); cfg = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4)\n"
        "dt = O.dt2d(cfg, st, 1.0 / %d, 1.0 / %d, 0.9)\n"
        "t0 = time.perf_counter()\n"
        "for _ in range(%d): st, bad = O.step2d(cfg, st, 1.0 / %d, 1.0 / %d, dt)\n"
        "print(json.dumps({'wall': time.perf_counter() - t0}))\n"
    ) % (ROOT, C5_COUNT, n, n, n, steps, n, n)
    env = dict(os.environ)
    if threads is not None:
        env["OMP_NUM_THREADS"] = str(threads)
    out = subprocess.run([sys.executable, "-c", code], env=env, check=True, capture_output=True,
                         text=True).stdout
    wall = json.loads(out.strip().splitlines()[-1])["wall"]
    return n * n * steps / wall, wall


def cpu_baseline_2d(n=256, steps=2):
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    v_all, w_all = oracle_2d_rate(n, steps)
    v_one, w_one = oracle_2d_rate(n, 1, threads=1)
    return {"value": v_all, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"one {n}x{n} instance of the four-quadrant batch, {steps} steps "
                      f"({n * n * steps} cell-updates) with the oracle's OpenMP over rows, "
                      f"{w_all:.1f} s wall",
            "one_thread": {"value": v_one, "sample": f"the same instance, 1 step on 1 thread, "
                                                     f"{w_one:.1f} s wall"}}


# ---- 1D batch -------------------------------------------------------------------

def c2_leg(S, args, gate):
    import torch
    from paper_2304_09724_amd import workloads as WL
    log("1D batch ...")
    insts = WL.riemann_batch_1d(count=C2_COUNT, T=C2_T)
    meshes = [S.Mesh.line(d.n, d.x0, d.x1, S.BC_TRANSMISSIVE) for d in insts]
    init = torch.from_numpy(np.concatenate([d.state().reshape(-1) for d in insts])).to("cuda:0")
    ncell = np.array([d.n for d in insts], dtype=np.int64)
    T = np.full(C2_COUNT, C2_T)
    reps = args.c2_repeats

    def job(prm, name, gate_params=None):
        s = S.Solver(meshes, prm, device="cuda:0")
        if gate_params is not None:
            s.gate_load(gate_params)
        s.state.copy_(init)
        s.set_times(np.zeros(C2_COUNT))
        tile, tile_ms = s.autotune(steps=8)
        s.state.copy_(init)
        s.set_times(np.zeros(C2_COUNT))
        s.advance_to(T, raise_nonphysical=False)               # warm-up
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        cus = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(reps):
            s.state.copy_(init)
            s.set_times(np.zeros(C2_COUNT))
            ev[k][0].record(s.stream)
            steps = s.advance_to(T, raise_nonphysical=False)
            ev[k][1].record(s.stream)
            cus.append(int((ncell * steps).sum()))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        out = {"value": float(np.mean(cus)) * reps / wall, "unit": "cell-updates/s",
               "ms_per_job": wall / reps * 1e3, "cell_updates_per_job": float(np.mean(cus)),
               "kernel_ms": round(ms, 3), "tile_threads": [128, 256, 512][tile],
               "nonphysical_instances": int((s.instance_status() != 0).sum())}
        log(f"  {name}: {out['value']:.3e} cell-updates/s")
        return s, out

    plain, res = job(S.Params.make(eq=S.EULER, cfl=0.9), "plain")
    res["workload"] = ("1D Euler batch: 4096 Riemann problems, N even in {200..2000}, t=0.14, "
                       "CFL 0.9, transmissive, one persistent launch per job")
    res["roofline"] = roofline_alu(flops_1d(), res["cell_updates_per_job"], res["kernel_ms"],
                                   "loop1d_kernel<EULER> (persistent batched time loop)",
                                   traffic=measured_traffic("loop1d_euler_riemann4096_hbm_counters.md",
                                                            KERNEL_SOURCES_1D),
                                   algo_bytes=96)
    if gate is not None:
        g, gres = job(S.Params.make(eq=S.EULER, cfl=0.9, weights=S.W_LEARNED,
                                    gate_threshold=GATE_THRESHOLD, gate_every=3), "gated", gate)
        gres["speedup_vs_plain"] = gres["value"] / res["value"]
        gres["gate_every_steps"] = 3
        gres.update(c2_gated_l1(insts, plain, g))
        res["gated"] = gres
        del g
    p, pres = job(S.Params.make(eq=S.EULER, cfl=0.9, positivity=True), "positivity")
    pres["vs_plain"] = pres["value"] / res["value"]
    res["positivity"] = pres
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_1d(insts)
    del plain, p
    torch.cuda.empty_cache()
    return res


def exact_density(d, t, sub=16):
    """Exact cell averages of the density of a Riemann instance at time t."""
    import oracle as O
    e = np.linspace(d.x0, d.x1, d.n + 1)
    xs = e[:-1, None] + (np.arange(sub) + 0.5) / sub * d.dx
    out = np.empty(xs.shape)
    for j in range(d.n):
        for k in range(sub):
            out[j, k] = O.exact_riemann(1.4, d.left, d.right, (xs[j, k] - 0.5) / t)[0][0]
    return out.mean(axis=1)


def c2_gated_l1(insts, plain, gated):
    okg, okp = gated.instance_status() == 0, plain.instance_status() == 0
    sample = [i for i in range(C2_COUNT) if okg[i] and okp[i]][:24]
    l1p = l1g = tvp = tvg = 0.0
    for i in sample:
        ex = exact_density(insts[i], C2_T)
        rp, rg = plain.get_state(i)[0, 0], gated.get_state(i)[0, 0]
        l1p += np.abs(rp - ex).mean()
        l1g += np.abs(rg - ex).mean()
        tvp += np.abs(np.diff(rp)).sum()
        tvg += np.abs(np.diff(rg)).sum()
    return {"l1_ratio_gated_over_plain": l1g / l1p, "l1_sample_instances": len(sample),
            "total_variation_ratio_gated_over_plain": tvg / tvp}


def cpu_baseline_1d(insts):
    """The CPU oracle on the first 16 instances (seeded order) with N <= 800,
    each run in full to t = 0.14 on its own host thread."""
    import oracle as O
    sample = [i for i, d in enumerate(insts) if d.n <= 800][:16]
    threads = min(len(sample), os.cpu_count() or 1)
    cfg = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4)

    def one(i):
        o, t, steps, bad = O.advance1d(cfg, insts[i].state(), insts[i].dx, 0.9, C2_T)
        return insts[i].n * steps

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        cu = sum(ex.map(one, sample))
    wall = time.perf_counter() - t0
    return {"value": cu / wall, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} instances of the seeded batch with N <= 800 "
                      f"({cu} cell-updates, full runs to t={C2_T}), one host thread each, "
                      f"{wall:.1f} s wall"}


# ---- single large 2D meshes --------------------------------------------------------

def mesh_leg(S, name, meshes, state, params, steps=None, T=None, gate=None):
    """One instance advanced from t = 0 for `steps` CFL steps or to T, with
    autotuned tiles; HIP events on the solver's stream around the advance."""
    import torch
    s = S.Solver(meshes, params, device="cuda:0")
    if gate is not None:
        s.gate_load(gate)
    s.set_state(0, state)
    init = s.state.clone()
    tile, _ = s.autotune(steps=4)
    s.advance_to(1e9, max_steps=2)
    s.state.copy_(init)
    s.set_times(0.0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s.stream)
    k = s.advance_to(T if T is not None else 1e9, max_steps=steps or 10 ** 9,
                     raise_nonphysical=False)
    e1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cu = meshes[0].nx * meshes[0].ny * int(k[0])
    out = {"value": cu / wall, "steps": int(k[0]), "cell_updates": cu, "wall_s": round(wall, 3),
           "event_ms": e0.elapsed_time(e1), "tile_lines": [1, 2, 4][tile],
           "nonphysical": bool(s.instance_status()[0] != 0)}
    rho = s.get_state(0)[0, 0]
    if gate is not None:
        out["cells_nonlinear_last_step"] = float(s.get_flags(0).mean())
    del s, init
    torch.cuda.empty_cache()
    log(f"  {name}: {out['value']:.3e} cell-updates/s ({out['steps']} steps)")
    return out, rho


def c3_leg(S):
    """The 2D density wave at 1024^2 advanced to t = 2 (the whole run timed),
    and the density's L1 error against the exact averages there and on the
    coarser meshes 128^2 .. 512^2 (the scheme's order under refinement)."""
    from paper_2304_09724_amd import workloads as WL
    log("2D density wave to t=2 ...")
    errs = {}
    for n in (128, 256, 512, 1024):
        m = [S.Mesh.rect(n, n, 0.0, 2.0, 0.0, 2.0)]
        if n < 1024:
            s = S.Solver(m, S.Params.make(eq=S.EULER), device="cuda:0")
            s.set_state(0, WL.density_wave_2d(n))
            s.advance_to(2.0)
            rho = s.get_state(0)[0, 0]
            del s
        else:
            res, rho = mesh_leg(S, "density wave 1024^2", m, WL.density_wave_2d(n),
                                S.Params.make(eq=S.EULER), T=2.0)
        errs[n] = float(np.abs(rho - WL.density_wave_2d_exact_rho(n, t=2.0)).mean())
        log(f"    {n}^2: L1 {errs[n]:.3e}")
    ns = sorted(errs)
    res["workload"] = ("2D Euler density wave rho=1+0.2 sin(pi(x+y)), u=v=1, p=1, periodic "
                       f"[0,2]^2 at 1024^2, the whole run to t=2 ({res['steps']} CFL steps)")
    res["unit"] = "cell-updates/s"
    res["l1_density_error"] = {f"{n}^2": errs[n] for n in ns}
    res["l1_order"] = {f"{a}->{b}": float(np.log2(errs[a] / errs[b])) for a, b in zip(ns, ns[1:])}
    res["roofline"] = roofline_alu(flops_2d(), res["cell_updates"], res["event_ms"],
                                   "sweep2d_kernel x and y with the per-step kernels",
                                   algo_bytes=256)
    return res


def c4_leg(S, gate, steps, full):
    from paper_2304_09724_amd import workloads as WL
    log("2D shock/sine 4096x1024 ...")
    nx, ny = 4096, 1024
    m = [S.Mesh.rect(nx, ny, -5.0, 5.0, 0.0, 2 * np.pi / 3, S.BC_TRANSMISSIVE, S.BC_PERIODIC)]
    st = WL.shock_sine_2d(nx, ny)
    kw = {"T": C4_T} if full else {"steps": steps}
    plain, rp = mesh_leg(S, "plain", m, st, S.Params.make(eq=S.EULER), **kw)
    out = {"workload": "2D Euler Mach-3 shock into rho=1+0.2 sin5x sin3y at rest on "
                       "(-5,5)x(0,2pi/3), 4096x1024, " +
                       (f"to t={C4_T}" if full else f"{plain['steps']} CFL steps from t=0"),
           "unit": "cell-updates/s", "plain": plain,
           "roofline_plain": roofline_alu(flops_2d(), plain["cell_updates"], plain["event_ms"],
                                          "sweep2d_kernel x and y with the per-step kernels",
                                          algo_bytes=256)}
    if gate is not None:
        gated, rg = mesh_leg(S, "gated", m, st,
                             S.Params.make(eq=S.EULER, weights=S.W_LEARNED,
                                           gate_threshold=GATE_THRESHOLD), gate=gate, **kw)
        out["gated"] = gated
        out["speedup"] = gated["value"] / plain["value"]
        R = float(rp.max() - rp.min())
        out["max_abs_density_diff_over_range"] = float(np.abs(rg - rp).max() / R)
        out["l1_density_diff"] = float(np.abs(rg - rp).mean())
    return out


# ---- main --------------------------------------------------------------------------

def copy_check(nbytes):
    """One device-to-device copy of a buffer of nbytes: a kernel of known
    traffic to scale the HBM counters by."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    n = int(src.numel() * 8)
    del src, dst
    return n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40,
                    help="timed CFL steps of the whole 256-problem batch")
    ap.add_argument("--warmup", type=int, default=8, help="untimed steps before them")
    ap.add_argument("--legs", default="c5,gated,c2,c3,c4",
                    help="comma list of c5 (the headline), gated (c5 with the learned gate), "
                         "c2, c3, c4; without c5 only the legs are printed (profiling runs)")
    ap.add_argument("--c2-repeats", type=int, default=3)
    ap.add_argument("--c5-full", action="store_true",
                    help="time the whole four-quadrant job to t=0.25 (plain and, with the gated "
                         "leg, gated) instead of the CFL-step window")
    ap.add_argument("--c4-full", action="store_true",
                    help=f"run the shock/sine leg to t={C4_T} instead of 40 steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-check", type=int, default=0, metavar="BYTES",
                    help="after the timed steps, copy a device buffer of this many bytes once "
                         "(a plain copy kernel of known traffic, to scale HBM counters by)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; a batch would be "
                                   "sharded by instance across GPUs, each GPU advancing its "
                                   "instances with no communication", "n_gpus": args.gpus}))
        sys.exit(2)
    legs = set(args.legs.split(","))

    import torch
    import paper_2304_09724_amd as S
    from paper_2304_09724_amd import workloads as WL

    gate = train_info = None
    if legs & {"gated", "c2", "c4"}:
        gate, train_info = train_gate()

    if "c5" not in legs:
        extra = {}
        if "c2" in legs:
            extra["c2"] = c2_leg(S, args, gate)
        if "c3" in legs:
            extra["c3"] = c3_leg(S)
        if "c4" in legs:
            extra["c4"] = c4_leg(S, gate, 40, args.c4_full)
        if args.copy_check > 0:
            copy_check(args.copy_check)
        print(json.dumps({"legs": extra}), flush=True)
        return

    insts = WL.four_quadrant_batch(count=C5_COUNT)
    cells = sum(d.n * d.n for d in insts)
    log(f"four-quadrant batch: {C5_COUNT} instances, {cells} cells; warm-up {args.warmup}, "
        f"timed {args.steps} steps ...")
    if args.c5_full:
        args.steps, args.warmup = 1, 0
        plain = c5_full_job(S, insts, S.Params.make(eq=S.EULER))
    else:
        plain = c5_window(S, insts, S.Params.make(eq=S.EULER), args.warmup, args.steps)
    log(f"  plain: {plain['value']:.3e} cell-updates/s")
    value = plain["value"]
    ms_step = plain["wall_s"] / args.steps * 1e3
    roofline = roofline_alu(
        flops_2d(), plain["cell_updates"], plain["event_ms"],
        "sweep2d_kernel<EULER> x and y over all instances' tiles (HIP events around the "
        "timed advance; the per-step prepare/finish kernels are included)",
        traffic=measured_traffic("sweep2d_euler_fourquad256_hbm_counters.md", KERNEL_SOURCES_2D,
                                 key="hbm_bytes_per_step"),
        algo_bytes=256)
    roofline["traffic_unit"] = "HBM bytes per batch step (both sweeps, counted)"

    out = {"metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded four-quadrant Riemann problems)",
           "config": {"workload": f"2D Euler batch: {C5_COUNT} four-quadrant Riemann problems on "
                                  f"[0,1]^2, n=128*U{{1..8}} ({cells} cells), rho,p~U[0.1,1.5], "
                                  f"u,v~U[-1,1], transmissive, CFL 0.9, nonlinear weights; " +
                                  (f"the whole job from t=0 to t=0.25 timed (one bench step; "
                                   f"{plain.get('steps_min_max')} CFL steps per instance)"
                                   if args.c5_full else
                                   f"{args.steps} CFL steps of the whole batch timed after "
                                   f"{args.warmup} from t=0 (the run to t=0.25 takes "
                                   f"~2300 steps on the largest meshes)"),
                      "instances": C5_COUNT, "cells": cells,
                      "cell_updates_timed": plain["cell_updates"],
                      "nonphysical_instances": plain["nonphysical_instances"],
                      "nonphysical_note": "instances on which the unlimited scheme (no positivity "
                                          "limiter, as in the paper) meets a non-physical state "
                                          "stop there; only performed cell-updates are counted",
                      "parallelism": "single GPU; per step one x- and one y-sweep launch over "
                                     "every instance's tiles, 8-step chunks replayed as HIP graphs",
                      "tile": {"lines": plain["tile_lines"], "autotune_ms": plain["autotune_ms"]}},
           "roofline": roofline}
    if "gated" in legs:
        log("  gated ...")
        gp = S.Params.make(eq=S.EULER, weights=S.W_LEARNED, gate_threshold=GATE_THRESHOLD)
        if args.c5_full:
            g = c5_full_job(S, insts, gp, gate=gate)
        else:
            g = c5_window(S, insts, gp, args.warmup, args.steps, gate=gate)
        g["speedup_vs_plain"] = g["value"] / value
        g["gate_threshold"] = GATE_THRESHOLD
        log(f"  gated: {g['value']:.3e} cell-updates/s ({g['speedup_vs_plain']:.3f}x)")
        log("  gated vs plain accuracy on a subset ...")
        g["accuracy"] = c5_accuracy(S, insts, gate)
        g["training"] = train_info
        out["gated"] = g
    if args.copy_check > 0:
        out["copy_check_bytes"] = copy_check(args.copy_check)
    extra = {}
    if "c2" in legs:
        extra["c2"] = c2_leg(S, args, gate)
    if "c3" in legs:
        extra["c3"] = c3_leg(S)
    if "c4" in legs:
        extra["c4"] = c4_leg(S, gate, 40, args.c4_full)
    if extra:
        out["legs"] = extra
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline_2d()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
