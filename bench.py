#!/usr/bin/env python3
"""Throughput of the batched 1D Euler ADER-SHWENO time loop on one MI355X.

Workload: 4096 independent 1D Euler Riemann problems on [0,1] (gamma 1.4),
N even and uniform in {200..2000} cells per instance, left/right rho, p ~
U[0.1, 2], u ~ U[-1, 1] (seeded), jump at x = 0.5, transmissive ends,
advanced to t = 0.14 with CFL 0.9 in one persistent launch.  One bench step =
the whole job: reset the batch to its initial state and advance every
instance to t = 0.14.  Inputs are resident in HBM before the timed region.

Prints one JSON line (metric, value = cell-updates/s, roofline of the
persistent kernel, CPU-oracle baseline on a bounded sample).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

T_END = 0.14
COUNT = 4096
# FP64 flops of one 1D Euler cell-update of the sweep (reconstruction of one
# cell in characteristic fields with nonlinear weights, GRP at one face,
# 4-point Lobatto flux, update), FMA counted as 2; counted from the kernel's
# own templated arithmetic by paper_2304_09724_amd/flopcount.
FLOPS_PER_CELL_UPDATE = None
FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X, dense FP64 vector
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# HBM bytes of one launch of the persistent kernel on this workload, from the
# two counter runs summarised in profiles/ (FETCH_SIZE and WRITE_SIZE scaled by
# a 1 GiB copy); valid only for the kernel code those runs measured (the
# sources compared without their comments and with whitespace collapsed).
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "loop1d_euler_riemann4096_hbm_counters.md")
KERNEL_SOURCES = ["sweep1d.hip", "shw_kernels.h", "sweep1d_math.h", "shw_math.h", "gate_math.h",
                  "lanes.h"]


def kernel_fingerprint():
    import hashlib
    import re
    # string literals kept, // and /* */ comments dropped, whitespace runs as one blank
    token = re.compile(r'"(?:\\.|[^"\\])*"|//[^\n]*|/\*.*?\*/', re.S)
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2304_09724_amd", "csrc", f)) as fh:
            text = token.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", fh.read())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """Counted HBM bytes per launch, or None if the kernel changed since."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("kernel_sources_sha256_16:", "hbm_bytes_per_launch:")))
    if fields.get("kernel_sources_sha256_16", "").strip() != kernel_fingerprint():
        return None
    return float(fields["hbm_bytes_per_launch"])


def flops_per_cell_update():
    global FLOPS_PER_CELL_UPDATE
    if FLOPS_PER_CELL_UPDATE is None:
        from paper_2304_09724_amd import flopcount
        FLOPS_PER_CELL_UPDATE = flopcount.euler1d_cell_update()["flops"]
    return FLOPS_PER_CELL_UPDATE


def make_batch():
    from paper_2304_09724_amd import workloads as WL
    insts = WL.riemann_batch_1d(count=COUNT, T=T_END)
    states = [d.state() for d in insts]
    return insts, states


def cpu_baseline(insts, states, budget_threads=None):
    """The CPU oracle, as it stands, on a bounded sample of the same batch:
    the first 16 instances (seeded order) with N <= 800, each run in full to
    t = 0.14 on its own host thread."""
    import oracle as O
    sample = [i for i, d in enumerate(insts) if d.n <= 800][:16]
    threads = min(len(sample), budget_threads or os.cpu_count() or 1)
    cfg = O.Config(eq=O.EULER, bc=(O.BC_TRANSMISSIVE,) * 4)

    def one(i):
        o, t, steps, bad = O.advance1d(cfg, states[i], insts[i].dx, 0.9, T_END)
        return insts[i].n * steps

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        cu = sum(ex.map(one, sample))
    wall = time.perf_counter() - t0
    return {"value": cu / wall, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} instances of the seeded batch with N <= 800 "
                      f"({cu} cell-updates, full runs to t={T_END}), one host thread each, "
                      f"{wall:.1f} s wall"}


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


def positivity_leg(S, insts, meshes, init, args, plain_value):
    """The same job with the positivity safeguard on (not in the paper; the
    headline value is the paper's scheme without it): throughput and the
    instances that still stop on a non-physical state."""
    import torch
    log("positivity safeguard ...")
    s = S.Solver(meshes, S.Params.make(eq=S.EULER, cfl=0.9, positivity=True), device="cuda:0")
    zeros = np.zeros(COUNT)
    T = np.full(COUNT, T_END)
    ncell = np.array([d.n for d in insts], dtype=np.int64)
    for _ in range(args.warmup):
        s.state.copy_(init)
        s.set_times(zeros)
        s.advance_to(T, raise_nonphysical=False)
    torch.cuda.synchronize()
    cus = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.state.copy_(init)
        s.set_times(zeros)
        cus.append(int((ncell * s.advance_to(T, raise_nonphysical=False)).sum()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = float(np.mean(cus)) * args.steps / wall
    return {"value": value, "unit": "cell-updates/s", "vs_plain": value / plain_value,
            "ms_per_step": wall / args.steps * 1e3, "cell_updates_per_step": float(np.mean(cus)),
            "nonphysical_instances": int((s.instance_status() != 0).sum())}


def gated_leg(S, insts, states, meshes, init, args, plain_value, plain):
    """The same job with the learned gate: network trained on the GPU from
    plain runs of separate seeded problems (untimed), then K timed steps; L1
    error against the exact solution compared with the plain run on a sample
    of instances both complete."""
    import torch
    from paper_2304_09724_amd import gate as GT
    log("gate: training data and training ...")
    t0 = time.perf_counter()
    X, y = GT.collect(GT.training_problems(), times=[0.0, 0.02, 0.06, 0.1, 0.14])
    params, hist = GT.train(X, y)
    train_s = time.perf_counter() - t0
    threshold = 0.05
    every = 3
    g = S.Solver(meshes, S.Params.make(eq=S.EULER, cfl=0.9, weights=S.W_LEARNED,
                                       gate_threshold=threshold, gate_every=every),
                 device="cuda:0")
    g.gate_load(params)
    zeros = np.zeros(COUNT)
    T = np.full(COUNT, T_END)
    ncell = np.array([d.n for d in insts], dtype=np.int64)
    for _ in range(args.warmup):
        g.state.copy_(init)
        g.set_times(zeros)
        g.advance_to(T, raise_nonphysical=False)
    torch.cuda.synchronize()
    cus = []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        g.state.copy_(init)
        g.set_times(zeros)
        steps = g.advance_to(T, raise_nonphysical=False)
        cus.append(int((ncell * steps).sum()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    value = float(np.mean(cus)) * args.steps / wall
    okg, okp = g.instance_status() == 0, plain.instance_status() == 0
    sample = [i for i in range(COUNT) if okg[i] and okp[i]][:24]
    l1p = l1g = tvp = tvg = 0.0
    for i in sample:
        ex = exact_density(insts[i], T_END)
        rp, rg = plain.get_state(i)[0, 0], g.get_state(i)[0, 0]
        l1p += np.abs(rp - ex).mean()
        l1g += np.abs(rg - ex).mean()
        tvp += np.abs(np.diff(rp)).sum()
        tvg += np.abs(np.diff(rg)).sum()
    # fraction of cells the gate passes as smooth, over the training data
    z = S.mlp_logits(X, torch.from_numpy(S.gate_pack(params)).to(X.device)).cpu().numpy()
    smooth = float((z < np.log(threshold / (1 - threshold))).mean())
    return {"value": value, "unit": "cell-updates/s", "speedup_vs_plain": value / plain_value,
            "ms_per_step": wall / args.steps * 1e3, "gate_threshold": threshold,
            "gate_every_steps": every,
            "l1_ratio_gated_over_plain": l1g / l1p, "l1_sample_instances": len(sample),
            "total_variation_ratio_gated_over_plain": tvg / tvp,
            "nonphysical_instances": int((~okg).sum()),
            "smooth_fraction_training_cells": smooth,
            "training": {"samples": int(X.shape[0]), "adam_steps": 800,
                         "loss_first_last": [hist[0], hist[-1]], "seconds": round(train_s, 2)},
            "gated_2d": gated_2d_leg(S, params)}


def gated_2d_leg(S, params, threshold=0.05, steps=40):
    """The learned gate on 2D Euler: the shock/sine problem (Mach-3 shock into
    rho = 1 + 0.2 sin 5x sin 3y on (-5,5) x (0,2pi/3); 2048 x 512 cells, a
    quarter of the 4096 x 1024 shape), a window of `steps` CFL steps from
    t = 0 with autotuned tiles, plain and gated: throughput, the plain run
    against the FP64 roofline (HIP events on the solver's stream around the
    whole advance, which holds the sweeps and the small time-loop kernels),
    and the gated density's departure from the plain one."""
    import torch
    from paper_2304_09724_amd import flopcount
    from paper_2304_09724_amd import workloads as WL
    nx, ny = 2048, 512
    m = [S.Mesh.rect(nx, ny, -5.0, 5.0, 0.0, 2 * np.pi / 3, S.BC_TRANSMISSIVE, S.BC_PERIODIC)]
    st = WL.shock_sine_2d(nx, ny)
    out = {"workload": f"2D Euler shock/sine {nx}x{ny}, {steps} CFL steps from t=0",
           "unit": "cell-updates/s"}
    res = {}
    for name, prm in (("plain", S.Params.make(eq=S.EULER)),
                      ("gated", S.Params.make(eq=S.EULER, weights=S.W_LEARNED,
                                              gate_threshold=threshold))):
        s = S.Solver(m, prm, device="cuda:0")
        if name == "gated":
            s.gate_load(params)
        s.set_state(0, st)
        init = s.state.clone()
        tile, _ = s.autotune(steps=8)
        s.advance_to(1e9, max_steps=2)
        s.state.copy_(init)
        s.set_times(0.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(s.stream)
        k = s.advance_to(1e9, max_steps=steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        cu = nx * ny * int(k[0])
        out[name] = cu / el
        out[name + "_tile_lines"] = [1, 2, 4][tile]
        res[name] = s.get_state(0)[0, 0]
        if name == "plain":
            ms = e0.elapsed_time(e1)
            flops = flopcount.euler2d_cell_update(True)["flops"]
            tf = flops * cu / (ms * 1e-3) / 1e12
            out["roofline_plain"] = {
                "bound": "alu", "achieved": round(tf, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4),
                "flops_per_cell_update": flops, "ms": round(ms, 3),
                "hbm_algorithmic_GBs": round(256 * cu / (ms * 1e-3) / 1e9, 1)}
        else:
            out["cells_gated_nonlinear_last_step"] = float(s.get_flags(0).mean())
        del s
    out["speedup"] = out["gated"] / out["plain"]
    R = float(res["plain"].max() - res["plain"].min())
    out["max_abs_density_diff_over_range"] = float(np.abs(res["gated"] - res["plain"]).max() / R)
    out["l1_density_diff"] = float(np.abs(res["gated"] - res["plain"]).mean())
    out["cpu_oracle_2d"] = cpu_baseline_2d()
    return out


def cpu_baseline_2d(n=48, steps=4):
    """The CPU oracle's 2D step on a 48 x 48 piece of the same problem, a few
    steps (its own OpenMP over rows)."""
    import oracle as O
    from paper_2304_09724_amd import workloads as WL
    st = WL.shock_sine_2d(10 * n // 2, n)[:, :, :, :n].copy()
    cfg = O.Config(eq=O.EULER, bc=(O.BC_PERIODIC,) * 4)
    dx, dy = 10.0 / (10 * n // 2), (2 * np.pi / 3) / n
    dt = O.dt2d(cfg, st, dx, dy, 0.9)
    t0 = time.perf_counter()
    for _ in range(steps):
        st, bad = O.step2d(cfg, st, dx, dy, dt)
    wall = time.perf_counter() - t0
    return {"value": n * n * steps / wall, "unit": "cell-updates/s", "kind": "oracle",
            "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())), "sample": f"{n}x{n} cells of the 2D shock/sine field, "
                                             f"{steps} steps, {wall:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gate", action="store_true")
    ap.add_argument("--only-2d", action="store_true",
                    help="train the gate and run only the 2D leg (plain and gated)")
    ap.add_argument("--copy-check", type=int, default=0, metavar="BYTES",
                    help="after the timed steps, copy a device buffer of this many bytes once "
                         "(a plain copy kernel of known traffic, to scale HBM counters by)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the batch would be "
                                   "sharded by instance across GPUs with no communication "
                                   "(see the multi-GPU design notes)", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.only_2d:
        import paper_2304_09724_amd as S
        from paper_2304_09724_amd import gate as GT
        X, y = GT.collect(GT.training_problems(), times=[0.0, 0.02, 0.06, 0.1, 0.14])
        params, _ = GT.train(X, y)
        print(json.dumps({"gated_2d": gated_2d_leg(S, params)}), flush=True)
        return

    import torch
    import paper_2304_09724_amd as S

    log("building the batch ...")
    insts, states = make_batch()
    meshes = [S.Mesh.line(d.n, d.x0, d.x1, S.BC_TRANSMISSIVE) for d in insts]
    solver = S.Solver(meshes, S.Params.make(eq=S.EULER, cfl=0.9), device="cuda:0")
    init = torch.from_numpy(np.concatenate([s.reshape(-1) for s in states])).to("cuda:0")
    stream = solver.stream
    zeros = np.zeros(COUNT)
    T = np.full(COUNT, T_END)
    ncell = np.array([d.n for d in insts], dtype=np.int64)

    def one_step():
        solver.state.copy_(init)
        solver.set_times(zeros)
        return solver.advance_to(T, raise_nonphysical=False)

    # tile variant from the project's autotuner (8 steps of every instance per
    # variant, untimed here)
    solver.state.copy_(init)
    solver.set_times(zeros)
    tile, tile_ms = solver.autotune(steps=8)
    log(f"autotuner: variant {tile} (ms per variant {tile_ms})")

    log(f"warmup x{args.warmup} ...")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    cell_updates = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        solver.state.copy_(init)
        solver.set_times(zeros)
        ev[k][0].record(stream)
        steps = solver.advance_to(T, raise_nonphysical=False)
        ev[k][1].record(stream)
        cell_updates.append(int((ncell * steps).sum()))
        ev[k][1].synchronize()
        log(f"step {k}: {cell_updates[-1]} cell-updates, "
            f"{ev[k][0].elapsed_time(ev[k][1]):.2f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    codes = solver.instance_status()
    nonphys = int((codes != 0).sum())
    cu_step = float(np.mean(cell_updates))
    value = cu_step * args.steps / wall

    flops = flops_per_cell_update()
    achieved_tflops = flops * cu_step / (kernel_ms * 1e-3) / 1e12
    algo_bytes = 2 * 2 * 3 * 8           # read + write of W and V (3 components) per cell-update
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 3),
                "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved_tflops / FP64_VECTOR_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(), "traffic_unit": "bytes per launch (HBM, counted)",
                "kernel": "loop1d_kernel<EULER> (persistent batched time loop)",
                "kernel_ms": round(kernel_ms, 3), "flops_per_cell_update": flops,
                "hbm_algorithmic_GBs": round(algo_bytes * cu_step / (kernel_ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(algo_bytes * cu_step / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    out = {"metric": "cell-updates/sec FP64 (plain vs learned-gated, batched) at fixed L1 error",
           "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded Riemann problems)",
           "config": {"workload": "1D Euler batch: 4096 Riemann problems, N in {200..2000}, "
                                  "t=0.14, CFL 0.9, transmissive, plain nonlinear weights",
                      "instances": COUNT, "cell_updates_per_step": cu_step,
                      "nonphysical_instances": nonphys,
                      "nonphysical_note": "instances on which the unlimited scheme (no "
                                          "positivity limiter, as in the paper) meets a "
                                          "non-physical state stop there; only the cell-"
                                          "updates actually performed are counted",
                      "parallelism": "single GPU, one persistent launch",
                      "tile": {"variant": tile, "threads_per_instance": [128, 256, 512][tile],
                               "autotune_ms_8_steps": [round(x, 3) for x in tile_ms]}},
           "roofline": roofline}
    if args.copy_check > 0:
        src = torch.ones(args.copy_check // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_check_bytes"] = int(src.numel() * 8)
        del src, dst
    if not args.no_gate:
        out["gated"] = gated_leg(S, insts, states, meshes, init, args, value, solver)
        out["positivity"] = positivity_leg(S, insts, meshes, init, args, value)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(insts, states)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
