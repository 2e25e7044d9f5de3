"""Training of the learned troubled-cell gate on the GPU.

Data come from the method itself: plain (nonlinear-weight) runs of 1D Euler
problems are stopped at several times and every cell contributes its 16
features (per conservative component the normalised shape of the jumps its
reconstruction reads and their size, and the normal Mach-like ratio
u / (|u| + c)) and its label (whether the nonlinear weights depart from the linear
ones), both computed by the library's kernels.  Training runs the library's
FP32 forward/backward kernel and its Adam kernel; this module only drives the
loop.
"""
from __future__ import annotations

import numpy as np

from . import Mesh, Params, Solver, EULER, W_NONLINEAR, BC_PERIODIC, BC_TRANSMISSIVE, \
    GATE_NFEATURES, GATE_NPARAMS, mlp_adam, mlp_grad
from . import workloads as WL

# A cell is labelled troubled where its quartic keeps less than this fraction
# of its linear weight in some characteristic field.
LABEL_LEVEL = 0.999


def init_params(seed: int = 0) -> np.ndarray:
    """He-initialised parameters (W1, b1, W2, b2, w3, b3)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(size=(32, GATE_NFEATURES)) * np.sqrt(2.0 / GATE_NFEATURES)
    W2 = rng.normal(size=(32, 32)) * np.sqrt(2.0 / 32)
    w3 = rng.normal(size=32) * np.sqrt(1.0 / 32)
    return np.concatenate([W1.ravel(), np.zeros(32), W2.ravel(), np.zeros(32), w3, [0.0]]
                          ).astype(np.float32)


def collect(problems, times, level=LABEL_LEVEL, device="cuda"):
    """Features and labels (the cell's weight test at the given level) of
    every cell of a 1D Euler batch, sampled at the given times of plain runs.
    problems: list of (mesh, state)."""
    import torch
    meshes = [m for m, _ in problems]
    s = Solver(meshes, Params.make(eq=EULER, weights=W_NONLINEAR), device=device)
    for i, (_, st) in enumerate(problems):
        s.set_state(i, st)
    feats, labs = [], []
    for t in times:
        if t > 0:
            s.advance_to(t, raise_nonphysical=False)
        f, lab = s.gate_data(level)
        ok = torch.isfinite(f).all(dim=1)
        feats.append(f[ok])
        labs.append(lab[ok])
    return torch.cat(feats), torch.cat(labs).float()


def training_problems(seed: int = 7, count: int = 48):
    """Riemann problems (the batched workload's distribution, smaller
    meshes), density waves moving and at rest at several wavenumbers, and the
    shock/sine problem: troubled and smooth cells of the kinds the gate
    meets."""
    probs = []
    for d in WL.riemann_batch_1d(count=count, seed=seed, nmin=100, nmax=400):
        probs.append((Mesh.line(d.n, d.x0, d.x1, BC_TRANSMISSIVE), d.state()))
    for u, amp, k in ((1.0, 0.2, 1), (0.0, 0.2, 1), (0.5, 0.2, 2), (-1.0, 0.1, 3), (0.0, 0.2, 4)):
        for n in (40, 80, 160):
            probs.append((Mesh.line(n, 0.0, 2.0, BC_PERIODIC),
                          WL.density_wave_1d(n, u=u, amp=amp, k=k)))
    for n in (400, 800):
        probs.append((Mesh.line(n, -5.0, 5.0, BC_TRANSMISSIVE), WL.shock_sine_1d(n)))
    return probs


def train(X, y, steps=800, lr=3e-3, pos_weight=8.0, seed=0, batch=16384, log=None):
    """Adam on the library's kernels; returns (params as numpy, loss history)."""
    import torch
    dev = X.device
    p = torch.from_numpy(init_params(seed)).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    n = X.shape[0]
    for k in range(1, steps + 1):
        idx = torch.randint(0, n, (min(batch, n),), generator=gen).to(dev)
        loss, g = mlp_grad(X[idx].contiguous(), y[idx].contiguous(), p, pos_weight)
        mlp_adam(p, g, m, v, k, lr)
        if k % 50 == 0 or k == 1:
            hist.append(float(loss.item()))
            if log:
                log(f"gate step {k}: loss {hist[-1]:.4f}")
    return p.cpu().numpy(), hist
