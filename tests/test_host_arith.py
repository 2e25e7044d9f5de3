"""CPU checks of the sweep kernels' own arithmetic against the oracle.

The per-point arithmetic of the kernels is templated on the real type;
tests/host/sweep_host.cpp instantiates it with double on the host (IEEE
division and square root in place of the device's refined hardware
estimates, everything else the same source).  These tests pin the generated
Lax-Wendroff series of sec. 3.1 and the whole 2D GRP of sec. 3 (HLLC leading
term, characteristic upwinding of every derivative, series) against the
oracle on random smooth data, and check that the committed generated header
is what its generator writes.
"""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2304_09724_amd", "csrc")
GAMMA = 1.4
L_SCALE = 0.1          # length scale of the random smooth fields


@pytest.fixture(scope="module")
def host(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("host") / "sweep_host.so")
    cmd = ["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", os.path.join(ROOT, "tests", "host", "sweep_host.cpp"),
           "-o", out]
    subprocess.run(cmd, check=True)
    lib = ctypes.CDLL(out)
    P = ctypes.POINTER(ctypes.c_double)
    lib.host_ck2d_euler.argtypes = [P, ctypes.c_double, P]
    lib.host_ck1d_euler.argtypes = [P, ctypes.c_double, P]
    lib.host_grp2d_euler.argtypes = [P, P, ctypes.c_double, P]
    lib.host_jidx.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.host_jidx.restype = ctypes.c_int
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _state(rng, dim):
    """Conservative point state with rho, p in [0.5, 2], |u| <= 1."""
    rho, p = rng.uniform(0.5, 2.0, 2)
    vel = rng.uniform(-1.0, 1.0, dim)
    E = p / (GAMMA - 1.0) + 0.5 * rho * float(vel @ vel)
    return np.concatenate([[rho], rho * vel, [E]])


def _series(rng, m, dim, base):
    """Spatial Taylor coefficients [m][5][5] (a + b <= 4; b = 0 in 1D) of a
    smooth field of length scale L_SCALE around the point state."""
    s = np.zeros((m, 5, 5))
    for a in range(5):
        for b in range(5 if dim == 2 else 1):
            if a + b > 4:
                continue
            if a + b == 0:
                s[:, 0, 0] = base
            else:
                s[:, a, b] = 0.3 * np.abs(base).max() * rng.uniform(-1, 1, m) / L_SCALE ** (a + b)
    return s


def _rel_err(got, want):
    """Worst error of each time order k over the components, relative to the
    largest coefficient of that order."""
    return np.abs(got - want).max(axis=0) / np.abs(want).max(axis=0)


def test_generated_series_header_is_current():
    """ck2d_gen.h is exactly what gen_ck2d.py writes."""
    gen = subprocess.run([sys.executable, "gen_ck2d.py"], cwd=CSRC, check=True,
                         capture_output=True, text=True).stdout
    with open(os.path.join(CSRC, "ck2d_gen.h")) as fh:
        assert fh.read() == gen


def test_ck2d_series_matches_oracle(host):
    """The generated 2D series (primitive-variable recursion) against the
    oracle's conservative trivariate series (sec. 3.1): the same truncated
    Taylor coefficients of one analytic solution, so they agree to
    rounding."""
    rng = np.random.default_rng(7)
    cfg = O.Config(eq=O.EULER, gamma=GAMMA)
    worst = np.zeros(5)
    for _ in range(200):
        s = _series(rng, 4, 2, _state(rng, 2))
        wt = np.zeros(20)
        host.host_ck2d_euler(_p(np.ascontiguousarray(s)), GAMMA, _p(wt))
        w = np.zeros((4, 5, 5, 5))
        w[:, :, :, 0] = s
        want = O.ck_fill(cfg, 2, w)[:, 0, 0, :]
        worst = np.maximum(worst, _rel_err(wt.reshape(4, 5), want))
    # k = 0: the energy comes back from the primitive pressure (rounding only)
    assert worst[0] <= 1e-15, worst
    assert (worst <= 1e-12).all(), worst


def test_ck1d_series_matches_oracle(host):
    """The 1D series (conservative, velocity by series division) against
    the oracle's."""
    rng = np.random.default_rng(8)
    cfg = O.Config(eq=O.EULER, gamma=GAMMA)
    worst = np.zeros(5)
    for _ in range(200):
        s = _series(rng, 3, 1, _state(rng, 1))
        w1 = np.ascontiguousarray(s[:, :, 0])
        wt = np.zeros(15)
        host.host_ck1d_euler(_p(w1), GAMMA, _p(wt))
        w = np.zeros((3, 5, 5, 5))
        w[:, :, 0, 0] = w1
        want = O.ck_fill(cfg, 1, w)[:, 0, 0, :]
        worst = np.maximum(worst, _rel_err(wt.reshape(3, 5), want))
    assert worst[0] == 0.0
    assert (worst <= 1e-12).all(), worst


@pytest.mark.parametrize("jump", [0.0, 0.02, 0.5])
def test_grp2d_matches_oracle(host, jump):
    """The whole 2D GRP at an interface point (leading HLLC state, each of
    the 14 derivatives upwinded field by field at the leading term's
    Jacobian, series) against the oracle's GRP on the same two sides: equal
    sides, a small and a large jump."""
    rng = np.random.default_rng(9 + int(100 * jump))
    cfg = O.Config(eq=O.EULER, gamma=GAMMA)
    fact = [1.0, 1.0, 2.0, 6.0, 24.0]
    worst = np.zeros(5)
    for _ in range(100):
        base = _state(rng, 2)
        other = base * (1.0 + jump * rng.uniform(-1, 1, 4))
        other[3] = max(other[3], 0.5 * other[1] ** 2 / other[0] + 0.3 / (GAMMA - 1.0))
        sl = _series(rng, 4, 2, base)
        sr = _series(rng, 4, 2, other)
        if jump == 0.0:
            sr = sl.copy()
        # library side: [15][4] series coefficients at jidx(a, n);
        # oracle side: (5, 5, m) derivatives d^{a+b}W/dx^a dy^b
        jl, jr = np.zeros((15, 4)), np.zeros((15, 4))
        dl, dr = np.zeros((5, 5, 4)), np.zeros((5, 5, 4))
        for a in range(5):
            for n in range(5 - a):
                i = host.host_jidx(a, n)
                jl[i], jr[i] = sl[:, a, n], sr[:, a, n]
                dl[a, n], dr[a, n] = sl[:, a, n] * fact[a] * fact[n], sr[:, a, n] * fact[a] * fact[n]
        wt = np.zeros(20)
        host.host_grp2d_euler(_p(jl), _p(jr), GAMMA, _p(wt))
        want = O.grp_face(cfg, 2, dl, dr)[:, 0, 0, :]
        worst = np.maximum(worst, _rel_err(wt.reshape(4, 5), want))
    assert (worst <= 1e-11).all(), worst
