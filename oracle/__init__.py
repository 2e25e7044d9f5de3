"""CPU oracle of the ADER-SHWENO time step (arXiv 2304.09724).

TEST INFRASTRUCTURE ONLY.  A plain, slow FP64 C implementation of the
scheme (``oracle/*.c``) plus this ctypes marshalling layer.  Only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
it; the GPU library never imports, links or calls it, and the two share no
source.

Section references are to the paper: sec. 2 (1D scheme), sec. 3 (2D scheme),
sec. 4 (algorithm, Steps 1-5).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_FMA_PATH = os.path.join(_HERE, "liboracle_fma.so")
_SOURCES = ["recon.c", "riemann.c", "ck.c", "step.c", "mlp.c"]

ADVECTION, BURGERS, EULER = 0, 1, 2
BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE = 0, 1, 2
W_NONLINEAR, W_LINEAR, W_GATED = 0, 1, 2


def build(verbose: bool = False, contracted: bool = False) -> str:
    """Compile the oracle into oracle/liboracle.so with gcc (strict FP64:
    no contraction into FMA, so the oracle's rounding is plain).

    contracted: build the same sources into liboracle_fma.so with every
    contractible a * b + c fused into one FMA instead.  That library computes
    the same arithmetic in another rounding order; the tests use it only to
    measure how much two valid roundings of the scheme can differ."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    path = _FMA_PATH if contracted else _LIB_PATH
    fp = ["-mfma", "-ffp-contract=fast"] if contracted else ["-ffp-contract=off"]
    # ORACLE_SANITIZE=1: an AddressSanitizer + UndefinedBehaviorSanitizer build
    # (run the tests with the ASan runtime preloaded into the interpreter)
    san = (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer", "-g"] if os.environ.get("ORACLE_SANITIZE") else [])
    cmd = ["gcc", "-O2", "-std=c11", *fp, "-fno-fast-math", *san,
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", "-fopenmp",
           "-o", path + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    return path


class _Cfg(ctypes.Structure):
    _fields_ = [("eq", ctypes.c_int), ("charwise", ctypes.c_int),
                ("weights", ctypes.c_int), ("bc", ctypes.c_int * 4),
                ("gamma", ctypes.c_double), ("adv_a", ctypes.c_double),
                ("adv_b", ctypes.c_double), ("eps", ctypes.c_double),
                ("lin_w", ctypes.c_double * 3), ("positivity", ctypes.c_int)]


@dataclass
class Config:
    """Scheme parameters.  Defaults are the paper's: linear weights
    0.994/0.003/0.003 (sec. 2.3), gamma = 1.4 (sec. 5); eps = 1e-6 is a
    reading (the paper omits it)."""
    eq: int = EULER
    charwise: bool = True
    weights: int = W_NONLINEAR
    bc: tuple = (BC_PERIODIC,) * 4
    gamma: float = 1.4
    adv_a: float = 1.0
    adv_b: float = 0.0
    eps: float = 1e-6
    lin_w: tuple = (0.994, 0.003, 0.003)
    positivity: bool = False        # Euler safeguard (not in the paper)

    def c(self) -> _Cfg:
        s = _Cfg()
        s.eq, s.charwise, s.weights = self.eq, int(self.charwise), self.weights
        for k in range(4):
            s.bc[k] = self.bc[k]
        s.gamma, s.adv_a, s.adv_b, s.eps = self.gamma, self.adv_a, self.adv_b, self.eps
        for k in range(3):
            s.lin_w[k] = self.lin_w[k]
        s.positivity = int(self.positivity)
        return s


_libs = {}
_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def lib(contracted: bool = False):
    """The strict oracle library, or (contracted=True) its FMA-contracted
    build, loaded once each."""
    if contracted not in _libs:
        path = _FMA_PATH if contracted else _LIB_PATH
        if not os.path.exists(path):
            build(contracted=contracted)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(_Cfg)
        L.orc_ncomp.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_big_quartic.argtypes = [_D, _D, _D]
        L.orc_smoothness.argtypes = [_D]
        L.orc_smoothness.restype = ctypes.c_double
        L.orc_weights.argtypes = [P, _D, _D, _D]
        L.orc_combine.argtypes = [P, _D, _D, _D, _D]
        L.orc_recon_scalar.argtypes = [P, ctypes.c_int, _D, _D, _D]
        L.orc_euler_eigen.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
        L.orc_hllc_state.argtypes = [ctypes.c_double, ctypes.c_int, _D, _D, _D]
        L.orc_hlle.argtypes = [ctypes.c_double, ctypes.c_int, _D, _D, _D, _D]
        L.orc_euler_flux_x.argtypes = [ctypes.c_double, ctypes.c_int, _D, _D]
        L.orc_exact_riemann.argtypes = [ctypes.c_double] * 7 + [ctypes.c_double, _D]
        L.orc_exact_riemann.restype = ctypes.c_double
        L.orc_ck_fill.argtypes = [P, ctypes.c_int, _D]
        L.orc_grp_face.argtypes = [P, ctypes.c_int, _D, _D, _D]
        L.orc_dt1d.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]
        L.orc_dt1d.restype = ctypes.c_double
        L.orc_dt2d.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, _D]
        L.orc_dt2d.restype = ctypes.c_double
        L.orc_step1d.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, _D, _U8]
        L.orc_step2d.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, _D, _D, _U8]
        L.orc_advance1d.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_long, _D, _D,
                                    ctypes.POINTER(ctypes.c_long)]
        L.orc_advance2d.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_long, _D, _D, ctypes.POINTER(ctypes.c_long)]
        L.orc_mlp_forward.argtypes = [ctypes.c_int, _D, _D, _D]
        L.orc_mlp_backward.argtypes = [ctypes.c_int, _D, _D, _D, ctypes.c_double, _D]
        L.orc_mlp_backward.restype = ctypes.c_double
        L.orc_gate_features1d.argtypes = [P, ctypes.c_int, ctypes.c_double, _D, ctypes.c_int, _D]
        L.orc_gate_features2d.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, _D, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, _D]
        L.orc_gate_label1d.argtypes = [P, ctypes.c_int, ctypes.c_double, _D, ctypes.c_int,
                                       ctypes.c_double]
        _libs[contracted] = L
    return _libs[contracted]


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _flags(flags, n):
    if flags is None:
        return None, None
    f = np.ascontiguousarray(np.asarray(flags, dtype=np.uint8).reshape(-1))
    assert f.size == n
    return f, f.ctypes.data_as(_U8)


# ---- building blocks --------------------------------------------------------

def big_quartic(a, b) -> np.ndarray:
    a, b, c = _f64(a), _f64(b), np.zeros(5)
    lib().orc_big_quartic(_p(a), _p(b), _p(c))
    return c


def smoothness(c) -> float:
    c = _f64(c)
    return lib().orc_smoothness(_p(c))


def weights(cfg: Config, a, b) -> np.ndarray:
    a, b, w = _f64(a), _f64(b), np.zeros(3)
    lib().orc_weights(ctypes.byref(cfg.c()), _p(a), _p(b), _p(w))
    return w


def combine(cfg: Config, a, b, w) -> np.ndarray:
    a, b, w, c = _f64(a), _f64(b), _f64(w), np.zeros(5)
    lib().orc_combine(ctypes.byref(cfg.c()), _p(a), _p(b), _p(w), _p(c))
    return c


def recon_scalar(cfg: Config, a, b, mode=W_NONLINEAR) -> np.ndarray:
    a, b, c = _f64(a), _f64(b), np.zeros(5)
    lib().orc_recon_scalar(ctypes.byref(cfg.c()), mode, _p(a), _p(b), _p(c))
    return c


def euler_eigen(gamma, W, direction=0):
    W = _f64(W)
    m = W.size
    lam, R, L = np.zeros(m), np.zeros(m * m), np.zeros(m * m)
    lib().orc_euler_eigen(gamma, 1 if m == 3 else 2, direction, _p(W), _p(lam), _p(R), _p(L))
    return lam, R.reshape(m, m), L.reshape(m, m)


def euler_flux_x(gamma, W) -> np.ndarray:
    W = _f64(W)
    F = np.zeros(W.size)
    lib().orc_euler_flux_x(gamma, 1 if W.size == 3 else 2, _p(W), _p(F))
    return F


def hllc_state(gamma, WL, WR) -> np.ndarray:
    WL, WR = _f64(WL), _f64(WR)
    out = np.zeros(WL.size)
    lib().orc_hllc_state(gamma, 1 if WL.size == 3 else 2, _p(WL), _p(WR), _p(out))
    return out


def hlle(gamma, WL, WR):
    """HLLE flux and state at x/t = 0 (the positivity safeguard's first-order
    face; not part of the paper's scheme)."""
    WL, WR = _f64(WL), _f64(WR)
    F, Ws = np.zeros(WL.size), np.zeros(WL.size)
    lib().orc_hlle(gamma, 1 if WL.size == 3 else 2, _p(WL), _p(WR), _p(F), _p(Ws))
    return F, Ws


def exact_riemann(gamma, left, right, s):
    """Exact solution (rho, u, p) of the 1D Euler Riemann problem at x/t = s,
    and the star pressure."""
    out = np.zeros(3)
    ps = lib().orc_exact_riemann(gamma, *[float(v) for v in left], *[float(v) for v in right],
                                 float(s), _p(out))
    return out, ps


def ck_fill(cfg: Config, dim: int, w) -> np.ndarray:
    """w: array (m, 5, 5, 5) [c][a][b][k] with the k=0 layer set."""
    w = _f64(w).copy()
    lib().orc_ck_fill(ctypes.byref(cfg.c()), dim, _p(w))
    return w


def grp_face(cfg: Config, dim: int, JL, JR) -> np.ndarray:
    """JL, JR: arrays (5, 5, m) of d^{a+b}W/dx^a dy^b.  Returns (m,5,5,5)."""
    JL, JR = _f64(JL), _f64(JR)
    m = JL.shape[-1]
    w = np.zeros((m, 5, 5, 5))
    lib().orc_grp_face(ctypes.byref(cfg.c()), dim, _p(JL), _p(JR), _p(w))
    return w


# ---- learned gate ------------------------------------------------------------

N_FEATURES = 16
N_PARAMS = 32 * N_FEATURES + 32 + 32 * 32 + 32 + 32 + 1


def gate_features1d(cfg: Config, state, dx):
    """(n, 16) features of every cell of a 1D Euler state (2, 3, n)."""
    st = _f64(state)
    n = st.shape[-1]
    c = cfg.c()
    out = np.zeros((n, N_FEATURES))
    for j in range(n):
        f = np.zeros(N_FEATURES)
        lib().orc_gate_features1d(ctypes.byref(c), n, dx, _p(st), j, _p(f))
        out[j] = f
    return out


def gate_features2d(cfg: Config, state, dx, dy, direction):
    """(ny, nx, 16) features of every cell of a 2D Euler state (4, 4, ny, nx)
    along x (direction 0) or y (1)."""
    st = _f64(state)
    ny, nx = st.shape[-2:]
    c = cfg.c()
    out = np.zeros((ny, nx, N_FEATURES))
    f = np.zeros(N_FEATURES)
    for j in range(ny):
        for i in range(nx):
            lib().orc_gate_features2d(ctypes.byref(c), nx, ny, dx, dy, _p(st), i, j, direction,
                                      _p(f))
            out[j, i] = f
    return out


def gate_labels1d(cfg: Config, state, dx, level=0.99, cells=None):
    """Labels of cells 0..n-1 (or of the given indices, -1..n allowed)."""
    st = _f64(state)
    n = st.shape[-1]
    c = cfg.c()
    idx = range(n) if cells is None else cells
    return np.array([lib().orc_gate_label1d(ctypes.byref(c), n, dx, _p(st), j, level)
                     for j in idx], dtype=np.uint8)


def mlp_forward(params, X):
    p, X = _f64(params), _f64(X)
    assert p.size == N_PARAMS and X.ndim == 2 and X.shape[1] == N_FEATURES
    z = np.zeros(X.shape[0])
    lib().orc_mlp_forward(X.shape[0], _p(p), _p(X), _p(z))
    return z


def mlp_backward(params, X, y, pos_weight=1.0):
    """Mean weighted BCE of sigmoid(logits) and its gradient (FP64)."""
    p, X, y = _f64(params), _f64(X), _f64(y)
    assert p.size == N_PARAMS and X.ndim == 2 and X.shape[1] == N_FEATURES
    assert y.shape == (X.shape[0],)
    g = np.zeros(N_PARAMS)
    loss = lib().orc_mlp_backward(X.shape[0], _p(p), _p(X), _p(y), pos_weight, _p(g))
    return loss, g


# ---- time stepping ----------------------------------------------------------

def dt1d(cfg: Config, state, dx, cfl) -> float:
    st = _f64(state)
    return lib().orc_dt1d(ctypes.byref(cfg.c()), st.shape[-1], dx, cfl, _p(st))


def dt2d(cfg: Config, state, dx, dy, cfl) -> float:
    st = _f64(state)
    ny, nx = st.shape[-2:]
    return lib().orc_dt2d(ctypes.byref(cfg.c()), nx, ny, dx, dy, cfl, _p(st))


def step1d(cfg: Config, state, dx, dt, flags=None, contracted=False):
    """state: (2, m, n).  Returns (new_state, nonphysical_flag).
    contracted: run the FMA-contracted build (another rounding order)."""
    st = _f64(state)
    out = np.empty_like(st)
    f, fp = _flags(flags, st.shape[-1])
    bad = lib(contracted).orc_step1d(ctypes.byref(cfg.c()), st.shape[-1], dx, dt, _p(st), _p(out), fp)
    return out, bool(bad)


def step2d(cfg: Config, state, dx, dy, dt, flags=None, contracted=False):
    """state: (4, m, ny, nx).  Returns (new_state, nonphysical_flag).
    contracted: run the FMA-contracted build (another rounding order)."""
    st = _f64(state)
    out = np.empty_like(st)
    ny, nx = st.shape[-2:]
    f, fp = _flags(flags, nx * ny)
    bad = lib(contracted).orc_step2d(ctypes.byref(cfg.c()), nx, ny, dx, dy, dt, _p(st), _p(out), fp)
    return out, bool(bad)


def advance1d(cfg: Config, state, dx, cfl, T, max_steps=10**9, t0=0.0):
    """CFL steps to time T.  Returns (state, t, steps, nonphysical)."""
    st = _f64(state).copy()
    t = ctypes.c_double(t0)
    steps = ctypes.c_long(0)
    bad = lib().orc_advance1d(ctypes.byref(cfg.c()), st.shape[-1], dx, cfl, T, max_steps,
                              _p(st), ctypes.byref(t), ctypes.byref(steps))
    return st, t.value, steps.value, bool(bad)


def advance2d(cfg: Config, state, dx, dy, cfl, T, max_steps=10**9, t0=0.0):
    st = _f64(state).copy()
    ny, nx = st.shape[-2:]
    t = ctypes.c_double(t0)
    steps = ctypes.c_long(0)
    bad = lib().orc_advance2d(ctypes.byref(cfg.c()), nx, ny, dx, dy, cfl, T, max_steps,
                              _p(st), ctypes.byref(t), ctypes.byref(steps))
    return st, t.value, steps.value, bool(bad)
