"""MI355X (gfx950) ADER-SHWENO library: Python binding of the C ABI in
include/shweno.h.

This module only marshals arguments: every step of the scheme runs in the HIP
kernels of libshweno.so.  PyTorch provides the device memory (state and
workspace tensors) and the stream.  Loading fails loudly when the library is
not built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshweno.so")

ADVECTION, BURGERS, EULER = 0, 1, 2
BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE = 0, 1, 2
W_NONLINEAR, W_LINEAR, W_GATED, W_LEARNED = 0, 1, 2, 3
GATE_NFEATURES = 16
GATE_NPARAMS = 1633
STATUS = {0: "SHW_OK", -1: "SHW_EINVAL", -2: "SHW_ENOMEM", -3: "SHW_EDEVICE",
          -4: "SHW_ENONPHYS", -5: "SHW_ESTATE", -6: "SHW_ESCRATCH"}


class ShwError(RuntimeError):
    def __init__(self, code, msg="", bad_instance=-1):
        super().__init__(f"{STATUS.get(code, code)}: {msg} (instance {bad_instance})")
        self.code = code
        self.bad_instance = bad_instance


class Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double),
                ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("bc", ctypes.c_int * 4)]

    @classmethod
    def line(cls, n, x0, x1, bc=BC_PERIODIC):
        return cls(1, n, 1, x0, x1, 0.0, 1.0, (ctypes.c_int * 4)(bc, bc, bc, bc))

    @classmethod
    def rect(cls, nx, ny, x0, x1, y0, y1, bcx=BC_PERIODIC, bcy=BC_PERIODIC):
        return cls(2, nx, ny, x0, x1, y0, y1, (ctypes.c_int * 4)(bcx, bcx, bcy, bcy))


class Params(ctypes.Structure):
    _fields_ = [("eq", ctypes.c_int), ("charwise", ctypes.c_int), ("weights", ctypes.c_int),
                ("gamma", ctypes.c_double), ("adv_a", ctypes.c_double),
                ("adv_b", ctypes.c_double), ("cfl", ctypes.c_double), ("eps", ctypes.c_double),
                ("lin_w", ctypes.c_double * 3), ("gate_threshold", ctypes.c_double),
                ("gate_every", ctypes.c_int), ("positivity", ctypes.c_int)]

    @classmethod
    def make(cls, eq=EULER, charwise=True, weights=W_NONLINEAR, gamma=1.4, adv_a=1.0,
             adv_b=0.0, cfl=0.9, eps=1e-6, lin_w=(0.994, 0.003, 0.003), gate_threshold=0.5,
             gate_every=1, positivity=False):
        """positivity: the Euler safeguard, 1D and 2D (not in the paper; off =
        the paper's scheme)."""
        return cls(eq, int(charwise), weights, gamma, adv_a, adv_b, cfl, eps,
                   (ctypes.c_double * 3)(*lin_w), gate_threshold, gate_every, int(positivity))


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_LL = ctypes.POINTER(ctypes.c_longlong)


def lib():
    """Load libshweno.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run python -m paper_2304_09724_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        MP, PP = ctypes.POINTER(Mesh), ctypes.POINTER(Params)
        vp = ctypes.c_void_p
        L.shw_version.restype = ctypes.c_char_p
        L.shw_state_doubles.argtypes = [MP, PP]
        L.shw_state_doubles.restype = ctypes.c_size_t
        L.shw_workspace_bytes.argtypes = [MP, ctypes.c_int, PP]
        L.shw_workspace_bytes.restype = ctypes.c_size_t
        L.shw_create.argtypes = [MP, ctypes.c_int, PP, vp, vp, vp, ctypes.POINTER(vp)]
        L.shw_destroy.argtypes = [vp]
        L.shw_destroy.restype = None
        L.shw_set_state.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
        L.shw_get_state.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
        L.shw_get_time.argtypes = [vp, _D, _LL]
        L.shw_set_time.argtypes = [vp, _D]
        L.shw_compute_dt.argtypes = [vp, _D]
        L.shw_step.argtypes = [vp, _D]
        L.shw_step_cfl.argtypes = [vp]
        L.shw_advance_to.argtypes = [vp, _D, ctypes.c_longlong, _LL]
        L.shw_instance_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        FP = ctypes.POINTER(ctypes.c_float)
        L.shw_gate_load.argtypes = [vp, FP]
        L.shw_gate_data.argtypes = [vp, ctypes.c_double, vp, vp]
        L.shw_gate_packed_bytes.restype = ctypes.c_size_t
        L.shw_gate_pack.argtypes = [FP, vp]
        L.shw_mlp_logits.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.shw_mlp_grad.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_float, vp, vp, vp]
        L.shw_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_float, vp]
        L.shw_set_flags.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8)]
        L.shw_get_flags.argtypes = [vp, ctypes.c_int, vp]
        L.shw_set_graphs.argtypes = [vp, ctypes.c_int]
        L.shw_set_tile.argtypes = [vp, ctypes.c_int]
        L.shw_get_tile.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.shw_autotune.argtypes = [vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_float)]
        L.shw_status_detail.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_char_p,
                                        ctypes.c_size_t]
        L.shw_advance1d_static.argtypes = [MP, ctypes.c_int, PP, vp, _D, ctypes.c_longlong,
                                           _LL, vp]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _check_free(code, what):
    if code != 0:
        raise ShwError(code, what)


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def gate_pack(params) -> np.ndarray:
    """Packed (matrix-instruction layout) network from FP32 parameters."""
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    assert p.size == GATE_NPARAMS
    out = np.zeros(lib().shw_gate_packed_bytes(), dtype=np.uint8)
    _check_free(lib().shw_gate_pack(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                    out.ctypes.data_as(ctypes.c_void_p)), "gate_pack")
    return out


def mlp_logits(X, packed):
    """Logits of the samples X (cuda float32 [n, 16]) with a packed network
    (cuda uint8 tensor), on the matrix cores."""
    import torch
    assert X.dtype == torch.float32 and X.is_contiguous() and X.shape[1:] == (GATE_NFEATURES,)
    n = X.shape[0]
    out = torch.empty(n, dtype=torch.float32, device=X.device)
    _check_free(lib().shw_mlp_logits(_vp(X), n, _vp(packed), _vp(out), _stream_ptr()), "mlp_logits")
    return out


def mlp_grad(X, y, params, pos_weight=1.0):
    """(loss, grad) of the weighted BCE on cuda tensors (FP32)."""
    import torch
    assert X.dtype == torch.float32 and X.is_contiguous() and X.shape[1:] == (GATE_NFEATURES,)
    assert y.dtype == torch.float32 and y.shape == (X.shape[0],) and params.numel() == GATE_NPARAMS
    g = torch.empty(GATE_NPARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check_free(lib().shw_mlp_grad(_vp(X), _vp(y), X.shape[0], _vp(params), pos_weight,
                                   _vp(g), _vp(loss), _stream_ptr()), "mlp_grad")
    return loss, g


def mlp_adam(params, grad, m, v, step, lr):
    _check_free(lib().shw_mlp_adam(_vp(params), _vp(grad), _vp(m), _vp(v), step, lr,
                                   _stream_ptr()), "mlp_adam")


STATIC_SCRATCH_BYTES = 64 << 20
STATIC_MAX_INSTANCES = 4096


def advance1d_static(meshes, params, state, T, max_steps=1_000_000, raise_nonphysical=True):
    """shw_advance1d_static: advance a 1D batch (state: cuda float64 tensor of
    the instances' states back to back, taken at t = 0) to the end times T in
    place, with the library's static scratch and no allocation.  Returns the
    steps per instance."""
    import torch
    n = len(meshes)
    assert state.dtype == torch.float64 and state.is_contiguous() and state.is_cuda
    arr = (Mesh * n)(*meshes)
    T = np.ascontiguousarray(np.broadcast_to(np.asarray(T, float), (n,)))
    steps = np.zeros(n, dtype=np.int64)
    code = lib().shw_advance1d_static(arr, n, ctypes.byref(params), _vp(state), _dptr(T),
                                      max_steps, steps.ctypes.data_as(_LL), _stream_ptr())
    if code != 0 and not (code == -4 and not raise_nonphysical):
        raise ShwError(code, "advance1d_static")
    return steps


class Solver:
    """A batch of instances on one GPU.  meshes: list of Mesh (same dim);
    params: Params.  State and workspace are torch tensors on `device`."""

    def __init__(self, meshes, params: Params, device="cuda", stream=None):
        import torch
        self.torch = torch
        L = lib()
        self.meshes = list(meshes)
        self.params = params
        self.n = len(self.meshes)
        arr = (Mesh * self.n)(*self.meshes)
        self._marr = arr
        self.sizes = [L.shw_state_doubles(ctypes.byref(m), ctypes.byref(params)) for m in self.meshes]
        if any(s == 0 for s in self.sizes):
            raise ShwError(-1, "invalid mesh or parameters")
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        ws = L.shw_workspace_bytes(arr, self.n, ctypes.byref(params))
        if ws == 0:
            raise ShwError(-1, "invalid batch")
        self.device = torch.device(device)
        self.state = torch.zeros(int(self.offsets[-1]), dtype=torch.float64, device=self.device)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        self._check(L.shw_create(arr, self.n, ctypes.byref(params),
                                 ctypes.c_void_p(self.state.data_ptr()),
                                 ctypes.c_void_p(self.workspace.data_ptr()),
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)),
                    ctx=None)
        self.ctx = ctx

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and _lib is not None:
            _lib.shw_destroy(ctx)
            self.ctx = None

    def _check(self, code, ctx="self"):
        if code == 0:
            return
        c = self.ctx if ctx == "self" else None
        bad, msg = ctypes.c_int(-1), ctypes.create_string_buffer(256)
        if c:
            lib().shw_status_detail(c, ctypes.byref(bad), msg, 256)
        raise ShwError(code, msg.value.decode(), bad.value)

    def shape(self, i):
        m = self.meshes[i]
        q = 2 if m.dim == 1 else 4
        comps = {ADVECTION: 1, BURGERS: 1, EULER: 3 if m.dim == 1 else 4}[self.params.eq]
        return (q, comps, m.nx) if m.dim == 1 else (q, comps, m.ny, m.nx)

    def set_state(self, i, arr):
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64).reshape(self.shape(i)))
        self._check(lib().shw_set_state(self.ctx, i, a.ctypes.data_as(ctypes.c_void_p), 0))

    def get_state(self, i) -> np.ndarray:
        a = np.empty(self.shape(i))
        self._check(lib().shw_get_state(self.ctx, i, a.ctypes.data_as(ctypes.c_void_p), 0))
        return a

    def state_view(self, i):
        """Device tensor view of instance i's state (no copy)."""
        return self.state[int(self.offsets[i]):int(self.offsets[i + 1])].view(self.shape(i))

    def times(self):
        t = np.zeros(self.n)
        s = np.zeros(self.n, dtype=np.int64)
        self._check(lib().shw_get_time(self.ctx, _dptr(t), s.ctypes.data_as(_LL)))
        return t, s

    def instance_status(self):
        """Per instance: 0 ok, -4 (SHW_ENONPHYS) stopped on a non-physical state."""
        codes = np.zeros(self.n, dtype=np.int32)
        self._check(lib().shw_instance_status(self.ctx, codes.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return codes

    def set_times(self, t):
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, float), (self.n,)))
        self._check(lib().shw_set_time(self.ctx, _dptr(t)))

    def compute_dt(self):
        dt = np.zeros(self.n)
        self._check(lib().shw_compute_dt(self.ctx, _dptr(dt)))
        return dt

    def step(self, dt):
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, float), (self.n,)))
        self._check(lib().shw_step(self.ctx, _dptr(dt)))

    def step_cfl(self, raise_nonphysical=True):
        """One step of every instance with the CFL step size of its own
        averages, computed on the device."""
        code = lib().shw_step_cfl(self.ctx)
        if not (code == -4 and not raise_nonphysical):
            self._check(code)

    def advance_to(self, T, max_steps=1_000_000, raise_nonphysical=True):
        """Advance instance i to T[i]; returns the steps taken per instance.
        With raise_nonphysical=False a non-physical instance does not raise
        (see instance_status())."""
        T = np.ascontiguousarray(np.broadcast_to(np.asarray(T, float), (self.n,)))
        steps = np.zeros(self.n, dtype=np.int64)
        code = lib().shw_advance_to(self.ctx, _dptr(T), max_steps, steps.ctypes.data_as(_LL))
        if not (code == -4 and not raise_nonphysical):
            self._check(code)
        return steps

    def gate_load(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        assert p.size == GATE_NPARAMS
        self._check(lib().shw_gate_load(self.ctx, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def gate_data(self, level=0.99):
        """(features [cells, 16] float32, labels [cells] uint8) cuda tensors
        for every cell of the (1D Euler) batch in its current state; a label
        is 1 where the cell's quartic keeps less than level times its linear
        weight."""
        torch = self.torch
        cells = sum(m.nx * m.ny for m in self.meshes)
        f = torch.empty((cells, GATE_NFEATURES), dtype=torch.float32, device=self.device)
        lab = torch.empty(cells, dtype=torch.uint8, device=self.device)
        self._check(lib().shw_gate_data(self.ctx, float(level), _vp(f), _vp(lab)))
        return f, lab

    def set_graphs(self, enable):
        """2D: replay chunks of steps as a captured HIP graph (default) or not."""
        self._check(lib().shw_set_graphs(self.ctx, int(bool(enable))))

    def set_tile(self, variant):
        self._check(lib().shw_set_tile(self.ctx, int(variant)))

    def get_tile(self):
        v = ctypes.c_int()
        self._check(lib().shw_get_tile(self.ctx, ctypes.byref(v)))
        return v.value

    def autotune(self, steps=8):
        """Time each tile variant for `steps` steps on this batch, keep the
        fastest; state and times are left unchanged.  Returns (variant,
        milliseconds per variant)."""
        scratch = self.torch.empty_like(self.state)
        best = ctypes.c_int()
        ms = (ctypes.c_float * 3)()
        self._check(lib().shw_autotune(self.ctx, ctypes.c_void_p(scratch.data_ptr()), int(steps),
                                       ctypes.byref(best), ms))
        return best.value, list(ms)

    def get_flags(self, i):
        """Per-cell flags of instance i as the last step used them ((ny, nx)
        or (nx,) uint8)."""
        m = self.meshes[i]
        out = np.zeros(m.nx * m.ny, dtype=np.uint8)
        self._check(lib().shw_get_flags(self.ctx, i, out.ctypes.data_as(ctypes.c_void_p)))
        return out.reshape((m.ny, m.nx) if m.dim == 2 else (m.nx,))

    def set_flags(self, i, flags):
        f = np.ascontiguousarray(np.asarray(flags, dtype=np.uint8).reshape(-1))
        self._check(lib().shw_set_flags(self.ctx, i, f.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
