"""CPU checks of the C-ABI library (no GPU work): it loads and exports every
function the public header declares, host-side validation rejects what the
header says it rejects, and the host packing of the gate network follows the
matrix-instruction layout the header and the kernels document."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2304_09724_amd as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shweno.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(shw_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(S.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_string():
    assert S.lib().shw_version().decode().startswith("shweno")


def line(n=64, bc=S.BC_PERIODIC):
    return S.Mesh.line(n, 0.0, 2.0, bc)


def state_doubles(mesh, params):
    return S.lib().shw_state_doubles(ctypes.byref(mesh), ctypes.byref(params))


def test_state_size_follows_the_layout():
    # 1D: W and V planes; 2D: W, V, Y, Z planes; per conservative component
    assert state_doubles(line(50), S.Params.make(eq=S.EULER)) == 2 * 3 * 50
    assert state_doubles(line(50), S.Params.make(eq=S.ADVECTION)) == 2 * 50
    rect = S.Mesh.rect(12, 10, 0.0, 1.0, 0.0, 1.0)
    assert state_doubles(rect, S.Params.make(eq=S.EULER)) == 4 * 4 * 120


@pytest.mark.parametrize("kw", [
    dict(cfl=0.0), dict(eps=0.0), dict(gamma=1.0), dict(lin_w=(0.5, 0.3, 0.3)),
    dict(weights=S.W_LEARNED, gate_threshold=0.0),
    dict(weights=S.W_LEARNED, gate_threshold=1.0),
    dict(weights=S.W_LEARNED, gate_threshold=0.5, gate_every=0),
    dict(weights=S.W_LEARNED, gate_threshold=0.5, gate_every=1025),
])
def test_invalid_parameters_are_rejected_on_the_host(kw):
    args = dict(eq=S.EULER)
    args.update(kw)
    assert state_doubles(line(), S.Params.make(**args)) == 0


def workspace(mesh, params):
    arr = (S.Mesh * 1)(mesh)
    return S.lib().shw_workspace_bytes(arr, 1, ctypes.byref(params))


def test_learned_gate_is_euler_only():
    rect = S.Mesh.rect(16, 16, 0.0, 1.0, 0.0, 1.0)
    for mesh in (line(), rect):
        p = S.Params.make(eq=S.EULER, weights=S.W_LEARNED, gate_threshold=0.5)
        assert workspace(mesh, p) > 0
        p = S.Params.make(eq=S.ADVECTION, weights=S.W_LEARNED, gate_threshold=0.5)
        assert workspace(mesh, p) == 0


def test_positivity_safeguard_is_euler_only():
    rect = S.Mesh.rect(16, 16, 0.0, 1.0, 0.0, 1.0)
    on = S.Params.make(eq=S.EULER, positivity=True)
    off = S.Params.make(eq=S.EULER)
    assert workspace(line(), on) > workspace(line(), off) > 0
    # 2D: 20 doubles for each of the 2 * 16 * 17 faces and a byte per cell
    assert workspace(rect, on) >= workspace(rect, off) + 20 * 8 * 2 * 16 * 17 + 256
    assert workspace(line(), S.Params.make(eq=S.BURGERS, positivity=True)) == 0
    assert workspace(rect, S.Params.make(eq=S.ADVECTION, positivity=True)) == 0
    bad = S.Params.make(eq=S.EULER)
    bad.positivity = 2
    assert state_doubles(line(), bad) == 0


def test_burgers_is_1d_only():
    rect = S.Mesh.rect(16, 16, 0.0, 1.0, 0.0, 1.0)
    assert workspace(line(), S.Params.make(eq=S.BURGERS)) > 0
    assert workspace(rect, S.Params.make(eq=S.BURGERS)) == 0


def bf16_bits(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF


def test_gate_packing_follows_the_matrix_layout():
    """Lane l holds, for the 32x32x16 BF16 instruction, W1[l%32][8(l/32)+e]
    (as BF16 pairs, element 2i in the low half of word i), W2 in K-chunk q at
    the hidden unit its first-layer accumulator item 8q+e holds, and b1, b2,
    w3 at its 16 accumulator rows 8(v/4)+4(l/32)+v%4."""
    nf = S.GATE_NFEATURES
    rng = np.random.default_rng(0)
    p = rng.normal(size=S.GATE_NPARAMS).astype(np.float32)
    W1 = p[:32 * nf].reshape(32, nf)
    b1 = p[32 * nf:32 * nf + 32]
    W2 = p[32 * nf + 32:32 * nf + 1056].reshape(32, 32)
    b2 = p[32 * nf + 1056:32 * nf + 1088]
    w3 = p[32 * nf + 1088:32 * nf + 1120]
    b3 = p[32 * nf + 1120]
    raw = S.gate_pack(p)
    assert raw.size == 64 * 256
    lanes = raw.view(np.uint32).reshape(64, 64)

    def row(lane, v):
        return 8 * (v // 4) + 4 * (lane // 32) + v % 4

    for lane in range(64):
        r, h = lane % 32, lane // 32
        words = lanes[lane]
        halves = np.stack([words & 0xFFFF, words >> 16], axis=1).reshape(-1)
        np.testing.assert_array_equal(halves[0:8], bf16_bits(W1[r, 8 * h:8 * h + 8]))
        for q in range(2):
            units = [row(32 * h, 8 * q + e) for e in range(8)]
            np.testing.assert_array_equal(halves[8 + 8 * q:16 + 8 * q], bf16_bits(W2[r, units]))
        f = words.view(np.float32)
        rows = [row(lane, v) for v in range(16)]
        np.testing.assert_array_equal(f[12:28], b1[rows])
        np.testing.assert_array_equal(f[28:44], b2[rows])
        np.testing.assert_array_equal(f[44:60], w3[rows])
        assert f[60] == b3
    # the second layer sees every hidden unit exactly once per lane half
    for h in range(2):
        units = sorted(row(32 * h, 8 * q + e) for q in range(2) for e in range(8))
        assert units == sorted(set(units)) and len(units) == 16
