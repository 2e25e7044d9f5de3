"""The entry point that allocates nothing (shw_advance1d_static), called
through the C ABI, against the context-based entry point (shw_create +
shw_advance_to) on the same batches: the same step counts and states bit for
bit, on two calls in a row (the second on a smaller batch, so stale scratch
contents from the first would show), plus the host-side rejection of a batch
that does not fit the static scratch."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2304_09724_amd as S
from paper_2304_09724_amd import workloads as WL

pytestmark = pytest.mark.gpu


def reference(meshes, params, states, T):
    s = S.Solver(meshes, params)
    for i, st in enumerate(states):
        s.set_state(i, st)
    steps = s.advance_to(T, raise_nonphysical=False)
    return steps, [s.get_state(i) for i in range(len(meshes))], s.instance_status()


@pytest.mark.parametrize("positivity", [False, True])
def test_static_entry_point_matches_the_context_path(positivity):
    params = S.Params.make(eq=S.EULER, positivity=positivity)
    for count, seed, nmax in ((40, 8, 700), (7, 9, 300)):
        insts = WL.riemann_batch_1d(count=count, seed=seed, nmin=20, nmax=nmax)
        meshes = [S.Mesh.line(d.n, d.x0, d.x1, S.BC_TRANSMISSIVE) for d in insts]
        states = [d.state() for d in insts]
        T = np.full(count, 0.1)
        ref_steps, ref_states, ref_codes = reference(meshes, params, states, T)
        flat = torch.from_numpy(np.concatenate([st.reshape(-1) for st in states])).cuda()
        steps = S.advance1d_static(meshes, params, flat, T, raise_nonphysical=False)
        torch.cuda.synchronize()
        assert np.array_equal(steps, ref_steps)
        out = flat.cpu().numpy()
        off = 0
        for i, st in enumerate(ref_states):
            got = out[off:off + st.size].reshape(st.shape)
            off += st.size
            assert np.array_equal(got, st), (count, i)


def test_static_entry_point_rejects_what_does_not_fit():
    params = S.Params.make(eq=S.EULER)
    n = 2_000_000                      # 2e6 cells: state copies alone exceed 64 MiB
    meshes = [S.Mesh.line(n, 0.0, 1.0, S.BC_TRANSMISSIVE)]
    flat = torch.zeros(6 * n, dtype=torch.float64, device="cuda")
    with pytest.raises(S.ShwError) as e:
        S.advance1d_static(meshes, params, flat, [0.1])
    assert e.value.code == -6
    meshes = [S.Mesh.line(8, 0.0, 1.0, S.BC_TRANSMISSIVE)] * (S.STATIC_MAX_INSTANCES + 1)
    flat = torch.zeros(48 * len(meshes), dtype=torch.float64, device="cuda")
    with pytest.raises(S.ShwError) as e:
        S.advance1d_static(meshes, params, flat, np.full(len(meshes), 0.1))
    assert e.value.code == -6
