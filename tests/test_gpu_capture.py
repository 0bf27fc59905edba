"""Calls that only enqueue kernels, recorded into a caller's HIP graph.

Every compute call except lope_iterate_until enqueues launches and nothing
else (no memset or copy nodes, no host wait), so a capturing stream records
it.  Each graph is replayed three times, with fresh inputs and unrelated
eager launches between replays, and every replay must equal the eager run
value for value.  lope_iterate_until refuses a capturing stream.
"""
import numpy as np
import pytest
import torch

import paper_1502_03504_amd as L
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests.gpu_util import empty_grid, grid_from

pytestmark = pytest.mark.gpu


def _field(shape, dtype, seed):
    rng = np.random.default_rng([synth.CFG_TEST, seed])
    return rng.uniform(-1, 1, size=shape).astype(dtype)


def _replay_matches(record, inputs, outputs):
    """record(): enqueue the calls under test.  inputs: (grid, array) pairs
    reset before each run.  outputs(): host arrays of the results, which
    every replay must reproduce exactly (reductions sum in a fixed order)."""

    def reset():
        for g, u in inputs:
            g.interior().copy_(torch.from_numpy(u).cuda())

    reset()
    record()
    torch.cuda.synchronize()
    want = outputs()
    other = _field((33, 21, 40), np.float32, 99)
    oa, ob = grid_from(other, 1), empty_grid(other.shape, 1, np.float32)
    g = torch.cuda.CUDAGraph()
    reset()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        record()
    for rep in range(3):
        reset()
        L.lope_iterate(oa, ob, synth.heat_star(3, 0.1), ((P, D, P), 0.5), 3)   # eager work in between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = outputs()
        for k, (x, y) in enumerate(zip(got, want)):
            np.testing.assert_array_equal(x, y, err_msg="replay %d output %d" % (rep, k))
    del g


@pytest.mark.parametrize("bc", [(P, P, P), (D, P, D)])
def test_iterate_3d_float32_captured(bc):
    """The tuned 3D path (fused sweeps per pass, remainder pass) in a graph."""
    u = _field((70, 45, 130), np.float32, 1)
    a, b = grid_from(u, 1), empty_grid(u.shape, 1, np.float32)
    idx = []

    def record():
        idx.append(L.lope_iterate(a, b, synth.heat_star(3, 0.1), (bc, 0.25), 11))

    _replay_matches(record, [(a, u)], lambda: [(a, b)[idx[0]].numpy()])
    assert len(set(idx)) == 1


def test_iterate_2d_and_stages_captured():
    u2 = _field((300, 257), np.float64, 2)
    a2, b2 = grid_from(u2, 1), empty_grid(u2.shape, 1, np.float64)
    u3 = _field((40, 37, 70), np.float32, 3)
    a3, b3 = grid_from(u3, 1), empty_grid(u3.shape, 1, np.float32)
    st = synth.heat_star(3, 0.1)
    box = synth.dyadic_stencil(synth.rng_for(synth.CFG_TEST, 8), "box")
    idx = []

    def record():
        idx.append(L.lope_iterate(a2, b2, box, ((P, D), 0.0), 9))
        idx.append(L.lope_iterate_stages(a3, b3, st, st, 0.5, ((P, P, P), 0.0), 5))

    def outputs():
        return [(a2, b2)[idx[0]].numpy(), (a3, b3)[idx[1]].numpy()]

    _replay_matches(record, [(a2, u2), (a3, u3)], outputs)


def test_adjoint_and_var_captured():
    y = _field((23, 31, 66), np.float64, 4)
    ya, xa = grid_from(y, 4), empty_grid(y.shape, 4, np.float64)
    gbar = L.gbar_buffer()
    u = _field((20, 24, 65), np.float32, 5)
    kap = (0.5 + 0.25 * _field(u.shape, np.float32, 6)).astype(np.float32)
    ua, ub = grid_from(u, 1), empty_grid(u.shape, 1, np.float32)
    ka = grid_from(kap, 1)
    st = synth.laplacian8_star(3, 0.05)

    def record():
        L.lope_apply_adjoint(ya, xa, st, ((D, D, D), 0.0), gbar=gbar)
        L.lope_apply_var(ua, ub, ka, 0.1, ((P, P, P), 0.0))

    def outputs():
        return [xa.numpy(), gbar[:1].cpu().numpy(), ub.numpy()]

    _replay_matches(record, [(ya, y), (ua, u)], outputs)


def test_iterate_until_refuses_capture():
    u = _field((16, 17, 18), np.float32, 7)
    a, b = grid_from(u, 1), empty_grid(u.shape, 1, np.float32)
    scratch = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with pytest.raises(L.LopeError, match="captured"):
        with torch.cuda.graph(g):
            L.lope_iterate_until(a, b, synth.heat_star(3, 0.1), ((P, P, P), 0.0), 100, 10, 1e-6, scratch=scratch)
    torch.cuda.synchronize()
