"""Grids past 32-bit indexing: more than 2^31 elements in one buffer, and 3D
planes of more than 2^31 bytes (where the kernels with 32-bit in-plane byte
offsets must step aside).  Checked on sampled outputs the oracle computes one
by one, corners included.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1502_03504_amd as L
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests.gpu_util import grid_from, rel_err

pytestmark = pytest.mark.gpu


def _points(shape, count, seed):
    rng = np.random.default_rng(seed)
    pts = [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(count)]
    pts += [tuple(0 for _ in shape), tuple(n - 1 for n in shape),
            tuple((0 if i % 2 else n - 1) for i, n in enumerate(shape))]
    return pts


def _check(u, st, bc, runs, seed):
    a = grid_from(u, st.radius)
    b = a.empty_like()
    for n, tdepth in runs:
        a.interior().copy_(torch.from_numpy(u).cuda())
        idx = L.lope_iterate(a, b, st, bc, n, tdepth=tdepth)
        out = (a, b)[idx].interior()
        pts = _points(u.shape, 32, seed + n)
        got = np.array([out[p].item() for p in pts])
        want = oracle.sweep_at(u, st.coeffs, bc.kinds, bc.value, n, pts)
        assert rel_err(got, want) <= 1e-5, (n, tdepth, rel_err(got, want))
    del a, b
    torch.cuda.empty_cache()


def test_2d_box_more_than_2_31_elements():
    shape = (46400, 46400)
    assert shape[0] * shape[1] > 2 ** 31
    rng = np.random.default_rng([synth.CFG_TEST, 501])
    u = rng.random(shape, dtype=np.float32)
    st = synth.dyadic_stencil(rng, "box")
    bc = synth.Boundary((D, P), 0.25)
    _check(u, st, bc, [(1, 1), (3, 0), (4, 4)], 510)


def test_3d_heat_plane_beyond_2_31_bytes():
    shape = (3, 23200, 23200)            # one plane holds 2.15 GB of float32
    assert shape[1] * shape[2] * 4 > 2 ** 31
    rng = np.random.default_rng([synth.CFG_TEST, 502])
    u = rng.random(shape, dtype=np.float32)
    st = synth.heat_star(3, 0.125)
    bc = synth.Boundary((P, P, P), 0.0)
    g = L.Grid.allocate(shape, 1, torch.float32, "cuda")
    for td in (0, 1, 2, 4):
        vid = L.lope_select_variant(g, st, tdepth=td, bc=bc)
        name = L.lope_variant_info(vid) if vid > 0 else "generic"
        assert not name.startswith(("star3dw_", "star3df_")), (td, name)
    del g
    _check(u, st, bc, [(1, 1), (2, 0), (4, 2), (4, 4)], 520)
