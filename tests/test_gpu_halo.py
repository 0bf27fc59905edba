"""Per-axis (left, right) halos and one-sided stencils on the GPU, against the
oracle: the halo fill, sweeps that read a halo on one side only, and the
adjoint, which reaches the other way."""
import numpy as np
import pytest
import torch

import oracle
import paper_1502_03504_amd as L
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests.gpu_util import TOL, rel_err

pytestmark = pytest.mark.gpu


def _grid(u, halo, fill=0.0):
    tdt = torch.float64 if u.dtype == np.float64 else torch.float32
    g = L.Grid.allocate(u.shape, halo, tdt, "cuda", fill=fill)
    g.interior().copy_(torch.from_numpy(np.ascontiguousarray(u)).cuda())
    return g


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape,halo,kinds", [
    ((9,), [(3, 0)], (P,)),
    ((9,), [(0, 2)], (D,)),
    ((6, 7), [(1, 0), (0, 2)], (D, P)),
    ((6, 7), [(2, 3), (4, 0)], (P, D)),
    ((4, 5, 6), [(0, 1), (2, 0), (1, 1)], (D, P, D)),
    ((2, 3, 2), [(4, 0), (0, 5), (3, 3)], (P, P, P)),   # wider than the interior
])
def test_asymmetric_halo_fill_bit_exact(shape, halo, kinds, dtype):
    rng = np.random.default_rng([synth.CFG_TEST, 960])
    u = rng.uniform(-1, 1, shape).astype(dtype)
    g = _grid(u, halo, fill=np.nan)
    L.lope_halo_fill(g, (kinds, 0.375))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g.padded().cpu().numpy(), oracle.halo_fill(u, halo, kinds, 0.375))


def _one_sided(rng, ndim):
    """Random taps on the low side of x and the high side of y (radius 1)."""
    c = np.zeros((3,) * ndim)
    if ndim == 2:
        c[1:, :2] = rng.uniform(-1, 1, (2, 2))
    else:
        c[:, 1:, :2] = rng.uniform(-1, 1, (3, 2, 2))
    c *= 0.9 / np.abs(c).sum()
    return c


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("ndim", [2, 3])
def test_one_sided_stencil_on_one_sided_halos(ndim, dtype):
    rng = np.random.default_rng([synth.CFG_TEST, 961 + ndim])
    c = _one_sided(rng, ndim)
    st = synth.Stencil(ndim, 1, c)
    reach = oracle.stencil_reach(c, dtype)
    assert reach[0] == (1, 0) and reach[1] == (0, 1)
    shape = (40, 37) if ndim == 2 else (12, 17, 21)
    kinds = (P, D) if ndim == 2 else (P, D, D)
    u = rng.uniform(0, 1, shape).astype(dtype)
    n = 7
    want = oracle.iterate(u, c, kinds, 0.5, n)
    ref = None
    for td in (1, 2, 3, 4):
        a, b = _grid(u, reach), _grid(np.zeros_like(u), reach)
        idx = L.lope_iterate(a, b, st, (kinds, 0.5), n, tdepth=td)
        got = (a, b)[idx].numpy()
        assert rel_err(got, want) <= TOL[dtype], (td, rel_err(got, want))
        if ref is None:
            ref = got
        else:
            np.testing.assert_array_equal(got, ref, err_msg="depth %d" % td)
    # the halo on the far side is not needed, and a missing near side is refused
    wrong = [(0, 1)] + reach[1:]
    with pytest.raises(L.LopeError) as e:
        L.lope_apply(_grid(u, wrong), _grid(u, wrong), st, (kinds, 0.5))
    assert e.value.code == -2


def test_upwind_roll_on_left_halo_only():
    """A single left tap on a periodic axis moves the field one cell per sweep."""
    rng = np.random.default_rng([synth.CFG_TEST, 964])
    u = rng.uniform(0, 1, (6, 50)).astype(np.float32)
    c = np.zeros((3, 3))
    c[1, 0] = 1.0
    st = synth.Stencil(2, 1, c)
    a, b = _grid(u, [(1, 0), (0, 0)]), _grid(np.zeros_like(u), [(1, 0), (0, 0)])
    idx = L.lope_iterate(a, b, st, ((P, D), 0.0), 13)
    np.testing.assert_array_equal((a, b)[idx].numpy(), np.roll(u, 13, axis=1))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_adjoint_of_one_sided_stencil_reads_the_other_side(dtype):
    rng = np.random.default_rng([synth.CFG_TEST, 965])
    c = _one_sided(rng, 2)
    st = synth.Stencil(2, 1, c)
    kinds = (D, P)
    ybar = rng.uniform(-1, 1, (23, 31)).astype(dtype)
    want, _ = oracle.adjoint(ybar, c, kinds)
    mirrored = [(0, 1), (1, 0)]                      # forward reach (1,0),(0,1) reflected
    y = _grid(ybar, mirrored)
    x = _grid(np.zeros_like(ybar), mirrored)
    L.lope_apply_adjoint(y, x, st, (kinds, 0.0))
    assert rel_err(x.numpy(), want) <= TOL[dtype]
    with pytest.raises(L.LopeError) as e:
        L.lope_apply_adjoint(_grid(ybar, [(1, 0), (0, 1)]), x, st, (kinds, 0.0))
    assert e.value.code == -2
