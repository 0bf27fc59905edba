"""Pins of per-axis (left/right) halo widths and the reach of a stencil: the
M:*:N halo of section 2.2 and the halo-width constraint of section 3.5."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests import brute


@pytest.mark.parametrize("shape,widths,kinds", [
    ((7,), [(2, 0)], (P,)),
    ((7,), [(0, 3)], (D,)),
    ((5, 6), [(1, 0), (0, 2)], (D, P)),
    ((5, 6), [(3, 1), (2, 0)], (P, P)),
    ((3, 4, 5), [(0, 1), (2, 0), (1, 1)], (D, P, D)),
    ((2, 3, 2), [(4, 0), (0, 5), (3, 3)], (P, D, P)),     # wider than the interior
])
def test_asymmetric_halo_fill_matches_cell_by_cell(shape, widths, kinds):
    rng = np.random.default_rng([synth.CFG_TEST, 950])
    u = rng.uniform(-1, 1, shape)
    g = 0.625
    pad = oracle.halo_fill(u, widths, kinds, g)
    d = u.ndim
    assert pad.shape == tuple(shape[npax] + sum(widths[d - 1 - npax]) for npax in range(d))
    for idx in itertools.product(*[range(s) for s in pad.shape]):
        z = [idx[npax] - widths[d - 1 - npax][0] for npax in range(d)]
        assert pad[idx] == brute.halo_value(u, z, kinds, g), (idx, z)


def test_symmetric_width_is_the_same_on_every_side():
    rng = np.random.default_rng([synth.CFG_TEST, 951])
    u = rng.uniform(0, 1, (4, 6)).astype(np.float32)
    np.testing.assert_array_equal(oracle.halo_fill(u, 2, (D, P), 0.5),
                                  oracle.halo_fill(u, [(2, 2), (2, 2)], (D, P), 0.5))
    with pytest.raises(ValueError):
        oracle.halo_widths([(1, -1), (0, 0)], 2)
    with pytest.raises(ValueError):
        oracle.halo_widths([(1, 1)], 2)


def test_reach_of_single_taps():
    """A single tap at offset o reaches max(0, -o_a) to the left and
    max(0, o_a) to the right of every axis."""
    r = 2
    for o in itertools.product(range(-r, r + 1), repeat=2):
        c = np.zeros((2 * r + 1,) * 2)
        c[o[1] + r, o[0] + r] = 0.75           # numpy order: (y, x)
        want = [(max(0, -o[0]), max(0, o[0])), (max(0, -o[1]), max(0, o[1]))]
        assert oracle.stencil_reach(c) == want, o
    assert oracle.stencil_reach(np.zeros((3, 3, 3))) == [(0, 0)] * 3


def test_reach_counts_taps_after_rounding():
    c = np.zeros((5,))
    c[2] = 1.0
    c[4] = 1e-50            # zero once rounded to float32
    assert oracle.stencil_reach(c, np.float64) == [(0, 2)]
    assert oracle.stencil_reach(c, np.float32) == [(0, 0)]


def test_one_sided_sweep_reads_only_within_reach():
    """The sweep equals the sum over taps of the padded array built with the
    reach as halo widths: the cells beyond the reach are never needed."""
    rng = np.random.default_rng([synth.CFG_TEST, 952])
    for kinds in ((P, D), (D, P), (P, P)):
        c = np.zeros((5, 5))
        c[2:, :3] = rng.uniform(-1, 1, (3, 3))     # taps at oy in 0..2, ox in -2..0
        u = rng.uniform(0, 1, (6, 7))
        reach = oracle.stencil_reach(c)
        assert reach == [(2, 0), (0, 2)]
        pad = oracle.halo_fill(u, reach, kinds, 0.25)
        want = np.zeros(u.shape)
        for (iy, ix), cv in np.ndenumerate(c):
            if cv == 0:
                continue
            oy, ox = iy - 2, ix - 2
            want += cv * pad[reach[1][0] + oy: reach[1][0] + oy + u.shape[0],
                             reach[0][0] + ox: reach[0][0] + ox + u.shape[1]]
        np.testing.assert_allclose(oracle.sweep(u, c, kinds, 0.25), want, rtol=0, atol=1e-13)


def test_upwind_shift_is_a_roll():
    """A one-sided tap taking the left neighbour on a periodic axis moves the
    field one cell right per sweep, exactly."""
    rng = np.random.default_rng([synth.CFG_TEST, 953])
    u = rng.uniform(0, 1, (5, 9)).astype(np.float32)
    c = np.zeros((3, 3))
    c[1, 0] = 1.0
    assert oracle.stencil_reach(c) == [(1, 0), (0, 0)]
    for n in (1, 4, 9):
        np.testing.assert_array_equal(oracle.iterate(u, c, (P, D), 0.0, n), np.roll(u, n, axis=1))
