"""Two local-element functions per step on the GPU against the oracle's
two-stage step: the one-thread-per-point path, the fused two-level 3D star
kernel, the composition case (alpha = 0) value for value, and Heun's method
on a full-size periodic mode."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1502_03504_amd as L
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests.gpu_util import TOL, empty_grid, grid_from, rel_err

pytestmark = pytest.mark.gpu


def _run(u, first, second, alpha, bc, n, h=1):
    a, b = grid_from(u, h), empty_grid(u.shape, h, u.dtype)
    idx = L.lope_iterate_stages(a, b, first, second, alpha, bc, n)
    return (a, b)[idx]


CASES = [
    # ndim, shape, kinds, first (kind, r), second (kind, r): the one-thread-per-point
    # path unless both are radius-1 3D stars or radius-1 2D stencils (fused kernels)
    (1, (50,), (D,), ("box", 2), ("box", 1)),
    (2, (33, 41), (P, D), ("box", 1), ("star", 2)),
    (3, (10, 13, 17), (D, P, D), ("box", 1), ("box", 1)),
    (3, (20, 24, 36), (P, P, P), ("star", 1), ("star", 1)),   # fused 3D
    (3, (20, 24, 36), (D, D, P), ("star", 1), ("star", 1)),   # fused 3D
    (2, (40, 150), (P, D), ("box", 1), ("star", 1)),          # fused 2D (wave)
    (2, (40, 150), (D, D), ("star", 1), ("box", 1)),          # fused 2D (wave)
]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("alpha", [0.0, 0.45])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_matches_oracle_and_composition(case, alpha, dtype):
    ndim, shape, kinds, (k1, r1), (k2, r2) = CASES[case]
    rng = np.random.default_rng([synth.CFG_TEST, 980 + case])
    c1 = synth.contractive(synth.random_stencil(rng, ndim, r1, k1)).coeffs
    c2 = synth.contractive(synth.random_stencil(rng, ndim, r2, k2)).coeffs * 0.5
    s1, s2 = synth.Stencil(ndim, r1, c1), synth.Stencil(ndim, r2, c2)
    u = rng.uniform(0, 1, shape).astype(dtype)
    bc = (kinds, 0.4)
    n = 5
    got = _run(u, s1, s2, alpha, bc, n, h=r1).numpy()
    want = oracle.stages_iterate(u, c1, c2, alpha, kinds, 0.4, n)
    assert rel_err(got, want) <= TOL[dtype], rel_err(got, want)
    if alpha == 0.0:
        # the composition of two sweeps, value for value
        a, b = grid_from(u, max(r1, r2)), empty_grid(shape, max(r1, r2), dtype)
        for _ in range(n):
            L.lope_apply(a, b, s1, bc)
            L.lope_apply(b, a, s2, bc)
        np.testing.assert_array_equal(got, a.numpy())


@pytest.mark.parametrize("kinds", [(P, P, P), (D, D, P), (P, D, D)])
def test_two_steps_per_pass_each_wave_kernel(kinds):
    """Every wave-brick variant, chosen through the tuning table, makes two
    steps per pass: against the oracle, and with alpha = 0 bitwise equal to
    two sweeps per step."""
    from tests.gpu_util import variants_for
    rng = np.random.default_rng([synth.CFG_TEST, 985])
    c1 = synth.contractive(synth.random_stencil(rng, 3, 1, "star")).coeffs
    c2 = synth.contractive(synth.random_stencil(rng, 3, 1, "star")).coeffs * 0.5
    s1, s2 = synth.Stencil(3, 1, c1), synth.Stencil(3, 1, c2)
    u = rng.uniform(0, 1, (13, 22, 70)).astype(np.float32)
    bc = (kinds, 0.4)
    n = 5                                           # two passes of two steps, one of one
    waves = [(vid, info) for vid, info in variants_for(3, 1, np.float32) if info.startswith("star3dw_")]
    assert waves
    want = oracle.stages_iterate(u, c1, c2, 0.45, kinds, 0.4, n)
    a, b = grid_from(u, 1), empty_grid(u.shape, 1, np.float32)
    for _ in range(n):
        L.lope_apply(a, b, s1, bc)
        L.lope_apply(b, a, s2, bc)
    composed = a.numpy()
    probe = grid_from(u, 1)
    try:
        for vid, info in waves:
            L.lope_tune_set(probe, s1, vid, 4, bc=bc)
            got = _run(u, s1, s2, 0.45, bc, n).numpy()
            assert rel_err(got, want) <= TOL[np.float32], (info, rel_err(got, want))
            np.testing.assert_array_equal(_run(u, s1, s2, 0.0, bc, n).numpy(), composed, err_msg=info)
    finally:
        L.lope_tune_set(probe, s1, 0, 4, bc=bc)


def test_first_stencil_reach_sets_the_halo():
    """The intermediate's halo comes from the rule, so only the first
    stencil's reach is checked against the grid."""
    rng = np.random.default_rng([synth.CFG_TEST, 990])
    u = rng.uniform(0, 1, (16, 20)).astype(np.float32)
    s1 = synth.Stencil(2, 1, synth.contractive(synth.random_stencil(rng, 2, 1, "box")).coeffs)
    s2 = synth.Stencil(2, 3, synth.contractive(synth.random_stencil(rng, 2, 3, "star")).coeffs)
    got = _run(u, s1, s2, 0.2, ((P, P), 0.0), 3, h=1).numpy()
    want = oracle.stages_iterate(u, s1.coeffs, s2.coeffs, 0.2, (P, P), 0.0, 3)
    assert rel_err(got, want) <= 1e-5, rel_err(got, want)
    with pytest.raises(L.LopeError) as e:
        _run(u, s2, s1, 0.2, ((P, P), 0.0), 1, h=1)
    assert e.value.code == -2


def test_heun_256_f64_closed_form():
    """Heun's method for the periodic heat equation at 256^3: a cosine mode
    decays by 1/2 + (1 + dt l)^2 / 2 per step."""
    n, dt, steps = 256, 0.1, 200
    ks = (3, 5, 2)
    lap = -4 * sum(math.sin(math.pi * k / n) ** 2 for k in ks)
    u = synth.mode_field((n, n, n), ks, (P, P, P))
    heat = synth.heat_star(3, dt)                  # I + dt * L (7-point)
    half = synth.Stencil(3, 1, 0.5 * heat.coeffs)
    out = _run(u, heat, half, 0.5, ((P, P, P), 0.0), steps).interior()
    want = torch.from_numpy(u).cuda() * (0.5 + 0.5 * (1 + dt * lap) ** 2) ** steps
    err = float((out - want).abs().max()) / float(want.abs().max())
    assert err <= 1e-12, err
