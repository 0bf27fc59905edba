"""Pins of the oracle's two-stage step (two local-element functions applied in
sequence with a share of the starting state): the fusion of small functions
the paper leaves to the compiler (section 3.5) and the intermediate results of
multi-step updates it does not store automatically (section 5, Limitations)."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests import brute


def _cos_mode(shape, ks):
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    u = np.ones(shape)
    for g, n, k in zip(grids, shape, ks):
        u = u * np.cos(2 * np.pi * k * g / n)
    return u


def _laplacian(ndim, scale):
    """scale * (5- or 7-point Laplacian), radius 1."""
    c = np.zeros((3,) * ndim)
    c[(1,) * ndim] = -2.0 * ndim * scale
    for a in range(ndim):
        for s in (0, 2):
            idx = [1] * ndim
            idx[a] = s
            c[tuple(idx)] = scale
    return c


def test_heun_and_midpoint_decay_closed_form():
    """Periodic heat equation du/dt = Lu on a cosine mode (L's eigenvalue l):
    Heun (v = Su, u' = u/2 + S v/2 with S = I + dt L) multiplies the mode by
    1/2 + (1 + dt l)^2/2 per step; the midpoint rule (v = u + dt/2 L u,
    u' = u + dt L v) by 1 + dt l + (dt l)^2 / 2."""
    shape, ks, dt = (24, 40), (2, 3), 0.1
    lap = -4 * sum(math.sin(math.pi * k / n) ** 2 for k, n in zip(ks, shape))
    u0 = _cos_mode(shape, ks)
    ident = np.zeros((3, 3))
    ident[1, 1] = 1.0
    S = ident + _laplacian(2, dt)
    n = 25
    heun = oracle.stages_iterate(u0, S, 0.5 * S, 0.5, (P, P), 0.0, n)
    np.testing.assert_allclose(heun, (0.5 + 0.5 * (1 + dt * lap) ** 2) ** n * u0, rtol=0, atol=1e-13)
    mid = oracle.stages_iterate(u0, ident + _laplacian(2, dt / 2), _laplacian(2, dt), 1.0, (P, P), 0.0, n)
    np.testing.assert_allclose(mid, (1 + dt * lap + (dt * lap) ** 2 / 2) ** n * u0, rtol=0, atol=1e-13)


def test_alpha_zero_is_the_composition():
    rng = np.random.default_rng([synth.CFG_TEST, 970])
    u = rng.uniform(0, 1, (9, 11)).astype(np.float32)
    c1 = synth.random_stencil(rng, 2, 1, "box").coeffs
    c2 = synth.random_stencil(rng, 2, 2, "star").coeffs
    want = oracle.sweep(oracle.sweep(u, c1, (D, P), 0.3), c2, (D, P), 0.3)
    np.testing.assert_array_equal(oracle.stages_step(u, c1, c2, 0.0, (D, P), 0.3), want)


@pytest.mark.parametrize("kinds", [(D, P), (P, D), (D, D)])
def test_brute_force_with_dirichlet_intermediate(kinds):
    """u' = alpha u + A2 (A1 u + g b1) + g b2 from dense operators built entry
    by entry: the intermediate's halo follows the same rule (g on Dirichlet)."""
    rng = np.random.default_rng([synth.CFG_TEST, 971])
    shape, g, alpha = (5, 6), 0.7, -0.35
    c1 = synth.random_stencil(rng, 2, 1, "box").coeffs
    c2 = synth.random_stencil(rng, 2, 1, "star").coeffs
    A1, b1 = brute.sweep_operator(shape, c1, kinds)
    A2, b2 = brute.sweep_operator(shape, c2, kinds)
    u = rng.uniform(-1, 1, shape)
    x = u.reshape(-1)
    want = alpha * x + A2 @ (A1 @ x + g * b1) + g * b2
    got = oracle.stages_step(u, c1, c2, alpha, kinds, g)
    np.testing.assert_allclose(got.reshape(-1), want, rtol=0, atol=1e-13)
    # and over several steps
    for _ in range(3):
        x = alpha * x + A2 @ (A1 @ x + g * b1) + g * b2
    np.testing.assert_allclose(oracle.stages_iterate(u, c1, c2, alpha, kinds, g, 4).reshape(-1),
                               alpha * x + A2 @ (A1 @ x + g * b1) + g * b2, rtol=0, atol=1e-12)


def test_float32_rounds_the_intermediate_and_the_result():
    """The first function's result is a float32 state (rounded once), the step
    result is rounded once: the float32 step equals the float64 arithmetic on
    the rounded intermediate."""
    rng = np.random.default_rng([synth.CFG_TEST, 972])
    u = rng.uniform(0, 1, (7, 8)).astype(np.float32)
    c1 = synth.random_stencil(rng, 2, 1, "box").coeffs
    c2 = synth.random_stencil(rng, 2, 1, "box").coeffs
    alpha = 0.3
    v = oracle.sweep(u, c1, (P, P), 0.0)
    assert v.dtype == np.float32
    ext = np.pad(v.astype(np.float64), 1, mode="wrap")
    c2r = c2.astype(np.float32).astype(np.float64)
    want = float(np.float32(alpha)) * u.astype(np.float64)
    for iy in range(3):
        for ix in range(3):
            want = want + c2r[iy, ix] * ext[iy:iy + 7, ix:ix + 8]
    np.testing.assert_array_equal(oracle.stages_step(u, c1, c2, alpha, (P, P), 0.0), want.astype(np.float32))
