"""Pins of the oracle's convergence-driven iteration (section 3.2, the
do-while loop; the paper leaves the test undefined: here the max-norm change
of one sweep, checked every m sweeps, against a tolerance)."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests import brute


def _cos_mode(shape, ks):
    """prod_a cos(2 pi k_a x_a / N_a): value exactly 1 at the origin, max |.| = 1."""
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    u = np.ones(shape)
    for g, n, k in zip(grids, shape, ks):
        u = u * np.cos(2 * np.pi * k * g / n)
    return u


@pytest.mark.parametrize("m", [1, 3, 7])
def test_stop_step_matches_closed_form(m):
    """Periodic heat stencil on a separable cosine mode: u_t = lam^t u_0, so
    the one-sweep change has max norm lam^(t-1) (1 - lam) exactly at the
    origin; the stop is the first multiple of m where that is <= tol."""
    shape, ks, r = (24, 40), (2, 3), 0.25
    lam = 1.0 - 4 * r * sum(math.sin(math.pi * k / n) ** 2 for k, n in zip(ks, shape))
    u0 = _cos_mode(shape, ks)
    st = synth.heat_star(2, r)
    tol = 1e-3
    res = lambda t: lam ** (t - 1) * (1 - lam)
    want = next(t for t in range(m, 100000, m) if res(t) <= tol)
    # tol is not within rounding of a checked residual
    assert res(want) < tol * (1 - 1e-6) and (want == m or res(want - m) > tol * (1 + 1e-6))
    u, steps, r_got = oracle.iterate_until(u0, st.coeffs, (P, P), 0.0, 10 * want, m, tol)
    assert steps == want
    assert abs(r_got - res(want)) <= 1e-12
    np.testing.assert_allclose(u, lam ** want * u0, atol=1e-12)


def test_brute_force_mixed_rule():
    """Dense operator u -> A u + g b on a tiny grid with mixed rules and a
    random stencil; the residual of every step taken from the matrix run."""
    rng = np.random.default_rng([synth.CFG_TEST, 900])
    shape, kinds, g = (5, 6), (D, P), 0.7
    st = synth.contractive(synth.random_stencil(rng, 2, 1, "box"))
    A, b = brute.sweep_operator(shape, st.coeffs, kinds)
    u0 = rng.uniform(-1, 1, shape)
    m, tol, max_steps = 2, 1e-4, 400
    x = u0.reshape(-1).copy()
    want_steps, want_res = max_steps, float("nan")
    for t in range(max_steps):
        y = A @ x + g * b
        if (t + 1) % m == 0:
            want_res = float(np.max(np.abs(y - x)))
            x = y
            if want_res <= tol:
                want_steps = t + 1
                break
        else:
            x = y
    u, steps, res = oracle.iterate_until(u0, st.coeffs, kinds, g, max_steps, m, tol)
    assert steps == want_steps < max_steps
    assert abs(res - want_res) <= 1e-12
    np.testing.assert_allclose(u.reshape(-1), x, atol=1e-12)


def test_special_cases():
    rng = np.random.default_rng([synth.CFG_TEST, 901])
    st = synth.heat_star(2, 0.125)
    u0 = rng.uniform(0, 1, (9, 11))
    # infinite tolerance: stops at the first check
    u, steps, _ = oracle.iterate_until(u0, st.coeffs, (P, P), 0.0, 50, 4, math.inf)
    assert steps == 4
    np.testing.assert_array_equal(u, oracle.iterate(u0, st.coeffs, (P, P), 0.0, 4))
    # negative tolerance: never converges, equals the fixed-count iteration
    u, steps, res = oracle.iterate_until(u0, st.coeffs, (P, P), 0.0, 13, 4, -1.0)
    assert steps == 13 and res > 0
    np.testing.assert_array_equal(u, oracle.iterate(u0, st.coeffs, (P, P), 0.0, 13))
    # check interval beyond the budget: no check, no residual
    u, steps, res = oracle.iterate_until(u0, st.coeffs, (P, P), 0.0, 5, 6, 1.0)
    assert steps == 5 and math.isnan(res)
    # a fixed point (constant field, dyadic weights summing to 1): residual 0 at the first check
    c = np.full((9, 11), 0.375, dtype=np.float32)
    u, steps, res = oracle.iterate_until(c, st.coeffs, (P, D), 0.375, 100, 3, 0.0)
    assert steps == 3 and res == 0.0 and u.dtype == np.float32
    np.testing.assert_array_equal(u, c)
    # empty field
    u, steps, res = oracle.iterate_until(np.zeros((0, 4)), st.coeffs, (P, P), 0.0, 10, 1, 0.0)
    assert steps == 0 and u.shape == (0, 4)


def test_float32_residual_is_exact_difference():
    """For float32 states the residual is the exact float64 difference of the
    two float32 states (no rounding), taken after the state was rounded."""
    rng = np.random.default_rng([synth.CFG_TEST, 902])
    st = synth.heat_star(3, 0.125)
    u0 = rng.uniform(0, 1, (6, 7, 8)).astype(np.float32)
    u, steps, res = oracle.iterate_until(u0, st.coeffs, (P, P, P), 0.0, 1, 1, -1.0)
    prev = u0.astype(np.float64)
    want = float(np.max(np.abs(oracle.sweep(u0, st.coeffs, (P, P, P), 0.0).astype(np.float64) - prev)))
    assert steps == 1 and res == want
    assert u.dtype == np.float32
