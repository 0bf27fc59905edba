"""Pins for the variable-coefficient diffusion oracle and its gradient."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import PERIODIC as P
from tests import brute


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    u = rng.uniform(0, 1, size=shape)
    k = rng.uniform(0.05, 0.2, size=shape)
    t = rng.uniform(0, 1, size=shape)
    return u, k, t


def test_constant_kappa_is_heat_stencil():
    u, _, _ = _fields((6, 7, 8), 1)
    k0, dt = 0.15, 0.1
    kap = np.full(u.shape, k0)
    got = oracle.diffusion_step(u, kap, dt)
    want = oracle.sweep(u, synth.heat_star(3, dt * k0).coeffs, (P, P, P), 0.0)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_step_matches_brute_force_and_is_symmetric():
    u, k, _ = _fields((3, 4, 5), 2)
    dt = 0.1
    A = brute.diffusion_operator(k, dt)
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-16)
    np.testing.assert_allclose(A.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.diffusion_step(u, k, dt).ravel(), A @ u.ravel(),
                               rtol=0, atol=1e-15)
    lam = np.random.default_rng(3).standard_normal(u.shape)
    np.testing.assert_allclose(oracle.diffusion_step_transpose(lam, k, dt).ravel(),
                               A.T @ lam.ravel(), rtol=0, atol=1e-15)


def test_step_conserves_sum():
    u, k, _ = _fields((8, 9, 10), 4)
    y = oracle.diffusion_step(u, k, 0.1)
    assert abs(math.fsum(y.ravel()) - math.fsum(u.ravel())) < 1e-12


def test_kappa_vjp_matches_brute_derivative():
    """d(A(kappa) u)/dkappa_j from brute-force operators at kappa +- eps e_j
    (exact here: the step is linear in kappa, so the central difference has
    no truncation error)."""
    u, k, _ = _fields((3, 3, 4), 5)
    dt = 0.1
    lam = np.random.default_rng(6).standard_normal(u.shape)
    g = oracle.diffusion_kappa_vjp(u, lam, dt)
    eps = 1e-3
    for j in range(u.size):
        kp = k.copy().ravel()
        km = k.copy().ravel()
        kp[j] += eps
        km[j] -= eps
        Ap = brute.diffusion_operator(kp.reshape(u.shape), dt)
        Am = brute.diffusion_operator(km.reshape(u.shape), dt)
        d = ((Ap - Am) @ u.ravel()) / (2 * eps)
        assert abs(g.ravel()[j] - d @ lam.ravel()) <= 1e-11


def test_gradient_central_differences():
    shape = (6, 6, 6)
    u0, k, t = _fields(shape, 7)
    dt, n = 0.1, 20

    def loss(uu, kk):
        return oracle.diffusion_loss(oracle.diffusion_forward(uu, kk, dt, n)[-1], t)

    L, gu, gk = oracle.diffusion_gradient(u0, k, t, dt, n)
    assert abs(L - loss(u0, k)) == 0.0
    rng = np.random.default_rng(8)
    # u0: the loss is quadratic in u0, so central differences are exact up to rounding
    for j in rng.choice(u0.size, 12, replace=False):
        e = np.zeros(u0.size)
        e[j] = 1e-3
        e = e.reshape(shape)
        fd = (loss(u0 + e, k) - loss(u0 - e, k)) / 2e-3
        assert abs(fd - gu.ravel()[j]) <= 1e-7 * max(1.0, np.abs(gu).max())
    for j in rng.choice(k.size, 12, replace=False):
        e = np.zeros(k.size)
        e[j] = 1e-5
        e = e.reshape(shape)
        fd = (loss(u0, k + e) - loss(u0, k - e)) / 2e-5
        assert abs(fd - gk.ravel()[j]) <= 1e-6 * np.abs(gk).max()
    for _ in range(3):
        du = rng.standard_normal(shape)
        dk = rng.standard_normal(shape)
        eps = 1e-6
        fd = (loss(u0 + eps * du, k + eps * dk) - loss(u0 - eps * du, k - eps * dk)) / (2 * eps)
        an = float(np.vdot(gu, du) + np.vdot(gk, dk))
        assert abs(fd - an) <= 1e-6 * abs(an)


@pytest.mark.parametrize("dtype", [np.float32])
def test_forward_rounds_state(dtype):
    u, k, _ = _fields((4, 5, 6), 9)
    y = oracle.diffusion_step(u.astype(dtype), k.astype(dtype), 0.1)
    assert y.dtype == dtype
    want = oracle.diffusion_step(u.astype(dtype).astype(np.float64),
                                 k.astype(dtype).astype(np.float64), 0.1).astype(dtype)
    np.testing.assert_array_equal(y, want)
