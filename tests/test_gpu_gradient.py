"""Gradients of the checkpointed diffusion driver against the oracle and
central finite differences."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1502_03504_amd.autograd import diffusion_gradient
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu


def _case(n, steps, seed=0):
    c = synth.case_diffusion(n=n, steps=steps, seed=seed)
    t = lambda a: torch.from_numpy(a).cuda()
    return c, t(c.u0), t(c.kappa), t(c.target)


def test_gradient_matches_central_differences_16():
    c, u0, k, tg = _case(16, 200)
    loss, gu, gk = diffusion_gradient(u0, k, tg, c.dt, c.steps, c.checkpoint_every)
    gu, gk = gu.cpu().numpy(), gk.cpu().numpy()
    u64, k64, t64 = (c.u0.astype(np.float64), c.kappa.astype(np.float64), c.target.astype(np.float64))

    def L(uu, kk):
        return oracle.diffusion_loss(oracle.diffusion_forward(uu, kk, c.dt, c.steps)[-1], t64)

    rng = np.random.default_rng(1)
    fd_u, an_u, fd_k, an_k = [], [], [], []
    for j in rng.choice(u64.size, 24, replace=False):
        e = np.zeros(u64.size)
        e[j] = 1e-3
        e = e.reshape(u64.shape)
        fd_u.append((L(u64 + e, k64) - L(u64 - e, k64)) / 2e-3)
        an_u.append(gu.ravel()[j])
    for j in rng.choice(k64.size, 24, replace=False):
        e = np.zeros(k64.size)
        e[j] = 1e-5
        e = e.reshape(k64.shape)
        fd_k.append((L(u64, k64 + e) - L(u64, k64 - e)) / 2e-5)
        an_k.append(gk.ravel()[j])
    assert rel_err(an_u, fd_u) <= 1e-4, rel_err(an_u, fd_u)
    assert rel_err(an_k, fd_k) <= 1e-4, rel_err(an_k, fd_k)
    for _ in range(4):
        du, dk = rng.standard_normal(u64.shape), rng.standard_normal(k64.shape)
        eps = 1e-6
        fd = (L(u64 + eps * du, k64 + eps * dk) - L(u64 - eps * du, k64 - eps * dk)) / (2 * eps)
        an = float(np.vdot(gu.astype(np.float64), du) + np.vdot(gk.astype(np.float64), dk))
        assert abs(fd - an) <= 1e-4 * abs(fd), (fd, an)


def test_gradient_matches_oracle_adjoint_48():
    c, u0, k, tg = _case(48, 200, seed=2)
    loss, gu, gk = diffusion_gradient(u0, k, tg, c.dt, c.steps, c.checkpoint_every)
    L, wu, wk = oracle.diffusion_gradient(c.u0, c.kappa, c.target, c.dt, c.steps)
    assert abs(float(loss) - L) <= 1e-5 * L
    assert rel_err(gu.cpu().numpy(), wu) <= 1e-5, rel_err(gu.cpu().numpy(), wu)
    assert rel_err(gk.cpu().numpy(), wk) <= 1e-4, rel_err(gk.cpu().numpy(), wk)


def test_gradient_float64_matches_oracle():
    """Float64 states: the kappa gradient is accumulated in float64 by the
    reverse kernels themselves; both gradients at the float64 bar."""
    c = synth.case_diffusion(n=20, steps=60, seed=5, dtype=np.float64)
    t = lambda a: torch.from_numpy(a).cuda()
    for every in (20, 7):
        loss, gu, gk = diffusion_gradient(t(c.u0), t(c.kappa), t(c.target), c.dt, c.steps, every)
        L, wu, wk = oracle.diffusion_gradient(c.u0, c.kappa, c.target, c.dt, c.steps)
        assert abs(float(loss) - L) <= 1e-12 * L
        assert rel_err(gu.cpu().numpy(), wu) <= 1e-12, rel_err(gu.cpu().numpy(), wu)
        assert rel_err(gk.cpu().numpy(), wk) <= 1e-12, rel_err(gk.cpu().numpy(), wk)


def test_checkpoint_interval_does_not_change_gradient():
    """dL/du0 is bitwise independent of the interval; dL/dkappa too for even
    intervals (every step pair fused); an odd interval splits some pairs,
    which changes only the order of the float32 accumulator's additions."""
    c, u0, k, tg = _case(24, 60, seed=3)
    ref = None
    for every in (20, 2, 60, 1, 7):
        loss, gu, gk = diffusion_gradient(u0, k, tg, c.dt, c.steps, every)
        cur = (loss.item(), gu.cpu().numpy(), gk.cpu().numpy())
        if ref is None:
            ref = cur
            continue
        assert cur[0] == ref[0]
        np.testing.assert_array_equal(cur[1], ref[1])
        if every % 2 == 0:
            np.testing.assert_array_equal(cur[2], ref[2])
        else:
            assert rel_err(cur[2], ref[2]) <= 1e-6


def test_fused_reverse_pair_matches_two_steps_and_oracle():
    import paper_1502_03504_amd as L
    from synth import PERIODIC as P
    from tests.gpu_util import grid_from
    rng = np.random.default_rng(7)
    shape = (19, 35, 70)
    for dtype in (np.float32, np.float64):
        u1 = rng.uniform(0, 1, shape).astype(dtype)      # u_t
        u0 = rng.uniform(0, 1, shape).astype(dtype)      # u_{t-1}
        kap = rng.uniform(0.05, 0.2, shape).astype(dtype)
        lam = rng.standard_normal(shape).astype(dtype)   # lam_{t+1}
        dt, bc = 0.1, ((P, P, P), 0.0)
        gl, gu1, gu0, gk = grid_from(lam, 1), grid_from(u1, 1), grid_from(u0, 1), grid_from(kap, 1)
        out2 = grid_from(np.zeros_like(lam), 1)
        acc2 = grid_from(np.zeros(shape, dtype=np.float64), 0)
        L.lope_apply_var_adjoint2(gl, out2, gu1, gu0, gk, dt, bc, acc2)
        # the same two steps one at a time
        mid = grid_from(np.zeros_like(lam), 1)
        out1 = grid_from(np.zeros_like(lam), 1)
        acc1 = grid_from(np.zeros(shape, dtype=np.float64), 0)
        L.lope_apply_var_adjoint(gl, mid, gu1, gk, dt, bc, acc1)
        L.lope_apply_var_adjoint(mid, out1, gu0, gk, dt, bc, acc1)
        np.testing.assert_array_equal(out2.numpy(), out1.numpy())
        assert rel_err(acc2.numpy(), acc1.numpy()) <= (1e-6 if dtype == np.float32 else 1e-14)
        # against the oracle's transposes
        l_t = oracle.diffusion_step_transpose(lam, kap, dt)
        want_l = oracle.diffusion_step_transpose(l_t, kap, dt)
        want_g = oracle.diffusion_kappa_vjp(u1, lam, dt) + oracle.diffusion_kappa_vjp(u0, l_t, dt)
        tol = 1e-5 if dtype == np.float32 else 1e-12
        assert rel_err(out2.numpy(), want_l) <= tol, rel_err(out2.numpy(), want_l)
        assert rel_err(acc2.numpy(), want_g) <= tol, rel_err(acc2.numpy(), want_g)
