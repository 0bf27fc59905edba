"""Differentiable variable-coefficient diffusion with checkpointed recomputation.

``diffusion(u0, kappa, dt, n_steps, checkpoint_every)`` advances
u <- u + dt * div(kappa grad u) (periodic 3D, arithmetic-mean faces) n_steps
times with the library's forward kernel and returns u_T.  Its backward pass
returns dL/du0 and dL/dkappa:

* the forward pass keeps only the states at t = 0, k, 2k, ... (k =
  checkpoint_every), so memory grows with n_steps / k, not n_steps;
* the backward pass walks the segments in reverse; for each it recomputes the
  segment's states from its checkpoint with the forward kernel, then runs the
  reverse kernels from the segment's last step down to its first, which turn
  lambda_{t+1} = dL/du_{t+1} into lambda_t and add each step's kappa
  derivative into an accumulator.  Steps (2m+1, 2m) that lie in one segment
  run as one fused two-step pass (lope_apply_var_adjoint2, which computes
  every lambda exactly as the one-step kernel does), the rest one step at a
  time;
* every FOLD_EVERY steps (at t divisible by it) the float32 accumulator is
  folded into a float64 total (lope_accumulate), so the kappa gradient is
  reduced in float64 over the time loop.  For float64 states the reverse
  kernels add each step's terms straight into the float64 total.

Recomputation is deterministic (same kernels, same inputs) and the folds sit
at fixed time indices.  So dL/du0 is bit-for-bit independent of the
checkpoint interval; dL/dkappa is too for every even interval (all pairs
fused), while an odd interval splits some pairs and changes only the rounding
of the kappa accumulator.  Everything runs on the current stream; nothing
synchronises with the host.
"""
from __future__ import annotations

import torch

from . import Grid, lope_accumulate, lope_apply_var, lope_apply_var_adjoint, lope_apply_var_adjoint2

_PERIODIC = (("periodic",) * 3, 0.0)
FOLD_EVERY = 20


def _grid_like(t: torch.Tensor, h: int = 1, dtype=None) -> Grid:
    return Grid.allocate(tuple(t.shape), h, dtype or t.dtype, t.device)


class DiffusionFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0: torch.Tensor, kappa: torch.Tensor, dt: float, n_steps: int, checkpoint_every: int):
        if u0.dim() != 3 or kappa.shape != u0.shape or kappa.dtype != u0.dtype:
            raise ValueError("u0 and kappa: 3D tensors of equal shape and dtype")
        k = max(1, int(checkpoint_every))
        n = int(n_steps)
        kap = _grid_like(kappa)
        kap.interior().copy_(kappa.detach())
        a = _grid_like(u0)
        a.interior().copy_(u0.detach())
        b = _grid_like(u0)
        checkpoints = []
        for t in range(n):
            if t % k == 0:
                cp = _grid_like(u0)
                cp.interior().copy_(a.interior())
                checkpoints.append(cp)
            lope_apply_var(a, b, kap, dt, _PERIODIC)
            a, b = b, a
        ctx.save_for_backward()
        ctx.lope = (kap, checkpoints, float(dt), n, k)
        return a.interior().clone()

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        kap, checkpoints, dt, n, k = ctx.lope
        shape = tuple(grad_out.shape)
        dev = grad_out.device
        lam = Grid.allocate(shape, 1, grad_out.dtype, dev)
        lam.interior().copy_(grad_out)
        lam2 = Grid.allocate(shape, 1, grad_out.dtype, dev)
        g64 = Grid.allocate(shape, 0, torch.float64, dev)
        # float32 states: per-step terms in a float32 partial, folded into g64;
        # float64 states: straight into g64
        fold = grad_out.dtype != torch.float64
        gacc = Grid.allocate(shape, 0, torch.float32, dev) if fold else g64
        seg_states = [Grid.allocate(shape, 1, grad_out.dtype, dev) for _ in range(min(k, n))]
        for s in range(len(checkpoints) - 1, -1, -1):
            t0 = s * k
            length = min(k, n - t0)
            # recompute u_{t0} .. u_{t0+length-1}
            seg_states[0].interior().copy_(checkpoints[s].interior())
            for i in range(1, length):
                lope_apply_var(seg_states[i - 1], seg_states[i], kap, dt, _PERIODIC)
            i = length - 1
            while i >= 0:
                t = t0 + i
                if t % 2 == 1 and i >= 1:
                    # steps t and t-1 fused (pairs sit at absolute indices (2m+1, 2m))
                    lope_apply_var_adjoint2(lam, lam2, seg_states[i], seg_states[i - 1], kap, dt, _PERIODIC, gacc)
                    low = t - 1
                    i -= 2
                else:
                    lope_apply_var_adjoint(lam, lam2, seg_states[i], kap, dt, _PERIODIC, gacc)
                    low = t
                    i -= 1
                lam, lam2 = lam2, lam
                if fold and low % FOLD_EVERY == 0:
                    lope_accumulate(gacc, g64)
        grad_u0 = lam.interior().clone()
        grad_kappa = g64.interior().to(grad_out.dtype)
        return grad_u0, grad_kappa, None, None, None


def diffusion(u0: torch.Tensor, kappa: torch.Tensor, dt: float, n_steps: int,
              checkpoint_every: int = 20) -> torch.Tensor:
    """u_T after n_steps diffusion steps; differentiable in u0 and kappa."""
    return DiffusionFunction.apply(u0, kappa, dt, n_steps, checkpoint_every)


def diffusion_gradient(u0, kappa, target, dt, n_steps, checkpoint_every=20):
    """(loss, dL/du0, dL/dkappa) for L = sum((u_T - target)^2), the loss summed
    in float64 by torch from the library's u_T."""
    u = u0.detach().clone().requires_grad_(True)
    kp = kappa.detach().clone().requires_grad_(True)
    uT = diffusion(u, kp, dt, n_steps, checkpoint_every)
    diff = uT.double() - target.double()
    loss = (diff * diff).sum()
    loss.backward()
    return loss.detach(), u.grad, kp.grad
