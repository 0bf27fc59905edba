"""Oracle for variable-coefficient diffusion and its gradient (test infrastructure only).

The paper's model is a local-element update over a read-only halo; this module
is one such update with a second, spatially varying input field kappa, used
for the gradient workload:

    u'_x = u_x + dt * sum_a sum_{s=+-1} K^s_a(x) * (u_{x+s e_a} - u_x),
    K^s_a(x) = (kappa_x + kappa_{x+s e_a}) / 2,

on a periodic grid with unit spacing (the flux form of u += dt*div(kappa grad u)
with arithmetic-mean face coefficients).  Reading: the paper does not give a
discretisation; this one is the usual conservative flux form.

The gradient of L = sum (u_T - target)^2 is taken by reverse accumulation
through the stored states: lambda_T = dL/du_T, then for t = T-1 .. 0
g_kappa += (du_{t+1}/dkappa)^T lambda_{t+1} and lambda_t = (du_{t+1}/du_t)^T
lambda_{t+1}.  Both transposes are formed by scattering every term of the
forward update to the cells it read (no hand-simplified closed form), so the
GPU kernels, which use a simplified per-cell formula, are checked against an
independent derivation.

Arithmetic: float64; forward states rounded to the input dtype after every
step (as the sweep); the reverse pass is float64 throughout.
"""
from __future__ import annotations

import numpy as np


def _shift(a: np.ndarray, s: int, ax: int) -> np.ndarray:
    """b[x] = a[x + s*e_ax] with periodic wrap."""
    return np.roll(a, -s, axis=ax)


def diffusion_step(u: np.ndarray, kappa: np.ndarray, dt: float) -> np.ndarray:
    """One forward step on a periodic grid; the result is rounded to u's dtype."""
    uf = u.astype(np.float64)
    kf = kappa.astype(kappa.dtype).astype(np.float64)
    acc = np.zeros_like(uf)
    for ax in range(u.ndim):
        for s in (-1, +1):
            face = 0.5 * (kf + _shift(kf, s, ax))
            acc += face * (_shift(uf, s, ax) - uf)
    return (uf + float(dt) * acc).astype(u.dtype)


def diffusion_forward(u0: np.ndarray, kappa: np.ndarray, dt: float, n_steps: int):
    """All states u_0 .. u_n (each in u0's dtype)."""
    states = [np.array(u0, copy=True)]
    for _ in range(int(n_steps)):
        states.append(diffusion_step(states[-1], kappa, dt))
    return states


def diffusion_loss(u_T: np.ndarray, target: np.ndarray) -> float:
    diff = u_T.astype(np.float64) - target.astype(np.float64)
    return float(np.sum(diff * diff))


def diffusion_step_transpose(lam: np.ndarray, kappa: np.ndarray, dt: float) -> np.ndarray:
    """(du'/du)^T lam, by scattering every term of the update (float64)."""
    lf = lam.astype(np.float64)
    kf = kappa.astype(np.float64)
    out = lf.copy()                                 # identity term u_x
    for ax in range(lam.ndim):
        for s in (-1, +1):
            face = 0.5 * (kf + _shift(kf, s, ax))
            w = float(dt) * face * lf              # weight of term (x, a, s)
            out -= w                               # it read u_x with sign -1 ...
            out += np.roll(w, s, axis=ax)          # ... and u_{x+s e_a} with sign +1
    return out


def diffusion_kappa_vjp(u: np.ndarray, lam: np.ndarray, dt: float, kappa_ndim: int = None) -> np.ndarray:
    """(du'/dkappa)^T lam at state u (float64), by scattering to both face cells."""
    uf = u.astype(np.float64)
    lf = lam.astype(np.float64)
    g = np.zeros_like(uf)
    for ax in range(u.ndim):
        for s in (-1, +1):
            t = 0.5 * float(dt) * lf * (_shift(uf, s, ax) - uf)
            g += t                                  # d face / d kappa_x
            g += np.roll(t, s, axis=ax)            # d face / d kappa_{x+s e_a}
    return g


def diffusion_gradient(u0: np.ndarray, kappa: np.ndarray, target: np.ndarray,
                       dt: float, n_steps: int):
    """(loss, dL/du0, dL/dkappa) by reverse accumulation through stored states."""
    states = diffusion_forward(u0, kappa, dt, n_steps)
    loss = diffusion_loss(states[-1], target)
    lam = 2.0 * (states[-1].astype(np.float64) - target.astype(np.float64))
    gk = np.zeros(u0.shape, dtype=np.float64)
    for t in range(int(n_steps) - 1, -1, -1):
        gk += diffusion_kappa_vjp(states[t], lam, dt)
        lam = diffusion_step_transpose(lam, kappa, dt)
    return loss, lam, gk
