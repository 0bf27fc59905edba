"""Oracle for the constant-coefficient sweep (test infrastructure only).

Arrays follow the ``synth`` conventions: a field of dimension d is a numpy
array whose LAST axis is the paper's first index x (left/right), the one
before it y (below/above), then z.  ``kinds[a]`` is the boundary kind of paper
axis a ('dirichlet' or 'periodic'); ``g`` is the one Dirichlet value of the
grid.

What is computed, and where the paper defines it:

* Halo rule (section 2.2, "Halo regions"; section 3.2, the HALO_TRANSFER call
  with BC=CYCLIC): a halo cell outside the interior along any Dirichlet axis
  holds g; otherwise it holds the interior value at the periodically wrapped
  index.  The paper shows only faces; corners follow this order-independent
  reading.
* Sweep (Fig. 1, section 2.2 "Concurrent functions", section 3.2 items 1-7):
  every interior element is rewritten from the read-only neighbourhood of the
  state at invocation time, y[x] = sum_o c_o * B(u)[x+o] (Jacobi: only the old
  state is read; the new one lives in a second buffer).
* Iteration (section 3.2, the do-while loop around the sweep and the halo
  transfer): n sweeps, alternating buffers; or, with a convergence test the
  paper leaves undefined, sweeps until the max-norm change of one sweep,
  checked every m sweeps, is at most a tolerance.
* Adjoint: the transpose of the sweep's linear part, obtained by scattering
  each tap (the transpose of the gather), and the derivative with respect to g.

Arithmetic: float64, taps summed in lexicographic offset order with x fastest,
coefficients rounded once to the grid dtype, the result rounded to the grid
dtype after every sweep.
"""
from __future__ import annotations

import numpy as np

DIRICHLET = "dirichlet"
PERIODIC = "periodic"


def _radius(coeffs: np.ndarray) -> int:
    r = (coeffs.shape[0] - 1) // 2
    if any(s != 2 * r + 1 for s in coeffs.shape):
        raise ValueError("coefficient table must be (2r+1)^d")
    return r


def _axis_map(n: int, lo: int, hi: int, kind: str):
    """For padded indices z in [lo, hi): wrapped interior index and 'outside' flag."""
    z = np.arange(lo, hi)
    outside = (z < 0) | (z >= n)
    if kind == PERIODIC:
        zi = np.mod(z, n)
        return zi, np.zeros_like(outside)
    zi = np.clip(z, 0, n - 1)
    return zi, outside


def _gather(u: np.ndarray, ranges, kinds, g: float) -> np.ndarray:
    """float64 values of the halo-extended field at the index box ``ranges``.

    ``ranges[npax] = (lo, hi)`` in interior coordinates of numpy axis npax.
    """
    d = u.ndim
    idx, masks = [], []
    for npax in range(d):
        a = d - 1 - npax
        zi, out = _axis_map(u.shape[npax], ranges[npax][0], ranges[npax][1], kinds[a])
        idx.append(zi)
        sh = [1] * d
        sh[npax] = len(zi)
        masks.append(out.reshape(sh))
    vals = u[np.ix_(*idx)].astype(np.float64)
    dirichlet_out = np.zeros(vals.shape, dtype=bool)
    for m in masks:
        dirichlet_out = dirichlet_out | m
    vals[dirichlet_out] = g
    return vals


def rule_extend(u: np.ndarray, w: int, kinds, g: float) -> np.ndarray:
    """The field extended by w cells per side with the halo rule (float64)."""
    return _gather(u, [(-w, n + w) for n in u.shape], kinds, float(g))


def halo_widths(h, ndim: int):
    """Per paper axis (x first) the halo widths (left/below, right/above).

    ``h`` is one width for both sides of every axis, or a sequence of
    (lo, hi) pairs, one per paper axis: the M:*:N halo of section 2.2 (M
    cells to the left, N to the right) given for each dimension.
    """
    if np.ndim(h) == 0:
        return [(int(h), int(h))] * ndim
    w = [(int(lo), int(hi)) for lo, hi in h]
    if len(w) != ndim or min(min(p) for p in w) < 0:
        raise ValueError("one (lo, hi) pair of non-negative widths per axis")
    return w


def halo_fill(u: np.ndarray, h, kinds, g: float) -> np.ndarray:
    """Padded array (interior plus the halo cells of every side) in u's dtype.

    This is what a halo transfer leaves in storage on one device: the interior
    unchanged and every halo cell set by the boundary rule, g rounded to the
    grid dtype.  ``h`` as in halo_widths (symmetric or per-axis lo/hi).
    """
    if u.size == 0:
        raise ValueError("an empty interior has no halo values to copy")
    gd = float(np.asarray(g, dtype=u.dtype))
    w = halo_widths(h, u.ndim)
    d = u.ndim
    ranges = [(-w[d - 1 - npax][0], u.shape[npax] + w[d - 1 - npax][1]) for npax in range(d)]
    return _gather(u, ranges, kinds, gd).astype(u.dtype)


def stencil_reach(coeffs: np.ndarray, dtype=np.float64):
    """Per paper axis (x first) how far the taps reach: (lo, hi) = the largest
    offset toward lower / higher indices over the taps whose coefficient is
    non-zero once rounded to ``dtype``.  A sweep reads exactly the halo cells
    within this reach, so the halo must be at least this wide on each side
    (section 3.5); a one-sided stencil needs a halo on one side only."""
    c = np.asarray(coeffs, dtype=np.float64).astype(dtype)
    r = _radius(c)
    d = c.ndim
    nz = np.argwhere(c != 0)
    out = []
    for a in range(d):
        npax = d - 1 - a
        if len(nz) == 0:
            out.append((0, 0))
            continue
        offs = nz[:, npax] - r
        out.append((max(0, int(-offs.min())), max(0, int(offs.max()))))
    return out


def _taps(coeffs: np.ndarray, dtype):
    """Non-zero taps (offset per numpy axis, coefficient) in lexicographic order.

    Offsets run with x (the last numpy axis) fastest; the coefficient is
    rounded once to the grid dtype and then used in float64.
    """
    r = _radius(coeffs)
    c = coeffs.astype(dtype).astype(np.float64)
    out = []
    for idx in np.ndindex(*c.shape):
        if c[idx] != 0.0:
            out.append((tuple(i - r for i in idx), float(c[idx])))
    return out


def sweep(u: np.ndarray, coeffs: np.ndarray, kinds, g: float) -> np.ndarray:
    """One Jacobi sweep: y[x] = sum_o c_o * B(u)[x+o] over the whole interior.

    An empty interior has no element to update and gives an empty result.
    """
    r = _radius(coeffs)
    if coeffs.ndim != u.ndim:
        raise ValueError("stencil and field dimension differ")
    if u.size == 0:
        return np.array(u, copy=True)
    gd = float(np.asarray(g, dtype=u.dtype))
    ext = rule_extend(u, r, kinds, gd)
    y = np.zeros(u.shape, dtype=np.float64)
    for off, c in _taps(coeffs, u.dtype):
        sl = tuple(slice(r + o, r + o + n) for o, n in zip(off, u.shape))
        y += c * ext[sl]
    return y.astype(u.dtype)


def iterate(u0: np.ndarray, coeffs: np.ndarray, kinds, g: float, n_steps: int) -> np.ndarray:
    """n_steps sweeps, each reading only the previous state (double buffering)."""
    u = np.array(u0, copy=True)
    for _ in range(int(n_steps)):
        u = sweep(u, coeffs, kinds, g)
    return u


def iterate_until(u0: np.ndarray, coeffs: np.ndarray, kinds, g: float, max_steps: int,
                  check_every: int, tol: float):
    """The do-while loop of section 3.2 with a convergence test: sweep until
    the change made by one sweep is small, or max_steps sweeps are done.

    After every sweep t+1 whose count is a multiple of check_every, the
    residual max_x |u_{t+1}[x] - u_t[x]| is taken over the interior (float64;
    the difference of two dtype values, then its magnitude, then the maximum,
    which does not depend on evaluation order).  The loop stops after the
    first checked sweep whose residual is <= tol.  Returns (u, steps, residual)
    with residual the last one computed (nan when none was).  An empty field
    stops at once with 0 steps.
    """
    u = np.array(u0, copy=True)
    res = float("nan")
    if u.size == 0:
        return u, 0, res
    m = int(check_every)
    for t in range(int(max_steps)):
        v = sweep(u, coeffs, kinds, g)
        if (t + 1) % m == 0:
            res = float(np.max(np.abs(v.astype(np.float64) - u.astype(np.float64))))
            u = v
            if res <= tol:
                return u, t + 1, res
        else:
            u = v
    return u, int(max_steps), res


def stages_step(u: np.ndarray, c1: np.ndarray, c2: np.ndarray, alpha: float, kinds, g: float) -> np.ndarray:
    """One step of two local-element functions applied in sequence, with a
    share of the starting state (two-stage schemes such as RK2/Heun; the
    paper leaves fusing small functions to the compiler, section 3.5, and
    notes that intermediate results of multi-step updates are not stored
    automatically, section 5):

        v  = S1(B(u))            the first function's result, a state of the
                                 grid's dtype whose halo follows the same rule;
        u' = alpha * u + S2(B(v))

    The second sum is taken in float64 with alpha and the coefficients rounded
    once to the grid dtype, and rounded to the dtype once.  With alpha = 0 the
    step is the composition of the two sweeps.
    """
    v = sweep(u, c1, kinds, g)
    if u.size == 0:
        return v
    r2 = _radius(c2)
    if c2.ndim != u.ndim:
        raise ValueError("stencil and field dimension differ")
    gd = float(np.asarray(g, dtype=u.dtype))
    ext = rule_extend(v, r2, kinds, gd)
    a = float(np.asarray(alpha, dtype=u.dtype))
    y = a * u.astype(np.float64)
    for off, c in _taps(c2, u.dtype):
        sl = tuple(slice(r2 + o, r2 + o + n) for o, n in zip(off, u.shape))
        y += c * ext[sl]
    return y.astype(u.dtype)


def stages_iterate(u0: np.ndarray, c1: np.ndarray, c2: np.ndarray, alpha: float, kinds, g: float,
                   n_steps: int) -> np.ndarray:
    """n_steps two-stage steps, each reading only the previous state."""
    u = np.array(u0, copy=True)
    for _ in range(int(n_steps)):
        u = stages_step(u, c1, c2, alpha, kinds, g)
    return u


def result_index(n_steps: int) -> int:
    """Which of the two ping-pong buffers holds the state after n_steps sweeps."""
    return int(n_steps) % 2


def sweep_at(u0: np.ndarray, coeffs: np.ndarray, kinds, g: float, n_steps: int,
             points) -> np.ndarray:
    """Values at selected interior points after n_steps sweeps, each computed
    on its own window.

    The value at x after n sweeps depends only on the initial state within
    n*r cells of x (taking the halo rule into account), so each sampled point
    is evaluated by iterating on that window, shrinking it by r cells per
    sweep.  Halo cells along Dirichlet axes keep the value g at every sweep;
    along periodic axes they are the wrapped cells and evolve with them.
    ``points`` is a sequence of numpy-order index tuples.
    """
    r = _radius(coeffs)
    d = u0.ndim
    gd = float(np.asarray(g, dtype=u0.dtype))
    taps = _taps(coeffs, u0.dtype)
    out = np.empty(len(points), dtype=u0.dtype)
    w = int(n_steps) * r
    for k, p in enumerate(points):
        ranges = [(p[npax] - w, p[npax] + w + 1) for npax in range(d)]
        cur = _gather(u0, ranges, kinds, gd).astype(u0.dtype).astype(np.float64)
        lo = [p[npax] - w for npax in range(d)]
        for _ in range(int(n_steps)):
            shape = tuple(s - 2 * r for s in cur.shape)
            nxt = np.zeros(shape, dtype=np.float64)
            for off, c in taps:
                sl = tuple(slice(r + o, r + o + s) for o, s in zip(off, shape))
                nxt += c * cur[sl]
            nxt = nxt.astype(u0.dtype).astype(np.float64)
            lo = [v + r for v in lo]
            # cells of the window that lie in the halo of a Dirichlet axis hold g
            for npax in range(d):
                a = d - 1 - npax
                if kinds[a] != DIRICHLET:
                    continue
                z = np.arange(lo[npax], lo[npax] + shape[npax])
                bad = (z < 0) | (z >= u0.shape[npax])
                if bad.any():
                    sl = [slice(None)] * d
                    sl[npax] = bad
                    nxt[tuple(sl)] = gd
            cur = nxt
        out[k] = cur.reshape(-1)[0]
    return out


def adjoint(ybar: np.ndarray, coeffs: np.ndarray, kinds):
    """Transpose of the sweep's linear part, and the derivative w.r.t. g.

    The sweep is y = A u + b g.  A^T ybar is obtained by scattering every tap:
    each output cell x sends c_o * ybar[x] to the cell x+o it read from; a read
    that landed in a Dirichlet halo went to b instead and is summed into
    gbar = b . ybar, and a read from a periodic halo cell goes to the interior
    cell that the rule copied it from.  Returns (xbar in ybar's dtype, gbar as a
    Python float).
    """
    r = _radius(coeffs)
    d = ybar.ndim
    if ybar.size == 0:
        return np.array(ybar, copy=True), 0.0
    yb = ybar.astype(np.float64)
    ext = np.zeros(tuple(n + 2 * r for n in ybar.shape), dtype=np.float64)
    for off, c in _taps(coeffs, ybar.dtype):
        sl = tuple(slice(r + o, r + o + n) for o, n in zip(off, ybar.shape))
        ext[sl] += c * yb
    # fold the extended array back onto the interior with the rule
    idx, masks = [], []
    for npax in range(d):
        a = d - 1 - npax
        zi, out = _axis_map(ybar.shape[npax], -r, ybar.shape[npax] + r, kinds[a])
        sh = [1] * d
        sh[npax] = len(zi)
        idx.append(zi.reshape(sh))
        masks.append(out.reshape(sh))
    dout = np.zeros(ext.shape, dtype=bool)
    for m in masks:
        dout = dout | m
    gbar = float(ext[dout].sum())
    full_idx = tuple(np.broadcast_to(i, ext.shape) for i in idx)
    keep = ~dout
    xbar = np.zeros(ybar.shape, dtype=np.float64)
    np.add.at(xbar, tuple(i[keep] for i in full_idx), ext[keep])
    return xbar.astype(ybar.dtype), gbar
