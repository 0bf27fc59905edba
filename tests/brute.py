"""Brute-force dense operators for tiny grids (pins for the oracle).

Built entry by entry from the statement of the method, with plain Python
loops, independent of the oracle's vectorised slicing:

* sweep: y = A u + b g where, for every interior cell x and tap o, the read
  at x+o either lands on an interior cell (after periodic wrapping) and adds
  c_o to A[x, cell], or lies outside along a Dirichlet axis and adds c_o to
  b[x] (the halo rule of section 2.2 / 3.2 with the corner reading "Dirichlet
  wins");
* diffusion: the matrix of one variable-coefficient step.
"""
import itertools

import numpy as np

DIRICHLET = "dirichlet"


def cells(shape):
    """All interior cells as numpy-order index tuples, in C order."""
    return list(itertools.product(*[range(n) for n in shape]))


def flat(shape, idx):
    f = 0
    for n, i in zip(shape, idx):
        f = f * n + i
    return f


def sweep_operator(shape, coeffs, kinds, dtype=np.float64):
    d = len(shape)
    r = (coeffs.shape[0] - 1) // 2
    c = coeffs.astype(dtype).astype(np.float64)
    npts = int(np.prod(shape))
    A = np.zeros((npts, npts))
    b = np.zeros(npts)
    for x in cells(shape):
        row = flat(shape, x)
        for tap in itertools.product(*[range(2 * r + 1)] * d):
            coef = c[tap]
            if coef == 0.0:
                continue
            z = [x[k] + tap[k] - r for k in range(d)]
            dirichlet_out = False
            for k in range(d):
                paper_axis = d - 1 - k
                if kinds[paper_axis] == DIRICHLET and not (0 <= z[k] < shape[k]):
                    dirichlet_out = True
            if dirichlet_out:
                b[row] += coef
            else:
                wrapped = [z[k] % shape[k] for k in range(d)]
                A[row, flat(shape, wrapped)] += coef
    return A, b


def halo_value(u, z, kinds, g):
    """The value the halo rule assigns to padded index z (numpy order)."""
    d = u.ndim
    for k in range(d):
        if kinds[d - 1 - k] == DIRICHLET and not (0 <= z[k] < u.shape[k]):
            return g
    return u[tuple(z[k] % u.shape[k] for k in range(d))]


def diffusion_operator(kappa, dt):
    """Matrix of u -> u + dt * sum_a sum_s K^s_a (u_{x+s e_a} - u_x), periodic."""
    shape = kappa.shape
    d = len(shape)
    k = kappa.astype(np.float64)
    npts = int(np.prod(shape))
    A = np.eye(npts)
    for x in cells(shape):
        row = flat(shape, x)
        for ax in range(d):
            for s in (-1, 1):
                y = list(x)
                y[ax] = (y[ax] + s) % shape[ax]
                face = 0.5 * (k[x] + k[tuple(y)])
                A[row, flat(shape, y)] += dt * face
                A[row, row] -= dt * face
    return A
