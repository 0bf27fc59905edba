"""Seeded synthetic inputs for the LOPe stencil sweep.

This module produces input data only: initial fields, stencil coefficient
tables, boundary descriptions and the batch mix.  It evaluates no part of the
method (no sweep, no halo rule, no adjoint); the CPU oracle and the GPU path
both take their inputs from here and from nowhere else they share.

Conventions (shared by every consumer):

* A d-dimensional field is a numpy array of shape ``(n_{d-1}, ..., n_1, n_0)``
  in C order, so the paper's first index (x, the fastest in memory, the
  "left/right" axis of the local index notation of section 2.2) is the LAST
  numpy axis.
* A stencil is a table of ``(2r+1)**d`` coefficients, stored as a float64
  array of shape ``(2r+1,)*d`` in the same axis order: ``coeffs[..., o1+r,
  o0+r]`` multiplies the neighbour at offset ``(o0, o1, ...)``.  Flattened in
  C order the entry for offset ``o`` sits at ``sum_a (o_a+r)*(2r+1)**a``.
* A boundary is a per-axis kind ('dirichlet' or 'periodic', indexed by paper
  axis, x first) plus one Dirichlet value g per grid.

Random draws use ``numpy.random.default_rng([config_id, seed])``; the field is
drawn first (C order, float64), then modes / coefficients, then cast to the
grid dtype.
"""
from __future__ import annotations

from collections import namedtuple

import numpy as np

DIRICHLET = "dirichlet"
PERIODIC = "periodic"

Boundary = namedtuple("Boundary", "kinds value")
Stencil = namedtuple("Stencil", "ndim radius coeffs")
Case = namedtuple("Case", "name field stencil bc steps h dtype")

# Config ids used to seed default_rng([config_id, seed]).
CFG_HEAT2D = 1
CFG_HEAT3D = 2
CFG_BOX9 = 3
CFG_STAR25 = 4
CFG_DIFFUSION = 5
CFG_BATCH = 6
CFG_TEST = 100


def rng_for(config_id: int, seed: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(config_id), int(seed)])


# --------------------------------------------------------------------------
# Stencil tables (inputs: the user hands these coefficients to the sweep).
# --------------------------------------------------------------------------
def _empty(ndim: int, r: int) -> np.ndarray:
    return np.zeros((2 * r + 1,) * ndim, dtype=np.float64)


def _set(c: np.ndarray, offset, value: float) -> None:
    """Set the coefficient of the neighbour at paper offset (o0, o1, ...)."""
    r = (c.shape[0] - 1) // 2
    c[tuple(o + r for o in reversed(offset))] = value


def _axis_offset(ndim: int, axis: int, k: int):
    o = [0] * ndim
    o[axis] = k
    return tuple(o)


def heat_star(ndim: int, r_coef: float) -> Stencil:
    """Explicit heat-equation stencil: centre 1-2*d*r, axis neighbours r."""
    c = _empty(ndim, 1)
    _set(c, (0,) * ndim, 1.0 - 2.0 * ndim * r_coef)
    for a in range(ndim):
        _set(c, _axis_offset(ndim, a, -1), r_coef)
        _set(c, _axis_offset(ndim, a, +1), r_coef)
    return Stencil(ndim, 1, c)


def fig1_laplacian() -> Stencil:
    """The 2D local-element function of Fig. 1: centre -3, four neighbours +1."""
    c = _empty(2, 1)
    _set(c, (0, 0), -3.0)
    for o in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        _set(c, o, 1.0)
    return Stencil(2, 1, c)


def numrich_reid_laplace() -> Stencil:
    """The coarray comparison kernel of section 3.3: centre -4, four neighbours +1."""
    c = _empty(2, 1)
    _set(c, (0, 0), -4.0)
    for o in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        _set(c, o, 1.0)
    return Stencil(2, 1, c)


# Eighth-order central second-difference weights (offsets 0..4).
LAPLACIAN8_WEIGHTS = (-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)


def laplacian8_star(ndim: int = 3, nu: float = 0.05) -> Stencil:
    """u + nu * L8 u with L8 the radius-4 eighth-order Laplacian (a star)."""
    w = LAPLACIAN8_WEIGHTS
    c = _empty(ndim, 4)
    _set(c, (0,) * ndim, 1.0 + nu * ndim * w[0])
    for a in range(ndim):
        for k in range(1, 5):
            _set(c, _axis_offset(ndim, a, -k), nu * w[k])
            _set(c, _axis_offset(ndim, a, +k), nu * w[k])
    return Stencil(ndim, 4, c)


def dyadic_stencil(rng: np.random.Generator, shape: str) -> Stencil:
    """2D radius-1 stencil with positive dyadic weights that sum to exactly 1.

    Off-centre weights are integers in [1, 2**10); the centre takes
    2**12 minus their sum; every weight is divided by 2**12, so each is exact
    in float32 and float64 and the sum is exactly one.
    """
    if shape == "box":
        offs = [(ox, oy) for oy in (-1, 0, 1) for ox in (-1, 0, 1) if (ox, oy) != (0, 0)]
    elif shape == "star":
        offs = [(0, -1), (-1, 0), (1, 0), (0, 1)]
    else:
        raise ValueError(shape)
    w = rng.integers(1, 2 ** 10, size=len(offs))
    c = _empty(2, 1)
    for o, wi in zip(offs, w):
        _set(c, o, float(wi) / 4096.0)
    _set(c, (0, 0), float(4096 - int(w.sum())) / 4096.0)
    return Stencil(2, 1, c)


def random_stencil(rng: np.random.Generator, ndim: int, r: int, shape: str = "box",
                   scale: float = 1.0) -> Stencil:
    """Arbitrary (non-symmetric) coefficients for parity tests."""
    c = _empty(ndim, r)
    vals = rng.uniform(-1.0, 1.0, size=c.shape) * scale
    if shape == "box":
        c[...] = vals
    elif shape == "star":
        for a in range(ndim):
            for k in range(-r, r + 1):
                o = _axis_offset(ndim, a, k)
                idx = tuple(oo + r for oo in reversed(o))
                c[idx] = vals[idx]
    else:
        raise ValueError(shape)
    return Stencil(ndim, r, c)


def contractive(st: Stencil) -> Stencil:
    """Scale a stencil so the sum of |coefficients| is 0.95 (iterates stay bounded)."""
    s = float(np.abs(st.coeffs).sum())
    return Stencil(st.ndim, st.radius, st.coeffs * (0.95 / s))


# --------------------------------------------------------------------------
# Fields.
# --------------------------------------------------------------------------
def uniform_field(rng: np.random.Generator, shape, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return rng.uniform(lo, hi, size=tuple(shape))


def sine_modes(rng: np.random.Generator, shape, n_modes: int = 4) -> np.ndarray:
    """U[0,1) plus n_modes periodic plane waves a*sin(2*pi*k.x/N + phi).

    a ~ U[0.1,0.5), each k component a uniform integer in [1,16],
    phi ~ U[0,2*pi).  x is the cell index; N the interior extent per axis.
    """
    shape = tuple(shape)
    d = len(shape)
    u = rng.uniform(0.0, 1.0, size=shape)
    amps = rng.uniform(0.1, 0.5, size=n_modes)
    ks = rng.integers(1, 17, size=(n_modes, d))
    phis = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    grids = np.ogrid[tuple(slice(0, n) for n in shape)]
    for m in range(n_modes):
        phase = phis[m]
        for npax in range(d):
            a = d - 1 - npax
            phase = phase + 2.0 * np.pi * ks[m, a] * grids[npax] / shape[npax]
        u += amps[m] * np.sin(phase)
    return u


def gaussian_bump(rng: np.random.Generator, shape, sigma: float = 20.0,
                  noise: float = 1e-3) -> np.ndarray:
    """exp(-|x-c|^2/(2 sigma^2)) + U[-noise, noise); c ~ U[N/4, 3N/4) per axis."""
    shape = tuple(shape)
    d = len(shape)
    u = rng.uniform(-noise, noise, size=shape)
    centre = [rng.uniform(n / 4.0, 3.0 * n / 4.0) for n in shape]
    grids = np.ogrid[tuple(slice(0, n) for n in shape)]
    r2 = 0.0
    for npax in range(d):
        r2 = r2 + (grids[npax] - centre[npax]) ** 2
    u += np.exp(-r2 / (2.0 * sigma * sigma))
    return u


def mode_field(shape, ks, kinds) -> np.ndarray:
    """One separable sine mode fitted to the boundary kinds (closed-form decay tests).

    Dirichlet axis: sin(pi*k*(x+1)/(N+1)); periodic axis: sin(2*pi*k*x/N + 0.3).
    ks and kinds are indexed by paper axis (x first).
    """
    shape = tuple(shape)
    d = len(shape)
    u = np.ones(shape)
    for npax in range(d):
        a = d - 1 - npax
        n = shape[npax]
        x = np.arange(n, dtype=np.float64)
        if kinds[a] == DIRICHLET:
            f = np.sin(np.pi * ks[a] * (x + 1.0) / (n + 1.0))
        else:
            f = np.sin(2.0 * np.pi * ks[a] * x / n + 0.3)
        sh = [1] * d
        sh[npax] = n
        u = u * f.reshape(sh)
    return u


# --------------------------------------------------------------------------
# The five workloads.
# --------------------------------------------------------------------------
def case_heat2d(n: int = 256, steps: int = 100, seed: int = 0) -> Case:
    """2D 5-point heat (r=1/4), float64, Dirichlet 0, h=1, U[0,1)."""
    rng = rng_for(CFG_HEAT2D, seed)
    u = uniform_field(rng, (n, n))
    return Case("heat2d_5pt_f64", u, heat_star(2, 0.25),
                Boundary((DIRICHLET, DIRICHLET), 0.0), steps, 1, np.float64)


def case_heat3d(n: int = 512, dtype=np.float32, steps: int = 1000, seed: int = 0) -> Case:
    """3D 7-point heat (r=1/8), periodic, h=1, U[0,1) + 4 sine modes."""
    rng = rng_for(CFG_HEAT3D, seed)
    u = sine_modes(rng, (n, n, n))
    name = "heat3d_7pt_%s" % np.dtype(dtype).name
    return Case(name, u.astype(dtype), heat_star(3, 0.125),
                Boundary((PERIODIC,) * 3, 0.0), steps, 1, dtype)


def case_box9(n: int = 8192, steps: int = 1000, seed: int = 0) -> Case:
    """2D 9-point box, dyadic seeded weights summing to 1, float32, periodic, h=1."""
    rng = rng_for(CFG_BOX9, seed)
    u = sine_modes(rng, (n, n))
    st = dyadic_stencil(rng, "box")
    return Case("box9_2d_f32", u.astype(np.float32), st,
                Boundary((PERIODIC, PERIODIC), 0.0), steps, 1, np.float32)


def case_star25(n: int = 512, steps: int = 500, nu: float = 0.05, seed: int = 0) -> Case:
    """3D 25-point star (radius 4, u + nu*L8 u), float32, Dirichlet 0, h=4."""
    rng = rng_for(CFG_STAR25, seed)
    u = gaussian_bump(rng, (n, n, n))
    return Case("star25_3d_f32", u.astype(np.float32), laplacian8_star(3, nu),
                Boundary((DIRICHLET,) * 3, 0.0), steps, 4, np.float32)


DiffusionCase = namedtuple("DiffusionCase", "u0 kappa target dt steps checkpoint_every dtype")


def case_diffusion(n: int = 256, steps: int = 200, dt: float = 0.1, k: int = 20,
                   dtype=np.float32, seed: int = 0) -> DiffusionCase:
    """Variable-kappa diffusion: u0, target ~ U[0,1), kappa ~ U[0.05,0.2), periodic."""
    rng = rng_for(CFG_DIFFUSION, seed)
    shape = (n, n, n)
    u0 = uniform_field(rng, shape)
    kappa = uniform_field(rng, shape, 0.05, 0.2)
    target = uniform_field(rng, shape)
    return DiffusionCase(u0.astype(dtype), kappa.astype(dtype), target.astype(dtype),
                         dt, steps, k, dtype)


BatchGrid = namedtuple("BatchGrid", "field stencil bc")


def batch_sizes(count: int = 512, lo: int = 64, hi: int = 1024, seed: int = 0):
    """Side lengths (nx, ny), independent integers in [lo, hi] with ny != nx."""
    rng = rng_for(CFG_BATCH, seed)
    sizes = []
    for _ in range(count):
        nx = int(rng.integers(lo, hi + 1))
        ny = int(rng.integers(lo, hi + 1))
        while ny == nx:
            ny = int(rng.integers(lo, hi + 1))
        sizes.append((nx, ny))
    return sizes, rng


def case_batch(count: int = 512, lo: int = 64, hi: int = 1024, steps: int = 50,
               seed: int = 0, dtype=np.float32):
    """The batched mix: uneven 2D grids, half 5-point and half 9-point stencils.

    Draw order: all sizes, the stencil-kind permutation, per-axis boundary kinds,
    the Dirichlet values, the coefficients, then one U[0,1) field per grid.
    """
    sizes, rng = batch_sizes(count, lo, hi, seed)
    kind = np.zeros(count, dtype=np.int64)
    kind[rng.permutation(count)[: count // 2]] = 1          # 1 = 9-point box
    bck = rng.integers(0, 2, size=(count, 2))               # 1 = periodic
    gs = rng.uniform(0.0, 1.0, size=count)
    stencils = [dyadic_stencil(rng, "box" if kind[i] else "star") for i in range(count)]
    grids = []
    for i, (nx, ny) in enumerate(sizes):
        u = uniform_field(rng, (ny, nx)).astype(dtype)
        kinds = tuple(PERIODIC if bck[i, a] else DIRICHLET for a in range(2))
        grids.append(BatchGrid(u, stencils[i], Boundary(kinds, float(gs[i]))))
    return grids, steps
