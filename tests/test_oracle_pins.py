"""Pins for the CPU oracle: what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
two printed stencils and its index orientation (section 2.2, Fig. 1, section
3.3), closed-form polynomial and sine-mode results, invariants (fixed points,
conservation), library spectral routines (numpy FFT, scipy DST-I) and brute
force dense operators on tiny grids.
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests import brute


# ---------------------------------------------------------------- orientation
def test_fig1_by_local_index_notation():
    """Fig. 1 written with the paper's local indices U(i,j), i = x (left/right),
    j = y (below/above), evaluated point by point on a Dirichlet grid."""
    rng = np.random.default_rng(1)
    nx, ny, g = 5, 4, 2.0
    u = rng.integers(-9, 10, size=(ny, nx)).astype(np.float64)

    def U(i, j):  # padded access with the Dirichlet rule; u[y, x]
        if 0 <= i < nx and 0 <= j < ny:
            return u[j, i]
        return g

    want = np.zeros_like(u)
    for j in range(ny):
        for i in range(nx):
            want[j, i] = (U(i, j + 1) + U(i - 1, j) - 3 * U(i, j) + U(i + 1, j)
                          + U(i, j - 1))
    got = oracle.sweep(u, synth.fig1_laplacian().coeffs, (D, D), g)
    np.testing.assert_array_equal(got, want)


def test_fig1_is_identity_plus_numrich_reid():
    """Fig. 1 (centre -3) and the coarray Laplace of section 3.3 (centre -4)
    differ by exactly the identity."""
    rng = np.random.default_rng(2)
    u = rng.integers(-50, 50, size=(7, 9)).astype(np.float64)
    for kinds in ((D, D), (P, P), (P, D)):
        f1 = oracle.sweep(u, synth.fig1_laplacian().coeffs, kinds, 3.0)
        nr = oracle.sweep(u, synth.numrich_reid_laplace().coeffs, kinds, 3.0)
        np.testing.assert_array_equal(f1, u + nr)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_single_tap_is_a_shift(ndim):
    """A lone coefficient at offset +1 along paper axis a returns u[x + e_a]:
    'right' is +1 on the first index, 'above' +1 on the second."""
    rng = np.random.default_rng(3)
    shape = (5, 6, 7)[:ndim]
    u = rng.standard_normal(shape)
    for a in range(ndim):
        c = np.zeros((3,) * ndim)
        idx = [1] * ndim
        idx[ndim - 1 - a] = 2           # offset +1 along paper axis a
        c[tuple(idx)] = 1.0
        got = oracle.sweep(u, c, (P,) * ndim, 0.0)
        np.testing.assert_array_equal(got, np.roll(u, -1, axis=ndim - 1 - a))


# ------------------------------------------------------ polynomial exactness
def _interior_poly_check(shape, st, p, lap_p, scale, tol):
    """S p = p + scale * Lap p at cells whose footprint stays in the interior."""
    r = st.radius
    got = oracle.sweep(p, st.coeffs, (D,) * len(shape), 123.0)
    inner = tuple(slice(r, n - r) for n in shape)
    want = p + scale * lap_p
    err = np.max(np.abs(got[inner] - want[inner])) / np.max(np.abs(want[inner]))
    assert err <= tol


def test_polynomial_exact_5pt_fig1():
    ny, nx = 9, 11
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    p = x ** 3 + 3 * x * y ** 2 - y ** 3 + 2 * x * y + 7
    lap = 6 * x + 6 * x - 6 * y                        # exact Laplacian of p
    _interior_poly_check((ny, nx), synth.fig1_laplacian(), p, lap, 1.0, 1e-15)


def test_polynomial_exact_7pt_heat():
    n = 8
    z, y, x = np.mgrid[0:n, 0:n + 1, 0:n + 2].astype(np.float64)
    p = x ** 3 + 2 * x ** 2 * y - y * z ** 2 + 3 * z ** 3 + x * y * z + 5
    lap = 6 * x + 4 * y - 2 * y + 18 * z
    _interior_poly_check(p.shape, synth.heat_star(3, 0.125), p, lap, 0.125, 1e-14)


def test_polynomial_exact_25pt_degree9():
    n = 12
    z, y, x = np.mgrid[0:n, 0:n + 1, 0:n + 2].astype(np.float64)
    p = x ** 9 + 2 * y ** 8 + y * z ** 5 - 4 * x ** 3 * z ** 2
    lap = 72 * x ** 7 + 112 * y ** 6 + 20 * y * z ** 3 - 24 * x * z ** 2 - 8 * x ** 3
    _interior_poly_check(p.shape, synth.laplacian8_star(3, 0.05), p, lap, 0.05, 1e-13)


def test_25pt_not_exact_degree10():
    """Sanity: the eighth-order weights stop being exact at degree 10."""
    n = 12
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(np.float64)
    p = x ** 10
    st = synth.laplacian8_star(3, 1.0)
    got = oracle.sweep(p, st.coeffs, (D, D, D), 0.0)
    want = p + 90 * x ** 8
    inner = (slice(4, 8),) * 3
    assert np.max(np.abs(got[inner] - want[inner])) > 1.0


# --------------------------------------------------------------- fixed points
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_constant_fixed_point_dyadic(dtype):
    rng = np.random.default_rng(5)
    for shape_kind in ("box", "star"):
        st = synth.dyadic_stencil(rng, shape_kind)
        c = dtype(0.7353515625)           # dyadic constant
        u = np.full((13, 17), c, dtype=dtype)
        np.testing.assert_array_equal(oracle.iterate(u, st.coeffs, (P, P), 0.0, 5), u)
        np.testing.assert_array_equal(oracle.iterate(u, st.coeffs, (D, P), float(c), 5), u)
        np.testing.assert_array_equal(oracle.iterate(u, st.coeffs, (D, D), float(c), 5), u)


def test_zero_fixed_under_dirichlet_zero():
    rng = np.random.default_rng(6)
    st = synth.random_stencil(rng, 3, 2, "box")
    u = np.zeros((6, 7, 8))
    np.testing.assert_array_equal(oracle.iterate(u, st.coeffs, (D, D, D), 0.0, 3), u)


# --------------------------------------------------------------- conservation
@pytest.mark.parametrize("ndim,r,shape_kind", [(1, 3, "box"), (2, 2, "box"), (3, 1, "star"), (3, 4, "star")])
def test_periodic_sum_scales_by_coefficient_sum(ndim, r, shape_kind):
    rng = np.random.default_rng(7)
    shape = (9, 10, 11)[:ndim]
    st = synth.random_stencil(rng, ndim, r, shape_kind)
    u = rng.standard_normal(shape)
    y = oracle.sweep(u, st.coeffs, (P,) * ndim, 0.0)
    lhs = math.fsum(y.ravel())
    rhs = math.fsum(st.coeffs.ravel()) * math.fsum(u.ravel())
    assert abs(lhs - rhs) <= 1e-12 * np.abs(u).sum() * np.abs(st.coeffs).sum()


# -------------------------------------------------- closed-form sine decay
@pytest.mark.parametrize("kinds", [(D, D, D), (P, P, P), (D, P, D)])
def test_heat_mode_decay_closed_form(kinds):
    shape = (10, 12, 14)                      # (nz, ny, nx)
    ks = (3, 2, 1)                            # per paper axis
    rc = 0.125
    u = synth.mode_field(shape, ks, kinds)
    lam = 1.0
    for a in range(3):
        n = shape[2 - a]
        theta = (np.pi * ks[a] / (n + 1)) if kinds[a] == D else (2 * np.pi * ks[a] / n)
        lam -= 4 * rc * np.sin(theta / 2) ** 2
    steps = 25
    got = oracle.iterate(u, synth.heat_star(3, rc).coeffs, kinds, 0.0, steps)
    np.testing.assert_allclose(got, lam ** steps * u, rtol=0, atol=1e-13)


def test_heat_1d_dirichlet_matches_stated_factor():
    """1D heat, Dirichlet 0: the per-step factor 1 - 4 r sin^2(pi k / 2N) with N
    the number of intervals between the two boundary nodes (interior + 1)."""
    n_int, k, rc = 31, 5, 0.25
    x = np.arange(n_int)
    u = np.sin(np.pi * k * (x + 1) / (n_int + 1))
    N = n_int + 1
    lam = 1 - 4 * rc * np.sin(np.pi * k / (2 * N)) ** 2
    got = oracle.iterate(u, synth.heat_star(1, rc).coeffs, (D,), 0.0, 40)
    np.testing.assert_allclose(got, lam ** 40 * u, rtol=0, atol=1e-14)


# ------------------------------------------------------- spectral (library)
@pytest.mark.parametrize("ndim,r,shape_kind", [(2, 2, "box"), (3, 2, "star"), (1, 4, "box")])
def test_periodic_matches_fft(ndim, r, shape_kind):
    rng = np.random.default_rng(8)
    shape = (6, 10, 12)[:ndim] if ndim == 3 else ((14, 18) if ndim == 2 else (40,))
    st = synth.contractive(synth.random_stencil(rng, ndim, r, shape_kind))
    u0 = rng.standard_normal(shape)
    steps = 6
    # symbol lambda(k) = sum_o c_o exp(2 pi i k.o / N)
    freqs = np.meshgrid(*[np.fft.fftfreq(n) * n for n in shape], indexing="ij")
    lam = np.zeros(shape, dtype=complex)
    for idx in np.ndindex(*st.coeffs.shape):
        c = st.coeffs[idx]
        if c == 0:
            continue
        ph = 0.0
        for npax in range(ndim):
            ph = ph + 2j * np.pi * freqs[npax] * (idx[npax] - r) / shape[npax]
        lam += c * np.exp(ph)
    want = np.fft.ifftn(lam ** steps * np.fft.fftn(u0)).real
    got = oracle.iterate(u0, st.coeffs, (P,) * ndim, 0.0, steps)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("ndim", [2, 3])
def test_dirichlet_zero_matches_dst(ndim):
    rng = np.random.default_rng(9)
    shape = (9, 11, 13)[:ndim] if ndim == 3 else (15, 17)
    cen = 0.3
    side = rng.uniform(0.02, 0.12, size=ndim)      # symmetric per axis
    c = np.zeros((3,) * ndim)
    c[(1,) * ndim] = cen
    for a in range(ndim):
        for s in (0, 2):
            idx = [1] * ndim
            idx[ndim - 1 - a] = s
            c[tuple(idx)] = side[a]
    u0 = rng.standard_normal(shape)
    lam = np.full(shape, cen)
    for npax in range(ndim):
        a = ndim - 1 - npax
        k = np.arange(1, shape[npax] + 1)
        sh = [1] * ndim
        sh[npax] = shape[npax]
        lam = lam + 2 * side[a] * np.cos(np.pi * k / (shape[npax] + 1)).reshape(sh)
    steps = 7
    want = scipy.fft.idstn(lam ** steps * scipy.fft.dstn(u0, type=1), type=1)
    got = oracle.iterate(u0, c, (D,) * ndim, 0.0, steps)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())


# --------------------------------------------------------------- brute force
BRUTE_CASES = [
    ((11,), 2, "box", (P,)),
    ((10,), 3, "box", (D,)),
    ((5, 6), 1, "box", (D, P)),
    ((6, 5), 2, "box", (P, D)),
    ((4, 5), 2, "box", (P, P)),
    ((3, 7), 1, "box", (D, D)),
    ((3, 4, 5), 1, "box", (D, P, P)),
    ((4, 3, 5), 1, "box", (P, D, P)),
    ((4, 4, 3), 2, "star", (P, P, D)),
    ((9, 9, 9), 4, "star", (D, D, D)),
    ((3, 3, 3), 2, "star", (P, P, P)),        # halo wider than the interior
]


@pytest.mark.parametrize("shape,r,shape_kind,kinds", BRUTE_CASES)
def test_sweep_iterate_adjoint_brute_force(shape, r, shape_kind, kinds):
    rng = np.random.default_rng(10 + len(shape) + r)
    nd = len(shape)
    st = synth.contractive(synth.random_stencil(rng, nd, r, shape_kind))
    g = 0.625
    A, b = brute.sweep_operator(shape, st.coeffs, kinds)
    u = rng.standard_normal(shape)
    np.testing.assert_allclose(oracle.sweep(u, st.coeffs, kinds, g).ravel(),
                               A @ u.ravel() + b * g, rtol=0, atol=1e-13)
    v = u.ravel()
    for _ in range(4):
        v = A @ v + b * g
    np.testing.assert_allclose(oracle.iterate(u, st.coeffs, kinds, g, 4).ravel(), v,
                               rtol=0, atol=1e-12)
    ybar = rng.standard_normal(shape)
    xbar, gbar = oracle.adjoint(ybar, st.coeffs, kinds)
    np.testing.assert_allclose(xbar.ravel(), A.T @ ybar.ravel(), rtol=0, atol=1e-13)
    assert abs(gbar - b @ ybar.ravel()) <= 1e-12


@pytest.mark.parametrize("shape,r,shape_kind,kinds", BRUTE_CASES[:8])
def test_float32_state_rounding(shape, r, shape_kind, kinds):
    """float32 grids: float64 sum of the float32-rounded taps, rounded once."""
    rng = np.random.default_rng(20)
    nd = len(shape)
    st = synth.contractive(synth.random_stencil(rng, nd, r, shape_kind))
    u = rng.standard_normal(shape).astype(np.float32)
    A, b = brute.sweep_operator(shape, st.coeffs, kinds, dtype=np.float32)
    g32 = float(np.float32(0.3))
    want = (A @ u.astype(np.float64).ravel() + b * g32).astype(np.float32)
    got = oracle.sweep(u, st.coeffs, kinds, 0.3)
    assert got.dtype == np.float32
    np.testing.assert_array_max_ulp(got.ravel(), want, maxulp=1)


@pytest.mark.parametrize("kinds", [(D, P), (P, D), (P, P), (D, D)])
def test_halo_fill_brute_force(kinds):
    rng = np.random.default_rng(11)
    u = rng.standard_normal((4, 5))
    h, g = 3, -1.5
    got = oracle.halo_fill(u, h, kinds, g)
    for zy in range(-h, 4 + h):
        for zx in range(-h, 5 + h):
            assert got[zy + h, zx + h] == brute.halo_value(u, (zy, zx), kinds, g)


@pytest.mark.parametrize("kinds", [(D, D, D), (P, P, P), (P, D, P), (D, P, D)])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_sweep_at_equals_full_iteration(kinds, dtype):
    rng = np.random.default_rng(12)
    shape = (7, 9, 8)
    st = synth.contractive(synth.random_stencil(rng, 3, 2, "star"))
    u = rng.standard_normal(shape).astype(dtype)
    full = oracle.iterate(u, st.coeffs, kinds, 0.4, 3)
    pts = [(0, 0, 0), (6, 8, 7), (3, 4, 4), (0, 8, 3), (6, 0, 0), (1, 2, 7)]
    got = oracle.sweep_at(u, st.coeffs, kinds, 0.4, 3, pts)
    np.testing.assert_array_equal(got, np.array([full[p] for p in pts]))


def test_adjoint_dot_product():
    rng = np.random.default_rng(13)
    for kinds in ((P, P, P), (D, D, D), (D, P, D)):
        st = synth.random_stencil(rng, 3, 2, "box")
        u = rng.standard_normal((6, 7, 8))
        v = rng.standard_normal((6, 7, 8))
        su = oracle.sweep(u, st.coeffs, kinds, 0.0)
        stv, _ = oracle.adjoint(v, st.coeffs, kinds)
        lhs, rhs = float(np.vdot(su, v)), float(np.vdot(u, stv))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_symmetric_stencil_is_self_adjoint():
    u = np.random.default_rng(14).standard_normal((9, 10, 11))
    st = synth.laplacian8_star(3, 0.05)
    for kinds in ((P, P, P), (D, D, D)):
        xb, _ = oracle.adjoint(u, st.coeffs, kinds)
        np.testing.assert_allclose(xb, oracle.sweep(u, st.coeffs, kinds, 0.0), rtol=0, atol=1e-14)


def test_result_index():
    assert [oracle.result_index(n) for n in (0, 1, 2, 7, 100)] == [0, 1, 0, 1, 0]


def test_empty_interior():
    st = synth.heat_star(3, 0.1)
    for shape in [(0, 4, 5), (3, 0, 2), (2, 3, 0)]:
        u = np.zeros(shape)
        assert oracle.sweep(u, st.coeffs, (P, D, P), 1.0).shape == shape
        assert oracle.iterate(u, st.coeffs, (D, D, D), 1.0, 3).shape == shape
        xb, gb = oracle.adjoint(u, st.coeffs, (D, D, D))
        assert xb.shape == shape and gb == 0.0
    with pytest.raises(ValueError):
        oracle.halo_fill(np.zeros((0, 3)), 1, (D, D), 0.0)


def test_extent_one_axes_brute_force():
    """Extent-1 axes: periodic wrap maps every neighbour onto the one cell."""
    rng = np.random.default_rng(15)
    for shape, kinds in [((1, 1, 1), (P, P, P)), ((1, 7, 1), (P, D, P)), ((3, 1, 4), (D, P, D)),
                         ((1, 1, 1), (D, D, D))]:
        st = synth.random_stencil(rng, 3, 1, "box")
        A, b = brute.sweep_operator(shape, st.coeffs, kinds)
        u = rng.standard_normal(shape)
        np.testing.assert_allclose(oracle.sweep(u, st.coeffs, kinds, 0.3).ravel(), A @ u.ravel() + 0.3 * b,
                                   rtol=0, atol=1e-14)
