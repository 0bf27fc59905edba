"""Variable-coefficient diffusion kernels (one wavefront per brick) on grids
that do not fill whole bricks: x extents around the 64-column strip, y
extents around the row count of a brick, very short z extents, and the
canaries that show the stored halo is never read and the destination halo
never written.  Forward step and one-step reverse against the oracle at the
stated tolerances."""
import numpy as np
import pytest

import oracle
import paper_1502_03504_amd as L
import synth
from synth import PERIODIC as P
from tests.gpu_util import empty_grid, grid_from, halo_mask, rel_err, tol

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (2, 3, 5), (3, 7, 63), (17, 8, 64), (5, 9, 65), (9, 13, 130), (4, 5, 200), (33, 17, 3)]


def _fields(shape, dtype, seed):
    rng = np.random.default_rng([synth.CFG_TEST, 900 + seed])
    u = rng.uniform(0, 1, shape).astype(dtype)
    k = rng.uniform(0.05, 0.2, shape).astype(dtype)
    lam = rng.standard_normal(shape).astype(dtype)
    return u, k, lam


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", SHAPES)
def test_forward_edges_and_canaries(shape, dtype):
    u, k, _ = _fields(shape, dtype, SHAPES.index(shape))
    dt = 0.1
    ug, kg = grid_from(u, 1, fill=np.nan), grid_from(k, 1, fill=np.nan)
    out = empty_grid(shape, 1, dtype, fill=np.nan)
    L.lope_apply_var(ug, out, kg, dt, (P, P, P))
    full = out.padded().cpu().numpy()
    assert np.all(np.isnan(full[halo_mask(out)])), "a halo cell of the destination was written"
    got = out.numpy()
    assert np.all(np.isfinite(got)), "the stored (NaN) halo was read"
    assert rel_err(got, oracle.diffusion_step(u, k, dt)) <= tol(dtype)


@pytest.mark.parametrize("gdt", [np.float64, np.float32])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", SHAPES)
def test_reverse_edges_and_canaries(shape, dtype, gdt):
    u, k, lam = _fields(shape, dtype, SHAPES.index(shape))
    dt = 0.1
    ug, kg, lg = (grid_from(a, 1, fill=np.nan) for a in (u, k, lam))
    out = empty_grid(shape, 1, dtype, fill=np.nan)
    gk = grid_from(np.full(shape, 0.5, dtype=gdt), 1, fill=np.nan)
    L.lope_apply_var_adjoint(lg, out, ug, kg, dt, (P, P, P), gk)
    for g in (out, gk):
        assert np.all(np.isnan(g.padded().cpu().numpy()[halo_mask(g)])), "a halo cell was written"
    got_l, got_g = out.numpy(), gk.numpy() - 0.5
    assert np.all(np.isfinite(got_l)) and np.all(np.isfinite(got_g)), "the stored (NaN) halo was read"
    assert rel_err(got_l, oracle.diffusion_step_transpose(lam, k, dt)) <= tol(dtype)
    want_g = oracle.diffusion_kappa_vjp(u, lam, dt)
    # the accumulator adds each step's terms in its own precision
    gtol = tol(gdt if gdt == np.float32 else dtype)
    assert rel_err(got_g, want_g) <= gtol, rel_err(got_g, want_g)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_forward_many_chunks_matches_oracle(dtype):
    """A tall column: the march is cut into many z-chunks (each re-reads the
    plane before and after it)."""
    shape = (300, 6, 70)
    u, k, _ = _fields(shape, dtype, 50)
    ug, kg = grid_from(u, 1), grid_from(k, 1)
    out = empty_grid(shape, 1, dtype)
    L.lope_apply_var(ug, out, kg, 0.1, (P, P, P))
    assert rel_err(out.numpy(), oracle.diffusion_step(u, k, 0.1)) <= tol(dtype)


@pytest.mark.parametrize("gdt", [np.float64, np.float32])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", SHAPES + [(70, 6, 130)])
def test_reverse_pair_edges_and_canaries(shape, dtype, gdt):
    """Two reverse steps in one pass: lam bitwise equal to two one-step
    passes, both against the oracle's transposes, halos neither read nor
    written."""
    u1, k, lam = _fields(shape, dtype, SHAPES.index(shape) if shape in SHAPES else 40)
    u0 = np.random.default_rng([synth.CFG_TEST, 950]).uniform(0, 1, shape).astype(dtype)
    dt = 0.1
    lg, g1, g0, kg = (grid_from(a, 1, fill=np.nan) for a in (lam, u1, u0, k))
    out = empty_grid(shape, 1, dtype, fill=np.nan)
    gk = grid_from(np.full(shape, 0.5, dtype=gdt), 1, fill=np.nan)
    L.lope_apply_var_adjoint2(lg, out, g1, g0, kg, dt, (P, P, P), gk)
    for g in (out, gk):
        assert np.all(np.isnan(g.padded().cpu().numpy()[halo_mask(g)])), "a halo cell was written"
    got_l, got_g = out.numpy(), gk.numpy() - 0.5
    assert np.all(np.isfinite(got_l)) and np.all(np.isfinite(got_g)), "the stored (NaN) halo was read"
    mid = empty_grid(shape, 1, dtype, fill=np.nan)
    two = empty_grid(shape, 1, dtype, fill=np.nan)
    acc = grid_from(np.zeros(shape, dtype=gdt), 1)
    L.lope_apply_var_adjoint(lg, mid, g1, kg, dt, (P, P, P), acc)
    L.lope_apply_var_adjoint(mid, two, g0, kg, dt, (P, P, P), acc)
    np.testing.assert_array_equal(got_l, two.numpy())
    l_t = oracle.diffusion_step_transpose(lam, k, dt)
    assert rel_err(got_l, oracle.diffusion_step_transpose(l_t, k, dt)) <= tol(dtype)
    want_g = oracle.diffusion_kappa_vjp(u1, lam, dt) + oracle.diffusion_kappa_vjp(u0, l_t, dt)
    gtol = tol(gdt if gdt == np.float32 else dtype)
    assert rel_err(got_g, want_g) <= gtol, rel_err(got_g, want_g)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_reverse_pair_mixed_layouts(dtype):
    """Inputs laid out differently (kappa with a wider halo) take the LDS pair
    kernel (test_gpu_log checks the choice); its results are the wave pair's
    value for value."""
    shape = (21, 19, 70)
    u1, k, lam = _fields(shape, dtype, 60)
    u0 = np.random.default_rng([synth.CFG_TEST, 951]).uniform(0, 1, shape).astype(dtype)
    dt = 0.1
    outs = []
    for kh in (1, 2):
        lg, g1, g0, kg = grid_from(lam, 1), grid_from(u1, 1), grid_from(u0, 1), grid_from(k, kh)
        out = empty_grid(shape, 1, dtype)
        gk = grid_from(np.zeros(shape, dtype=np.float64), 1)
        L.lope_apply_var_adjoint2(lg, out, g1, g0, kg, dt, (P, P, P), gk)
        outs.append((out.numpy(), gk.numpy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
