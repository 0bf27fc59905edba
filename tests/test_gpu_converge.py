"""lope_iterate_until on the GPU against the oracle's convergence-driven loop,
its special cases, and properties at the full 512^3 size."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1502_03504_amd as L
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests.gpu_util import TOL, empty_grid, grid_from, rel_err

pytestmark = pytest.mark.gpu


def _trajectory(u0, st, kinds, g, m, checks):
    """Oracle residuals at the first `checks` checked sweeps."""
    u, out = u0, []
    for t in range(m * checks):
        v = oracle.sweep(u, st.coeffs, kinds, g)
        if (t + 1) % m == 0:
            out.append(float(np.max(np.abs(v.astype(np.float64) - u.astype(np.float64)))))
        u = v
    return out


def _tol_between(res):
    """A tolerance that falls strictly between two consecutive checked residuals
    far from both (so rounding differences cannot move the stop), and the
    index of the check where the loop must stop."""
    for k in range(len(res) // 2, len(res) - 1):
        if res[k] > 1.05 * res[k + 1]:
            return math.sqrt(res[k] * res[k + 1]), k + 1
    raise AssertionError("residuals do not decrease")


def _max_diff(x, y):
    return float((x.double() - y.double()).abs().max())


def _plain(u0, h, st, bc, n):
    """The grid holding the state after n sweeps of lope_iterate."""
    a, b = grid_from(u0, h), empty_grid(u0.shape, h, u0.dtype)
    return (a, b)[L.lope_iterate(a, b, st, bc, n)]


CASES = [
    ("heat2d_f64_dirichlet", (40, 56), np.float64, lambda: synth.heat_star(2, 0.2), (D, D), 0.0, 3),
    ("heat3d_f32_periodic", (20, 24, 36), np.float32, lambda: synth.heat_star(3, 0.125), (P, P, P), 0.0, 4),
    ("box9_f32_mixed", (33, 70), np.float32, lambda: synth.dyadic_stencil(np.random.default_rng(5), "box"),
     (P, D), 0.4, 5),
    ("star25_f64_dirichlet", (18, 20, 22), np.float64, lambda: synth.laplacian8_star(3, 0.05),
     (D, D, D), 0.0, 2),
]


@pytest.mark.parametrize("name,shape,dtype,mk,kinds,g,m", CASES, ids=[c[0] for c in CASES])
def test_matches_oracle(name, shape, dtype, mk, kinds, g, m):
    rng = np.random.default_rng([synth.CFG_TEST, 910])
    st = mk()
    u0 = rng.uniform(0, 1, shape).astype(dtype)
    res = _trajectory(u0, st, kinds, g, m, 12)
    tol, k = _tol_between(res)
    want_u, want_steps, want_res = oracle.iterate_until(u0, st.coeffs, kinds, g, 1000, m, tol)
    assert want_steps == (k + 1) * m
    h = st.radius
    a, b = grid_from(u0, h), empty_grid(shape, h, dtype)
    idx, steps, r = L.lope_iterate_until(a, b, st, (kinds, g), 1000, m, tol)
    assert steps == want_steps
    out = (a, b)[idx]
    err = rel_err(out.numpy(), want_u)
    assert err <= TOL[dtype], (name, err)
    # each residual is a difference of two states, each within the state bar
    # of the oracle's, so the residuals differ by at most twice that bar
    assert abs(r - want_res) <= 2 * TOL[dtype] * float(np.abs(want_u).max()), (r, want_res)
    # the residual is exact: the max change between plain runs of steps-1 and steps sweeps
    assert r == _max_diff(out.interior(), _plain(u0, h, st, (kinds, g), steps - 1).interior())


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_residual_is_exact_and_state_equals_plain_iteration(dtype):
    rng = np.random.default_rng([synth.CFG_TEST, 911])
    st = synth.heat_star(3, 0.125)
    u0 = rng.uniform(0, 1, (30, 17, 45)).astype(dtype)
    a, b = grid_from(u0, 1), empty_grid(u0.shape, 1, dtype)
    idx, steps, r = L.lope_iterate_until(a, b, st, (P, D, P), 1, 1, -1.0)
    assert (idx, steps) == (1, 1)
    assert r == _max_diff(b.interior(), torch.from_numpy(u0).cuda())
    # fused checked passes (the residual comes from inside the pass) at every depth
    for tdepth in (1, 2, 3, 4):
        a, b = grid_from(u0, 1), empty_grid(u0.shape, 1, dtype)
        idx, steps, r = L.lope_iterate_until(a, b, st, (P, D, P), 12, 6, -1.0, tdepth=tdepth)
        assert steps == 12
        assert r == _max_diff((a, b)[idx].interior(), _plain(u0, 1, st, (P, D, P), 11).interior()), tdepth
    # a run that stops on a check: same values as lope_iterate for that count
    for tdepth in (0, 1, 3):
        a, b = grid_from(u0, 1), empty_grid(u0.shape, 1, dtype)
        idx, steps, r = L.lope_iterate_until(a, b, st, (P, D, P), 500, 7, 1e-3, tdepth=tdepth)
        assert steps % 7 == 0 and 0 < steps < 500 and r <= 1e-3
        c, d = grid_from(u0, 1), empty_grid(u0.shape, 1, dtype)
        j = L.lope_iterate(c, d, st, (P, D, P), steps)
        assert torch.equal((a, b)[idx].interior(), (c, d)[j].interior()), tdepth


@pytest.mark.parametrize("kinds", [(P, P, P), (D, P, D), (P, D, P)])
def test_residual_from_each_fused_3d_kernel(kinds):
    """Every fused 3D radius-1 float32 kernel that reports the residual of its
    last sweep, chosen through the tuning table, gives the exact residual and
    the state of the plain iteration."""
    from tests.gpu_util import variants_for
    rng = np.random.default_rng([synth.CFG_TEST, 913])
    st = synth.heat_star(3, 0.125)
    u0 = rng.uniform(0, 1, (26, 19, 70)).astype(np.float32)
    bc = (kinds, 0.3)
    want_prev = _plain(u0, 1, st, bc, 11).interior()
    want = _plain(u0, 1, st, bc, 12).interior()
    fused = [(vid, info) for vid, info in variants_for(3, 1, np.float32)
             if info.startswith(("star3dw_", "star3df_")) and "tdepth=1 " not in info]
    assert any(info.startswith("star3dw_") for _, info in fused)
    probe = grid_from(u0, 1)
    try:
        for vid, info in fused:
            td = int(info.split("tdepth=")[1].split()[0])
            L.lope_tune_set(probe, st, vid, td, bc=bc)
            L.lope_tune_set(probe, st, vid, 0, bc=bc)
            a, b = grid_from(u0, 1), empty_grid(u0.shape, 1, np.float32)
            idx, steps, r = L.lope_iterate_until(a, b, st, bc, 12, 6, -1.0, tdepth=td)
            assert steps == 12, info
            assert torch.equal((a, b)[idx].interior(), want), info
            assert r == _max_diff(want, want_prev), info
    finally:
        for td in (0, 2, 3, 4):
            L.lope_tune_set(probe, st, 0, td, bc=bc)


def test_special_cases():
    rng = np.random.default_rng([synth.CFG_TEST, 912])
    st = synth.heat_star(2, 0.125)
    u0 = rng.uniform(0, 1, (21, 35)).astype(np.float32)
    bc = ((P, P), 0.0)
    scratch = torch.empty(1, dtype=torch.float64, device="cuda")
    # infinite tolerance: stops at the first check
    a, b = grid_from(u0, 1), empty_grid(u0.shape, 1, np.float32)
    idx, steps, r = L.lope_iterate_until(a, b, st, bc, 50, 4, math.inf, scratch=scratch)
    assert steps == 4 and idx == 0 and r > 0
    # negative tolerance: the fixed-count iteration, bit for bit
    a, b = grid_from(u0, 1), empty_grid(u0.shape, 1, np.float32)
    idx, steps, r = L.lope_iterate_until(a, b, st, bc, 13, 4, -1.0, scratch=scratch)
    c, d = grid_from(u0, 1), empty_grid(u0.shape, 1, np.float32)
    j = L.lope_iterate(c, d, st, bc, 13)
    assert steps == 13 and torch.equal((a, b)[idx].interior(), (c, d)[j].interior())
    # no check within the budget: no residual
    a, b = grid_from(u0, 1), empty_grid(u0.shape, 1, np.float32)
    idx, steps, r = L.lope_iterate_until(a, b, st, bc, 5, 6, 1.0, scratch=scratch)
    assert steps == 5 and idx == 1 and math.isnan(r)
    # zero sweeps
    idx, steps, r = L.lope_iterate_until(a, b, st, bc, 0, 6, 1.0, scratch=scratch)
    assert (idx, steps) == (0, 0) and math.isnan(r)
    # a fixed point: residual exactly 0 at the first check
    c = np.full((21, 35), 0.375, dtype=np.float32)
    a, b = grid_from(c, 1), empty_grid(c.shape, 1, np.float32)
    idx, steps, r = L.lope_iterate_until(a, b, st, ((P, D), 0.375), 100, 3, 0.0, scratch=scratch)
    assert steps == 3 and r == 0.0
    assert bool(((a, b)[idx].interior() == 0.375).all())
    # an empty interior
    e0, e1 = empty_grid((0, 8), 1, np.float32), empty_grid((0, 8), 1, np.float32)
    idx, steps, r = L.lope_iterate_until(e0, e1, st, bc, 10, 1, 0.0, scratch=scratch)
    assert (idx, steps) == (0, 0)
    # a scratch tensor in host memory is rejected before any launch
    with pytest.raises(TypeError):
        L.lope_iterate_until(a, b, st, bc, 10, 1, 0.0, scratch=torch.zeros(1, dtype=torch.float64))


def test_heat3d_512_f32_properties():
    """Full size, checks every 100 sweeps: the state equals lope_iterate's for
    the same sweep count, bit for bit, and the residual equals the max change
    made by the last sweep exactly."""
    case = synth.case_heat3d(n=512, dtype=np.float32, steps=1000)
    a = grid_from(case.field, 1)
    b = a.empty_like()
    idx, steps, r = L.lope_iterate_until(a, b, case.stencil, case.bc, 1000, 100, 1e-5)
    assert steps % 100 == 0 and 0 < steps <= 1000
    assert steps == 1000 or r <= 1e-5
    out = (a, b)[idx]
    # same values as lope_iterate for that count, and the residual is exact
    c = grid_from(case.field, 1)
    d = c.empty_like()
    j = L.lope_iterate(c, d, case.stencil, case.bc, steps - 1)
    prev = (c, d)[j]
    nxt = (d, c)[j]
    L.lope_apply(prev, nxt, case.stencil, case.bc)
    assert torch.equal(out.interior(), nxt.interior())
    assert r == _max_diff(nxt.interior(), prev.interior())
