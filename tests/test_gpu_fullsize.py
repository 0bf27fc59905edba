"""Parity at the full workload sizes, in the launch configuration bench.py uses.

At these sizes the oracle cannot run whole sweep sequences, so each case is
checked on outputs the oracle computes one by one (sampled points, each on its
own window, after a few sweeps) and on properties that hold at any size:
closed-form sine-mode decay, the spectral (FFT) solution of periodic
constant-coefficient runs, sum conservation, the maximum principle of
positive weights summing to one, bitwise agreement of fused and unfused
passes, of checkpoint intervals and of batched and per-grid launches.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1502_03504_amd as L
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests.gpu_util import empty_grid, grid_from, rel_err
from tests.spectral import spectral

pytestmark = pytest.mark.gpu


def _points(shape, count, seed, edge=True):
    rng = np.random.default_rng(seed)
    pts = [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(count)]
    if edge:
        pts += [tuple(0 for _ in shape), tuple(n - 1 for n in shape),
                tuple((0 if i % 2 else n - 1) for i, n in enumerate(shape))]
    return pts


def _run(u, st, bc, n, tdepth=0, h=None):
    a = grid_from(u, h or st.radius)
    b = a.empty_like()
    idx = L.lope_iterate(a, b, st, bc, n, tdepth=tdepth)
    return (a, b)[idx]


def _sampled(u, st, bc, n, tdepth, count=48, seed=0):
    out = _run(u, st, bc, n, tdepth).interior()
    pts = _points(u.shape, count, seed)
    got = np.array([out[p].item() for p in pts])
    want = oracle.sweep_at(u, st.coeffs, bc.kinds, bc.value, n, pts)
    return got, want


def test_heat3d_512_f32_sampled_and_properties():
    case = synth.case_heat3d(n=512, dtype=np.float32, steps=1000)
    u = case.field
    for n, td in ((1, 0), (2, 0), (3, 2), (4, 4)):
        got, want = _sampled(u, case.stencil, case.bc, n, td, seed=n)
        assert rel_err(got, want) <= 1e-5, (n, td, rel_err(got, want))
    # the whole 1000-sweep run: conservation and maximum principle
    out = _run(u, case.stencil, case.bc, case.steps).interior()
    s0 = float(torch.from_numpy(u).cuda().double().sum())
    s1 = float(out.double().sum())
    assert abs(s1 - s0) <= 1e-5 * abs(s0)
    assert float(out.min()) >= float(u.min()) - 1e-6 and float(out.max()) <= float(u.max()) + 1e-6


def test_heat3d_512_f32_dirichlet_sampled_and_bitwise():
    """The 512^3 heat grid under a Dirichlet rule on every axis, with the tuned
    default (the wave brick, 4 sweeps per pass, blends only in the bricks on
    the interior's edge): sampled outputs (corners and faces included) against
    the oracle, and the 8-sweep state bitwise equal to one sweep per pass; the
    1000-sweep run stays within [min(u0, 0), max(u0, 0)] (weights >= 0 summing
    to one, g = 0)."""
    case = synth.case_heat3d(n=512, dtype=np.float32, steps=1000)
    bc = synth.Boundary((D, D, D), 0.0)
    u = case.field
    for n in (4, 8):
        got, want = _sampled(u, case.stencil, bc, n, 0, seed=20 + n)
        assert rel_err(got, want) <= 1e-5, (n, rel_err(got, want))
    fused = _run(u, case.stencil, bc, 8).interior().cpu().numpy()
    plain = _run(u, case.stencil, bc, 8, tdepth=1).interior().cpu().numpy()
    np.testing.assert_array_equal(fused, plain)
    out = _run(u, case.stencil, bc, case.steps).interior()
    lo, hi = min(float(u.min()), 0.0), max(float(u.max()), 0.0)
    assert float(out.min()) >= lo - 1e-6 and float(out.max()) <= hi + 1e-6


def test_heat3d_512_f32_fused_kernels_bitwise():
    """At the full size every fused 3D radius-1 float32 kernel (each wave-brick
    variant and the automatic choice) gives the values of one sweep per pass,
    bit for bit."""
    from tests.gpu_util import variants_for
    case = synth.case_heat3d(n=512, dtype=np.float32, steps=8)
    u = case.field
    ref = _run(u, case.stencil, case.bc, 8, tdepth=1).interior().clone()
    assert torch.equal(_run(u, case.stencil, case.bc, 8, tdepth=0).interior(), ref)
    waves = [(vid, info) for vid, info in variants_for(3, 1, np.float32) if info.startswith("star3dw_")]
    assert waves
    for vid, info in waves:
        for chunk in (0, 100):
            a = grid_from(u, 1)
            b = a.empty_like()
            idx = L.lope_iterate_tuned(a, b, case.stencil, case.bc, 8, variant=vid, chunk=chunk)
            assert torch.equal((a, b)[idx].interior(), ref), (info, chunk)
            del a, b


def test_heat3d_512_f32_closed_form_mode():
    """A pure separable mode decays by lambda^n at the full size."""
    n, steps, rc = 512, 1000, 0.125
    kinds = (P, P, P)
    ks = (3, 5, 2)
    u = synth.mode_field((n, n, n), ks, kinds).astype(np.float32)
    lam = 1.0 - 4 * rc * sum(np.sin(np.pi * k / n) ** 2 for k in ks)
    out = _run(u, synth.heat_star(3, rc), synth.Boundary(kinds, 0.0), steps).interior()
    want = torch.from_numpy(u).cuda().double() * lam ** steps
    err = float((out.double() - want).abs().max()) / float(want.abs().max())
    assert err <= 1e-5, err


def test_heat3d_512_f32_headline_run_matches_fft():
    """The benchmark's whole run (1000 sweeps of the 512^3 float32 field, the
    launch configuration bench.py times) element by element against the
    spectral solution."""
    case = synth.case_heat3d(n=512, dtype=np.float32, steps=1000)
    out = _run(case.field, case.stencil, case.bc, case.steps).numpy()
    want = spectral(case.field, case.stencil.coeffs, case.steps)
    err = rel_err(out, want)
    print("headline 512^3 f32 1000 sweeps: normwise error vs FFT %.3e" % err, flush=True)
    assert err <= 1e-5, err


def test_heat3d_256_f64_matches_fft():
    case = synth.case_heat3d(n=256, dtype=np.float64, steps=1000)
    out = _run(case.field, case.stencil, case.bc, case.steps).numpy()
    want = spectral(case.field, case.stencil.coeffs, case.steps)
    assert rel_err(out, want) <= 1e-12, rel_err(out, want)


def test_box9_8192_f32_sampled_and_fft():
    case = synth.case_box9(n=8192, steps=1000)
    u = case.field
    for n in (1, 2):
        got, want = _sampled(u, case.stencil, case.bc, n, 0, seed=10 + n)
        assert rel_err(got, want) <= 1e-5, (n, rel_err(got, want))
    out = _run(u, case.stencil, case.bc, case.steps).numpy()
    want = spectral(u, case.stencil.coeffs, case.steps)
    assert rel_err(out, want) <= 1e-5, rel_err(out, want)


def test_star25_512_sampled_depths_and_stability():
    case = synth.case_star25(n=512, steps=500)
    u = case.field
    for n, td in ((1, 1), (2, 2), (2, 1)):
        got, want = _sampled(u, case.stencil, case.bc, n, td, count=24, seed=20 + n)
        assert rel_err(got, want) <= 1e-5, (n, td, rel_err(got, want))
    # fused and unfused passes agree exactly at full size
    ref = _run(u, case.stencil, case.bc, 4, tdepth=1).numpy()
    for td in (2, 4):
        np.testing.assert_array_equal(_run(u, case.stencil, case.bc, 4, tdepth=td).numpy(), ref)
    out = _run(u, case.stencil, case.bc, case.steps)
    x = out.interior()
    assert torch.isfinite(x).all()
    assert float(x.double().norm()) <= float(torch.from_numpy(u).cuda().double().norm())


def test_heat2d_256_f64_full_oracle():
    case = synth.case_heat2d()
    out = _run(case.field, case.stencil, case.bc, case.steps).numpy()
    want = oracle.iterate(case.field, case.stencil.coeffs, case.bc.kinds, case.bc.value, case.steps)
    assert rel_err(out, want) <= 1e-12


def test_diffusion_256_checkpoint_invariance():
    from paper_1502_03504_amd.autograd import diffusion_gradient
    c = synth.case_diffusion(n=256, steps=200)
    t = lambda a: torch.from_numpy(a).cuda()
    l20, gu20, gk20 = diffusion_gradient(t(c.u0), t(c.kappa), t(c.target), c.dt, c.steps, 20)
    l1, gu1, gk1 = diffusion_gradient(t(c.u0), t(c.kappa), t(c.target), c.dt, c.steps, 2)
    assert float(l20) == float(l1)
    assert torch.equal(gu20, gu1) and torch.equal(gk20, gk1)
    assert torch.isfinite(gu20).all() and torch.isfinite(gk20).all()


def test_batch_512_grids_matches_per_grid_and_oracle():
    grids, steps = synth.case_batch()
    entries = [(grid_from(g.field, 1), empty_grid(g.field.shape, 1, np.float32), g.stencil, g.bc) for g in grids]
    plan = L.BatchPlan(entries, steps)
    plan.apply()
    torch.cuda.synchronize()
    got = [plan.result(i).interior().clone() for i in range(len(grids))]
    for (src, _, _, _), g in zip(entries, grids):
        src.interior().copy_(torch.from_numpy(g.field).cuda())
    plan.apply_per_grid()
    torch.cuda.synchronize()
    for i in range(len(grids)):
        assert torch.equal(plan.per_grid_result(i).interior(), got[i]), i
    order = sorted(range(len(grids)), key=lambda i: grids[i].field.size)
    for i in order[:3]:
        g = grids[i]
        want = oracle.iterate(g.field, g.stencil.coeffs, g.bc.kinds, g.bc.value, steps)
        err = rel_err(got[i].cpu().numpy(), want)
        assert err <= 1e-5, (i, err)
    for i in order[-2:]:
        g = grids[i]
        pts = _points(g.field.shape, 16, i)
        want = oracle.sweep_at(g.field, g.stencil.coeffs, g.bc.kinds, g.bc.value, steps, pts)
        have = np.array([got[i][p].item() for p in pts])
        assert rel_err(have, want) <= 1e-5, (i, rel_err(have, want))
    plan.close()
