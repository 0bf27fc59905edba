"""GPU parity: every kernel against the CPU oracle on seeded inputs.

Sizes span several tiles and ragged tails; every boundary mix; float32 and
float64.  Bar: normwise relative error <= 1e-12 (float64) and <= 1e-5
(float32); halo fills are bit-exact; kernel variants agree exactly.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1502_03504_amd as L
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests.gpu_util import empty_grid, grid_from, halo_mask, packed_grid_from, rel_err, tol, variants_for

pytestmark = pytest.mark.gpu

SHAPES = {1: (301,), 2: (37, 133), 3: (19, 37, 70)}
BCS = {
    1: [(D,), (P,)],
    2: [(D, D), (P, P), (D, P), (P, D)],
    3: [(P, P, P), (D, D, D), (P, D, P), (D, P, D)],
}


def _field(shape, dtype, seed):
    rng = np.random.default_rng([synth.CFG_TEST, seed])
    return rng.uniform(-1, 1, size=shape).astype(dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_halo_fill_bit_exact(ndim, dtype):
    u = _field(SHAPES[ndim], dtype, 1)
    for kinds in BCS[ndim]:
        for h in (1, 3):
            g = grid_from(u, h, fill=np.nan)
            L.lope_halo_fill(g, (kinds, 0.375))
            got = g.padded().cpu().numpy()
            want = oracle.halo_fill(u, h, kinds, 0.375)
            np.testing.assert_array_equal(got, want)


CASES = [
    # ndim, radius, shape
    (1, 2, "box"), (2, 1, "box"), (2, 1, "star"), (2, 2, "box"), (2, 2, "star"),
    (3, 1, "star"), (3, 2, "star"), (3, 3, "star"), (3, 4, "star"), (3, 1, "box"),
]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("ndim,r,shape_kind", CASES)
def test_apply_matches_oracle(ndim, r, shape_kind, dtype):
    rng = np.random.default_rng([synth.CFG_TEST, 10 * ndim + r])
    st = synth.random_stencil(rng, ndim, r, shape_kind)
    u = _field(SHAPES[ndim], dtype, 2)
    for kinds in BCS[ndim]:
        src = grid_from(u, r, fill=np.nan)          # stored halo is never read
        dst = empty_grid(u.shape, r, dtype, fill=np.nan)
        L.lope_apply(src, dst, st, (kinds, 0.25))
        got = dst.numpy()
        want = oracle.sweep(u, st.coeffs, kinds, 0.25)
        assert rel_err(got, want) <= tol(dtype), (kinds, rel_err(got, want))
        # src untouched, dst halo untouched
        np.testing.assert_array_equal(src.numpy(), u)
        assert np.isnan(dst.padded().cpu().numpy()[halo_mask(dst)]).all()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("ndim,r,shape_kind", [(2, 1, "box"), (2, 1, "star"), (3, 1, "star"), (3, 2, "star"),
                                               (3, 3, "star"), (3, 4, "star")])
def test_every_variant_and_depth_agrees(ndim, r, shape_kind, dtype):
    """All tiles, depths and chunk sizes give identical values (same fma
    order), and match the oracle after n sweeps."""
    rng = np.random.default_rng([synth.CFG_TEST, 100 + 10 * ndim + r])
    st = synth.contractive(synth.random_stencil(rng, ndim, r, shape_kind))
    u = _field(SHAPES[ndim], dtype, 3)
    n = 7
    vids = variants_for(ndim, r, dtype, shape=None)
    if shape_kind == "box":
        vids = [v for v in vids if "shape=box" in v[1]]
    assert vids, "no tuned variant for this case"
    for kinds in BCS[ndim][:3]:
        want = oracle.iterate(u, st.coeffs, kinds, 0.5, n)
        ref = None
        for vid, info in vids:
            for chunk in (0, 5, 16):
                a = grid_from(u, r)
                b = empty_grid(u.shape, r, dtype)
                idx = L.lope_iterate_tuned(a, b, st, (kinds, 0.5), n, variant=vid, chunk=chunk)
                got = (a, b)[idx].numpy()
                assert rel_err(got, want) <= tol(dtype), (info, chunk, kinds, rel_err(got, want))
                if ref is None:
                    ref = got
                else:
                    np.testing.assert_array_equal(got, ref, err_msg=info)
        # the generic one-thread-per-point kernel agrees in value
        x, y = grid_from(u, r), empty_grid(u.shape, r, dtype)
        for _ in range(n):
            L.lope_iterate_tuned(x, y, st, (kinds, 0.5), 1, variant=-1)
            x, y = y, x
        np.testing.assert_array_equal(x.numpy(), ref)


@pytest.mark.parametrize("shape", [(3, 5, 7), (9, 2, 130), (1, 17, 57), (40, 9, 56), (6, 33, 113)])
def test_wave_brick_kernels_edge_shapes(shape):
    """The wave-brick 3D kernels on grids narrower than one brick, thinner than
    one row segment, shorter than one z-chunk or than the fused depth, and on
    ragged multiples: every rule mix and chunk, against one sweep per pass
    (bitwise) and the oracle."""
    rng = np.random.default_rng([synth.CFG_TEST, 120 + shape[2]])
    st = synth.contractive(synth.random_stencil(rng, 3, 1, "star"))
    u = rng.uniform(-1, 1, size=shape).astype(np.float32)
    n = 8                                   # two full passes of four sweeps
    waves = [(vid, info) for vid, info in variants_for(3, 1, np.float32) if info.startswith("star3dw_")]
    assert waves
    for kinds in BCS[3] + [(D, D, P), (P, P, D)]:
        want = oracle.iterate(u, st.coeffs, kinds, 0.5, n)
        x, y = grid_from(u, 1), empty_grid(u.shape, 1, np.float32)
        ref = (x, y)[L.lope_iterate(x, y, st, (kinds, 0.5), n, tdepth=1)].numpy()
        assert rel_err(ref, want) <= tol(np.float32), rel_err(ref, want)
        for vid, info in waves:
            for chunk in (0, 1, 3):
                a, b = grid_from(u, 1), empty_grid(u.shape, 1, np.float32)
                idx = L.lope_iterate_tuned(a, b, st, (kinds, 0.5), n, variant=vid, chunk=chunk)
                np.testing.assert_array_equal((a, b)[idx].numpy(), ref, err_msg="%s chunk %d %s" % (info, chunk, kinds))


@pytest.mark.parametrize("shape,dtype,kind", [((120000, 40), np.float32, "box"), ((30000, 100), np.float64, "star"),
                                              ((80000, 9, 2), np.float32, "star")])
def test_wave_kernels_tall_columns(shape, dtype, kind):
    """Columns of tiles far longer than wide (one or two strips of 2D rows, a
    3D z axis of 80000 planes): the automatic chunk then cuts each column
    into thousands of chunks.  Every wave variant at every depth, automatic
    chunk, against one sweep per pass (bitwise) and the oracle."""
    rng = np.random.default_rng([synth.CFG_TEST, 130 + len(shape)])
    ndim = len(shape)
    st = synth.contractive(synth.random_stencil(rng, ndim, 1, kind))
    prefix = "star3dw_" if ndim == 3 else "plane2dw_"
    u = rng.uniform(-1, 1, size=shape).astype(dtype)
    n = 8
    kinds = (D, P, D)[:ndim] if ndim == 3 else (P, D)
    want = oracle.iterate(u, st.coeffs, kinds, 0.5, n)
    x, y = grid_from(u, 1), empty_grid(u.shape, 1, dtype)
    ref = (x, y)[L.lope_iterate(x, y, st, (kinds, 0.5), n, tdepth=1)].numpy()
    assert rel_err(ref, want) <= tol(dtype), rel_err(ref, want)
    waves = [(vid, info) for vid, info in variants_for(ndim, 1, dtype, shape=kind) if info.startswith(prefix)]
    assert waves
    for vid, info in waves:
        a, b = grid_from(u, 1), empty_grid(u.shape, 1, dtype)
        idx = L.lope_iterate_tuned(a, b, st, (kinds, 0.5), n, variant=vid, chunk=0)
        np.testing.assert_array_equal((a, b)[idx].numpy(), ref, err_msg=info)


@pytest.mark.parametrize("n_steps", [0, 1, 2, 5, 8])
def test_iterate_result_index_and_auto_depth(n_steps):
    u = _field((21, 40, 66), np.float32, 4)
    st = synth.heat_star(3, 0.125)
    kinds = (P, P, P)
    want = oracle.iterate(u, st.coeffs, kinds, 0.0, n_steps)
    for tdepth in (0, 1, 2, 3, 4):
        a = grid_from(u, 1)
        b = empty_grid(u.shape, 1, np.float32)
        idx = L.lope_iterate(a, b, st, kinds, n_steps, tdepth=tdepth)
        assert idx in (0, 1)
        if tdepth == 1:
            assert idx == oracle.result_index(n_steps)
        assert rel_err((a, b)[idx].numpy(), want) <= 1e-5


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_empty_and_degenerate_grids(dtype):
    st = synth.heat_star(3, 0.1)
    for shape in [(0, 5, 5), (1, 1, 1), (1, 7, 1), (3, 1, 130), (2, 2, 2)]:
        u = _field(shape, dtype, 5)
        for kinds in BCS[3]:
            a = grid_from(u, 1)
            b = empty_grid(u.shape, 1, dtype)
            idx = L.lope_iterate(a, b, st, (kinds, 0.7), 3)
            want = oracle.iterate(u, st.coeffs, kinds, 0.7, 3)
            assert rel_err((a, b)[idx].numpy(), want) <= tol(dtype), (shape, kinds)


def test_radius_zero_and_large_halo():
    u = _field((9, 10, 11), np.float64, 6)
    st = np.array([[[2.5]]])
    a = grid_from(u, 0)
    b = empty_grid(u.shape, 0, np.float64)
    L.lope_apply(a, b, st, (P, P, P))
    np.testing.assert_array_equal(b.numpy(), 2.5 * u)
    st3 = synth.heat_star(3, 0.1)
    a = grid_from(u, 4)
    b = empty_grid(u.shape, 2, np.float64)
    L.lope_apply(a, b, st3, (D, D, D))
    assert rel_err(b.numpy(), oracle.sweep(u, st3.coeffs, (D, D, D), 0.0)) <= 1e-12


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("ndim,r,shape_kind", [(2, 1, "box"), (3, 1, "star"), (3, 4, "star"), (1, 3, "box")])
def test_adjoint_matches_oracle(ndim, r, shape_kind, dtype):
    rng = np.random.default_rng([synth.CFG_TEST, 200 + ndim + r])
    st = synth.random_stencil(rng, ndim, r, shape_kind)
    yb = _field(SHAPES[ndim], dtype, 7)
    for kinds in BCS[ndim]:
        a = grid_from(yb, r)
        b = empty_grid(yb.shape, r, dtype)
        gb = L.gbar_buffer(fill=123.0)
        L.lope_apply_adjoint(a, b, st, (kinds, 0.9), gbar=gb)
        xw, gw = oracle.adjoint(yb, st.coeffs, kinds)
        assert rel_err(b.numpy(), xw) <= tol(dtype), kinds
        assert abs(gb[0].item() - gw) <= 1e-9 * max(1.0, abs(gw)), (gb[0].item(), gw)
        # the fixed summation order: a second run gives the same bits
        again = L.gbar_buffer(fill=-5.0)
        L.lope_apply_adjoint(a, b, st, (kinds, 0.9), gbar=again)
        assert again[0].item() == gb[0].item()


@pytest.mark.parametrize("packed", [False, True])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_diffusion_forward_and_reverse(dtype, packed):
    """Aligned grids take the vector kernels, packed (misaligned) grids the
    scalar ones; both against the oracle."""
    rng = np.random.default_rng([synth.CFG_TEST, 300])
    shape = (21, 35, 70)
    u = rng.uniform(0, 1, shape).astype(dtype)
    k = rng.uniform(0.05, 0.2, shape).astype(dtype)
    lam = rng.standard_normal(shape).astype(dtype)
    dt = 0.1
    mk = packed_grid_from if packed else grid_from
    ug, kg = mk(u, 1), mk(k, 1)
    out = empty_grid(shape, 1, dtype)
    L.lope_apply_var(ug, out, kg, dt, (P, P, P))
    assert rel_err(out.numpy(), oracle.diffusion_step(u, k, dt)) <= tol(dtype)
    lg = grid_from(lam, 1)
    lam_out = empty_grid(shape, 1, dtype)
    for gdt in (np.float64, np.float32):
        gk = grid_from(np.full(shape, 0.5, dtype=gdt), 0)
        L.lope_apply_var_adjoint(lg, lam_out, ug, kg, dt, (P, P, P), gk)
        want_l = oracle.diffusion_step_transpose(lam, k, dt)
        want_g = 0.5 + oracle.diffusion_kappa_vjp(u, lam, dt)
        assert rel_err(lam_out.numpy(), want_l) <= tol(dtype)
        gtol = tol(gdt if gdt == np.float32 else dtype)   # the coarser of the two precisions
        assert rel_err(gk.numpy() - 0.5, want_g - 0.5) <= gtol, rel_err(gk.numpy() - 0.5, want_g - 0.5)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("r", [1, 4])
def test_packed_grids_take_scalar_kernels(r, dtype):
    """Misaligned grids fall back from the vector kernels and still match."""
    rng = np.random.default_rng([synth.CFG_TEST, 500 + r])
    st = synth.contractive(synth.random_stencil(rng, 3, r, "star"))
    u = _field((19, 37, 70), dtype, 11)
    for kinds in BCS[3][:2]:
        a = packed_grid_from(u, r)
        b = packed_grid_from(np.zeros_like(u), r)
        idx = L.lope_iterate(a, b, st, (kinds, 0.3), 3, tdepth=1)
        want = oracle.iterate(u, st.coeffs, kinds, 0.3, 3)
        assert rel_err((a, b)[idx].numpy(), want) <= tol(dtype)


def test_accumulate():
    rng = np.random.default_rng(8)
    part = rng.standard_normal((5, 6, 7)).astype(np.float32)
    tot = rng.standard_normal((5, 6, 7))
    pg, tg = grid_from(part, 0), grid_from(tot, 1)
    L.lope_accumulate(pg, tg)
    np.testing.assert_array_equal(tg.numpy(), tot + part.astype(np.float64))
    assert (pg.numpy() == 0).all()


def _batch_entries(rng, count, dtype, lo=3, hi=300):
    entries, fields = [], []
    for i in range(count):
        nx, ny = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        st = synth.dyadic_stencil(rng, "box" if i % 2 else "star")
        kinds = (P if rng.integers(2) else D, P if rng.integers(2) else D)
        u = rng.uniform(0, 1, (ny, nx)).astype(dtype)
        entries.append((grid_from(u, 1), empty_grid(u.shape, 1, dtype), st, (kinds, float(rng.uniform()))))
        fields.append(u)
    return entries, fields


@pytest.mark.skip(reason="the persistent work-queue batch kernel hung on the GPU twice (second time after "
                         "a fix of its polling); its cause is not shown, so that path is switched off and "
                         "this case stays off the GPU; the step-wise batch path is tested below")
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batch_matches_per_grid_and_oracle(dtype):
    rng = np.random.default_rng([synth.CFG_TEST, 400])
    n = 9
    entries, fields = _batch_entries(rng, 24, dtype)
    plan = L.BatchPlan(entries, n)
    plan.apply()
    assert plan.error() == 0
    got = [plan.result(i).numpy() for i in range(len(entries))]
    for i, (e, u) in enumerate(zip(entries, fields)):
        want = oracle.iterate(u, e[2].coeffs, e[3][0], e[3][1], n)
        assert rel_err(got[i], want) <= tol(dtype), (i, rel_err(got[i], want))
    # same grids through one launch per grid per sweep: identical values
    for (src, dst, _, _), u in zip(entries, fields):
        src.interior().copy_(torch.from_numpy(u).cuda())
    plan.apply_per_grid()
    torch.cuda.synchronize()
    for i in range(len(entries)):
        np.testing.assert_array_equal(plan.result(i).numpy(), got[i])
    # a second launch of the same graph continues from the current state
    plan.apply()
    assert plan.error() == 0
    plan.close()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_stepwise_batch_matches_per_grid_and_oracle(dtype):
    """Per-pass batched launches (every tile of every grid per launch, 1..8
    sweeps fused) against the oracle and, value for value, against one launch
    per grid per sweep."""
    rng = np.random.default_rng([synth.CFG_TEST, 401])
    n = 9
    entries, fields = _batch_entries(rng, 24, dtype, lo=3, hi=700)
    plan = L.BatchPlan(entries, n)
    ref = None
    for depth in (2, 1, 3, 4, 5, 6, 7, 8):
        for (src, _, _, _), u in zip(entries, fields):
            src.interior().copy_(torch.from_numpy(u).cuda())
        plan.set_depth(depth)
        plan.apply_passes()
        torch.cuda.synchronize()
        got = [plan.result(i).numpy() for i in range(len(entries))]
        if ref is None:
            ref = got
            for i, (e, u) in enumerate(zip(entries, fields)):
                want = oracle.iterate(u, e[2].coeffs, e[3][0], e[3][1], n)
                assert rel_err(got[i], want) <= tol(dtype), (i, rel_err(got[i], want))
        else:
            for i in range(len(entries)):
                np.testing.assert_array_equal(got[i], ref[i], err_msg="depth %d grid %d" % (depth, i))
    for (src, dst, _, _), u in zip(entries, fields):
        src.interior().copy_(torch.from_numpy(u).cuda())
    plan.apply_per_grid()
    torch.cuda.synchronize()
    for i in range(len(entries)):
        np.testing.assert_array_equal(plan.per_grid_result(i).numpy(), ref[i])
    plan.close()


def test_batch_graph_replays_and_caller_capture():
    """lope_batch_apply_passes replays its recorded graph; replays with eager
    work in between, and a caller's own captured graph, give the eager
    result."""
    rng = np.random.default_rng([synth.CFG_TEST, 402])
    n = 7
    entries, fields = _batch_entries(rng, 12, np.float32, lo=3, hi=300)

    def reset():
        for (src, _, _, _), u in zip(entries, fields):
            src.interior().copy_(torch.from_numpy(u).cuda())

    plan = L.BatchPlan(entries, n)
    plan.set_depth(3)
    reset()
    plan.apply_per_grid()
    torch.cuda.synchronize()
    ref = [plan.per_grid_result(i).numpy() for i in range(len(entries))]
    for rep in range(3):
        reset()
        plan.apply_passes()
        torch.cuda.synchronize()
        for i in range(len(entries)):
            np.testing.assert_array_equal(plan.result(i).numpy(), ref[i], err_msg="replay %d grid %d" % (rep, i))
    g = torch.cuda.CUDAGraph()
    reset()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.apply_passes()
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(entries)):
            np.testing.assert_array_equal(plan.result(i).numpy(), ref[i], err_msg="captured %d grid %d" % (rep, i))
    del g
    plan.close()


def test_errors_on_device():
    u = _field((8, 9, 10), np.float32, 9)
    a = grid_from(u, 1)
    b = empty_grid(u.shape, 1, np.float32)
    st = synth.heat_star(3, 0.1)
    # host memory is rejected before any launch
    host = torch.zeros(2000, dtype=torch.float32)
    hg = L.Grid(host, (8, 9, 10), 1, 1, 12, 12 * 11)
    with pytest.raises(L.LopeError) as e:
        L.lope_apply(hg, b, st, (P, P, P))
    assert e.value.code == -1
    # storage that does not hold the padded box is rejected
    with pytest.raises(ValueError):
        L.Grid(torch.zeros(100, dtype=torch.float32, device="cuda"), (8, 9, 10), 1, 1, 12, 12 * 11)
    with pytest.raises(L.LopeError) as e:
        L.lope_apply(a, a, st, (P, P, P))
    assert e.value.code == -3
    assert L.lope_get_device(0) == 0
