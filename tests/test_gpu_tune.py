"""The autotuner end to end on a small grid: it times every fitting
(variant, chunk), registers the fastest per request and rule class, writes
the JSON table, and lope_iterate then follows the registered choice with
results identical to one sweep per pass."""
import json

import numpy as np
import pytest

import paper_1502_03504_amd as L
import synth
from paper_1502_03504_amd import tune
from synth import DIRICHLET as D, PERIODIC as P
from tests.gpu_util import empty_grid, grid_from, variants_for

pytestmark = pytest.mark.gpu


def test_autotune_registers_and_caches(tmp_path):
    rng = np.random.default_rng([synth.CFG_TEST, 600])
    u = rng.uniform(-1, 1, size=(40, 33, 70)).astype(np.float32)
    st = synth.heat_star(3, 0.1)
    bc = ((P, P, P), 0.0)
    a, b = grid_from(u, 1), empty_grid(u.shape, 1, np.float32)
    before = L.lope_select_variant(a, st, tdepth=0, bc=bc)
    dirichlet_before = L.lope_select_variant(a, st, tdepth=0, bc=((D, P, P), 0.0))
    path = tmp_path / "table.json"
    try:
        best, results = tune.autotune(a, b, st, bc, sweeps=8, chunks=(0, 16), repeats=1, cache_path=str(path))
        assert results and best == min(results, key=lambda r: r["s_per_sweep"])
        assert all(r["tdepth"] >= 1 and r["chunk"] in (0, 16) for r in results)
        # the fastest answers automatic requests; each explicit depth gets its own best
        assert L.lope_select_variant(a, st, tdepth=0, bc=bc) == best["id"]
        for d in range(1, tune.MAX_REQUEST + 1):
            of_d = [r for r in results if r["tdepth"] == d]
            if of_d:
                want = min(of_d, key=lambda r: r["s_per_sweep"])["id"]
                assert L.lope_select_variant(a, st, tdepth=d, bc=bc) == want, d
        # the periodic choice does not answer a Dirichlet request
        assert L.lope_select_variant(a, st, tdepth=0, bc=((D, P, P), 0.0)) == dirichlet_before
        table = json.loads(path.read_text())
        keys = [k for k in table if k.endswith("|0|periodic")]
        assert len(keys) == 1 and table[keys[0]]["variant"] == best["variant"]
        # the registered choice runs and equals one sweep per pass, value for value
        n = 11
        x, y = grid_from(u, 1), empty_grid(u.shape, 1, np.float32)
        ref = (x, y)[L.lope_iterate(x, y, st, bc, n, tdepth=1)].numpy()
        x, y = grid_from(u, 1), empty_grid(u.shape, 1, np.float32)
        got = (x, y)[L.lope_iterate(x, y, st, bc, n)].numpy()
        np.testing.assert_array_equal(got, ref)
    finally:
        for d in range(0, tune.MAX_REQUEST + 1):
            L.lope_tune_set(a, st, 0, tdepth=d, bc=bc)
    assert L.lope_select_variant(a, st, tdepth=0, bc=bc) == before


def test_untuned_size_keeps_a_fused_kernel():
    """A 256^3 float32 periodic heat grid (a size bucket the committed table
    was not tuned on) asked for tdepth 0 runs a fused variant of its class,
    with values identical to one sweep per pass."""
    import torch
    case = synth.case_heat3d(n=256, dtype=np.float32, steps=8)
    a = L.Grid.from_array(case.field, 1)
    vid = L.lope_select_variant(a, case.stencil, tdepth=0, bc=case.bc)
    info = L.lope_variant_info(vid)
    depth = int(dict(kv.split("=") for kv in info.split()[1:])["tdepth"])
    assert depth >= 2, info
    b = a.empty_like()
    got = (a, b)[L.lope_iterate(a, b, case.stencil, case.bc, 8)].interior().clone()
    x = L.Grid.from_array(case.field, 1)
    y = x.empty_like()
    ref = (x, y)[L.lope_iterate(x, y, case.stencil, case.bc, 8, tdepth=1)].interior()
    assert torch.equal(got, ref)


def test_huge_chunk_marches_the_whole_axis():
    """A chunk far beyond the marched extent (up to INT_MAX) is clamped: the
    values equal those of the automatic chunk."""
    rng = np.random.default_rng([synth.CFG_TEST, 610])
    for shape in ((12, 20, 70), (50, 130)):
        u = rng.uniform(-1, 1, size=shape).astype(np.float32)
        st = synth.heat_star(len(shape), 0.1)
        bc = ((P,) * len(shape), 0.0)
        x, y = grid_from(u, 1), empty_grid(shape, 1, np.float32)
        ref = (x, y)[L.lope_iterate(x, y, st, bc, 4, tdepth=1)].numpy()
        for vid, info in variants_for(len(shape), 1, np.float32, shape="star"):
            if "_t1_" not in info.split()[0] and "_t2_" not in info.split()[0] and "_t4_" not in info.split()[0]:
                continue
            a, b = grid_from(u, 1), empty_grid(shape, 1, np.float32)
            idx = L.lope_iterate_tuned(a, b, st, bc, 4, variant=vid, chunk=2 ** 31 - 1)
            np.testing.assert_array_equal((a, b)[idx].numpy(), ref, err_msg=info)


def test_batch_plan_starts_with_registered_tiling():
    """A new plan takes the tiling registered for its dtype and size bucket,
    records and replays it, and equals one launch per grid per sweep."""
    import torch
    rng = np.random.default_rng([synth.CFG_TEST, 620])
    entries, fields = [], []
    for i in range(12):
        ny, nx = (int(v) for v in rng.integers(20, 300, size=2))
        st = synth.dyadic_stencil(rng, "box" if i % 2 else "star")
        kinds = (P if rng.integers(2) else D, P if rng.integers(2) else D)
        u = rng.uniform(0, 1, (ny, nx)).astype(np.float32)
        entries.append((grid_from(u, 1), empty_grid(u.shape, 1, np.float32), st, (kinds, 0.3)))
        fields.append(u)
    points = sum(u.size for u in fields)
    try:
        L.lope_batch_tune_set(torch.float32, points, 5, 48)
        plan = L.BatchPlan(entries, 11)
        assert plan.tiles() == (5, 48)
        plan.apply()
        torch.cuda.synchronize()
        got = [plan.result(i).numpy() for i in range(len(entries))]
        for (src, _, _, _), u in zip(entries, fields):
            src.interior().copy_(torch.from_numpy(u).cuda())
        plan.apply_per_grid()
        torch.cuda.synchronize()
        for i in range(len(entries)):
            np.testing.assert_array_equal(plan.per_grid_result(i).numpy(), got[i], err_msg=str(i))
        plan.close()
    finally:
        L.lope_batch_tune_set(torch.float32, points, 0, 0)


def test_committed_batch_tiling_is_the_default():
    """The benchmark's 512-grid batch starts with the committed table's tiling."""
    grids, steps = synth.case_batch()
    points = sum(int(g.field.size) for g in grids)
    table = json.load(open(tune.DEFAULT_CACHE))
    key = tune.batch_key(0, points)
    assert key in table, key
    entries = [(grid_from(g.field, 1), empty_grid(g.field.shape, 1, np.float32), g.stencil, g.bc) for g in grids]
    plan = L.BatchPlan(entries, steps)
    assert plan.tiles() == (table[key]["tdepth"], table[key]["rows"])
    plan.close()
