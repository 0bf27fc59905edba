"""GPU: the persistent batched launch, lope_batch_apply (every pass of every
grid in one kernel).

Its result must equal the per-pass launches (lope_batch_apply_passes) value
for value (same
strip body, same order of passes per grid) for every depth, remainder and
edge shape, and match the oracle at the 1e-5 / 1e-12 bar; launches in a row,
and replays of a captured graph, must each start from a cleared queue.  Its
scheduling logic is exercised on the CPU by ``tests/emul/pq_emul.cpp``.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1502_03504_amd as L
import synth
from synth import DIRICHLET as D, PERIODIC as P
from tests.gpu_util import empty_grid, grid_from, rel_err, tol

pytestmark = pytest.mark.gpu


def _entries(rng, count, dtype, lo, hi):
    entries, fields = [], []
    for i in range(count):
        nx, ny = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        st = synth.dyadic_stencil(rng, "box" if i % 2 else "star")
        kinds = (P if rng.integers(2) else D, P if rng.integers(2) else D)
        u = rng.uniform(0, 1, (ny, nx)).astype(dtype)
        entries.append((grid_from(u, 1), empty_grid(u.shape, 1, dtype), st, (kinds, float(rng.uniform()))))
        fields.append(u)
    return entries, fields


def _reset(entries, fields):
    for (src, dst, _, _), u in zip(entries, fields):
        src.interior().copy_(torch.from_numpy(u).cuda())
        dst.interior().fill_(float("nan"))


def _results(plan, n):
    return [plan.result(i).interior().clone() for i in range(n)]


def test_small_persistent_batch_matches_passes():
    """One small batch first (two grids, four sweeps at depth 2)."""
    print("persistent batch: 2 grids, 4 sweeps, depth 2", flush=True)
    rng = np.random.default_rng([synth.CFG_TEST, 500])
    entries, fields = _entries(rng, 2, np.float32, 20, 90)
    plan = L.BatchPlan(entries, 4)
    plan.set_depth(2)
    _reset(entries, fields)
    plan.apply_passes()
    torch.cuda.synchronize()
    ref = _results(plan, 2)
    _reset(entries, fields)
    plan.apply()
    plan.check_persistent()
    for i in range(2):
        assert torch.equal(plan.result(i).interior(), ref[i]), i
    plan.close()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_persistent_batch_every_depth_matches_passes_and_oracle(dtype):
    """24 uneven grids (3..700 a side, mixed rules, 5- and 9-point), 9 sweeps:
    at every depth 1..8 (with and without a remainder pass) one persistent
    launch equals the per-pass launches value for value and the oracle to the
    bar."""
    rng = np.random.default_rng([synth.CFG_TEST, 501])
    n = 9
    entries, fields = _entries(rng, 24, dtype, 3, 700)
    plan = L.BatchPlan(entries, n)
    for depth in (1, 2, 3, 4, 5, 6, 7, 8):
        print("persistent batch: 24 grids, %d sweeps, depth %d, %s" % (n, depth, np.dtype(dtype).name), flush=True)
        plan.set_depth(depth)
        _reset(entries, fields)
        plan.apply_passes()
        torch.cuda.synchronize()
        ref = _results(plan, len(entries))
        _reset(entries, fields)
        plan.apply()
        plan.check_persistent()
        for i in range(len(entries)):
            assert torch.equal(plan.result(i).interior(), ref[i]), (depth, i)
        if depth == 3:
            for i, (e, u) in enumerate(zip(entries, fields)):
                want = oracle.iterate(u, e[2].coeffs, e[3][0], e[3][1], n)
                err = rel_err(plan.result(i).numpy(), want)
                assert err <= tol(dtype), (i, err)
    plan.close()


@pytest.mark.parametrize("n,depth,rows", [(0, 3, 64), (1, 4, 64), (2, 8, 7), (12, 4, 1), (13, 6, 300), (50, 6, 64)])
def test_persistent_batch_edge_shapes(n, depth, rows):
    """No sweeps; fewer sweeps than the depth (only the remainder pass); no
    remainder; one-row strips; strips taller than the grids; empty and 1x1
    grids in the batch."""
    print("persistent batch edges: n=%d depth=%d rows=%d" % (n, depth, rows), flush=True)
    rng = np.random.default_rng([synth.CFG_TEST, 502, n])
    entries, fields = _entries(rng, 9, np.float32, 1, 160)
    for shape in [(0, 5), (1, 1), (4, 0), (1, 70)]:
        u = rng.uniform(0, 1, shape).astype(np.float32)
        st = synth.dyadic_stencil(rng, "box")
        entries.append((grid_from(u, 1), empty_grid(u.shape, 1, np.float32), st, ((P, D), 0.5)))
        fields.append(u)
    plan = L.BatchPlan(entries, n)
    plan.set_tiles(depth, rows)
    _reset(entries, fields)
    plan.apply_passes()
    torch.cuda.synchronize()
    ref = _results(plan, len(entries))
    _reset(entries, fields)
    plan.apply()
    plan.check_persistent()
    for i in range(len(entries)):
        got = plan.result(i).interior()
        assert torch.equal(got, ref[i]) or (got.numel() == 0 and ref[i].numel() == 0), i
    plan.close()


def test_persistent_batch_launches_in_a_row_and_graph_replays():
    """Launches in a row continue from the current state (each finds the queue
    cleared by the previous launch's last wave); a graph capturing one launch,
    replayed with eager work in between, gives the eager result every time."""
    print("persistent batch: launches in a row and graph replays", flush=True)
    rng = np.random.default_rng([synth.CFG_TEST, 503])
    n = 7
    entries, fields = _entries(rng, 12, np.float32, 3, 300)
    plan = L.BatchPlan(entries, n)
    plan.set_depth(3)
    _reset(entries, fields)
    plan.apply_passes()
    plan.apply_passes()
    plan.apply_passes()
    torch.cuda.synchronize()
    ref3 = _results(plan, len(entries))
    _reset(entries, fields)
    plan.apply()
    plan.apply()
    plan.apply()
    plan.check_persistent()
    for i in range(len(entries)):
        assert torch.equal(plan.result(i).interior(), ref3[i]), ("three in a row", i)
    _reset(entries, fields)
    plan.apply_passes()
    torch.cuda.synchronize()
    ref = _results(plan, len(entries))
    g = torch.cuda.CUDAGraph()
    _reset(entries, fields)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.apply()
    for rep in range(3):
        _reset(entries, fields)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        plan.check_persistent()
        for i in range(len(entries)):
            assert torch.equal(plan.result(i).interior(), ref[i]), ("replay %d" % rep, i)
    del g
    plan.close()


def test_persistent_batch_abort_path(monkeypatch):
    """A zero wait limit (set from the host) makes any dependency wait not met
    at its first poll run out: the launch then ends early through the abort
    flag and check_persistent reports it, or no wait was needed and the result
    is exact.  Either way the next launch with the normal limit is exact."""
    print("persistent batch: abort path with a zero wait limit", flush=True)
    rng = np.random.default_rng([synth.CFG_TEST, 504])
    n = 12
    entries, fields = _entries(rng, 4, np.float32, 200, 400)
    plan = L.BatchPlan(entries, n)
    plan.set_tiles(2, 16)
    _reset(entries, fields)
    plan.apply_passes()
    torch.cuda.synchronize()
    ref = _results(plan, len(entries))
    monkeypatch.setenv("LOPE_PERSISTENT_WAIT_US", "0")
    _reset(entries, fields)
    plan.apply()
    try:
        plan.check_persistent()
        timed_out = False
    except L.LopeError as e:
        assert e.code == -7
        timed_out = True
    if not timed_out:
        for i in range(len(entries)):
            assert torch.equal(plan.result(i).interior(), ref[i]), i
    monkeypatch.delenv("LOPE_PERSISTENT_WAIT_US")
    _reset(entries, fields)
    plan.apply()
    plan.check_persistent()
    for i in range(len(entries)):
        assert torch.equal(plan.result(i).interior(), ref[i]), ("after abort", i)
    plan.close()


def test_persistent_batch_512_grids_matches_passes():
    """The 512-grid, 50-sweep batch at its tuned tiling: one persistent launch
    equals the graph of per-pass launches value for value."""
    print("persistent batch: 512 grids, 50 sweeps", flush=True)
    grids, steps = synth.case_batch()
    entries = [(grid_from(g.field, 1), empty_grid(g.field.shape, 1, np.float32), g.stencil, g.bc) for g in grids]
    fields = [g.field for g in grids]
    plan = L.BatchPlan(entries, steps)
    plan.apply_passes()
    torch.cuda.synchronize()
    ref = _results(plan, len(grids))
    _reset(entries, fields)
    plan.apply()
    plan.check_persistent()
    for i in range(len(grids)):
        assert torch.equal(plan.result(i).interior(), ref[i]), i
    plan.close()


def test_persistent_batch_repeated_launches_stay_exact():
    """Coherence under load: the 512-grid batch at three tilings, six
    persistent launches each (from a reset state, and two in a row), every
    grid equal to the per-pass launches value for value every time."""
    print("persistent batch: repeated launches of the 512-grid batch", flush=True)
    grids, steps = synth.case_batch()
    entries = [(grid_from(g.field, 1), empty_grid(g.field.shape, 1, np.float32), g.stencil, g.bc) for g in grids]
    fields = [g.field for g in grids]
    plan = L.BatchPlan(entries, steps)
    for depth, rows in [(8, 256), (3, 128), (5, 32)]:
        plan.set_tiles(depth, rows)
        _reset(entries, fields)
        plan.apply_passes()
        torch.cuda.synchronize()
        ref = _results(plan, len(grids))
        _reset(entries, fields)
        plan.apply_passes()
        plan.apply_passes()
        torch.cuda.synchronize()
        ref2 = _results(plan, len(grids))
        for rep in range(4):
            _reset(entries, fields)
            plan.apply()
            plan.check_persistent()
            bad = [i for i in range(len(grids)) if not torch.equal(plan.result(i).interior(), ref[i])]
            assert not bad, (depth, rows, rep, bad[:5])
        for rep in range(2):
            _reset(entries, fields)
            plan.apply()
            plan.apply()
            plan.check_persistent()
            bad = [i for i in range(len(grids)) if not torch.equal(plan.result(i).interior(), ref2[i])]
            assert not bad, (depth, rows, "two in a row", rep, bad[:5])
    plan.close()
