"""lope_batch_apply_noalloc (the batch call that allocates no device memory:
its tables go to the library's static scratch) against lope_batch_apply on a
plan, value for value, on two calls in a row, the second with a smaller
batch; the oracle pins both at the stated tolerance.  Also: a batch whose
tables exceed the scratch is refused before anything runs, and a capturing
stream is refused."""
import numpy as np
import pytest
import torch

import oracle
import paper_1502_03504_amd as L
import synth
from paper_1502_03504_amd import _lib
from synth import DIRICHLET as D
from synth import PERIODIC as P
from tests.gpu_util import empty_grid, grid_from, rel_err, tol

pytestmark = pytest.mark.gpu


def _batch(rng, count, dtype, lo, hi):
    specs = []
    for i in range(count):
        nx, ny = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        st = synth.dyadic_stencil(rng, "box" if i % 2 else "star")
        kinds = (P if rng.integers(2) else D, P if rng.integers(2) else D)
        u = rng.uniform(0, 1, (ny, nx)).astype(dtype)
        specs.append((u, st, (kinds, float(rng.uniform()))))
    return specs


def _entries(specs, dtype):
    return [(grid_from(u, 1), empty_grid(u.shape, 1, dtype, fill=np.nan), st, bc) for u, st, bc in specs]


def _via_plan(specs, dtype, n, tiles=None):
    entries = _entries(specs, dtype)
    plan = L.BatchPlan(entries, n)
    if tiles:
        plan.set_tiles(*tiles)
    plan.apply()
    torch.cuda.synchronize()
    out = [plan.result(i).numpy() for i in range(len(entries))]
    plan.close()
    return out


def _via_noalloc(specs, dtype, n, tdepth=0, rows=0):
    entries = _entries(specs, dtype)
    idx = L.lope_batch_apply_noalloc(entries, n, tdepth=tdepth, rows=rows)
    torch.cuda.synchronize()
    return [(e[1] if idx else e[0]).numpy() for e in entries]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_two_calls_match_the_plan_and_the_oracle(dtype):
    rng = np.random.default_rng([synth.CFG_TEST, 700])
    big = _batch(rng, 40, dtype, 3, 400)
    small = _batch(rng, 7, dtype, 3, 90)
    n = 11
    for specs in (big, small):          # the second call reuses the scratch with a smaller batch
        got = _via_noalloc(specs, dtype, n)
        want = _via_plan(specs, dtype, n)
        for i in range(len(specs)):
            np.testing.assert_array_equal(got[i], want[i])
        for i in range(0, len(specs), 5):
            u, st, (kinds, g) = specs[i]
            ref = oracle.iterate(u, st.coeffs, kinds, g, n)
            assert rel_err(got[i], ref) <= tol(dtype), (i, rel_err(got[i], ref))


def test_explicit_tiling_matches_the_plan():
    rng = np.random.default_rng([synth.CFG_TEST, 701])
    specs = _batch(rng, 16, np.float32, 3, 300)
    n = 9
    for tdepth, rows in ((4, 32), (8, 200), (1, 7)):
        got = _via_noalloc(specs, np.float32, n, tdepth, rows)
        want = _via_plan(specs, np.float32, n, tiles=(tdepth, rows))
        for i in range(len(specs)):
            np.testing.assert_array_equal(got[i], want[i])


def test_tables_beyond_the_scratch_are_refused():
    """16 grids of 1024 x 1024 cut into one-row strips need about 4.4 MB of
    strip tables (more than the 4 MiB scratch): refused, nothing written."""
    rng = np.random.default_rng([synth.CFG_TEST, 702])
    st = synth.dyadic_stencil(rng, "star")
    entries = []
    for _ in range(16):
        src = empty_grid((1024, 1024), 1, np.float32, fill=1.0)
        dst = empty_grid((1024, 1024), 1, np.float32, fill=7.0)
        entries.append((src, dst, st, ((P, P), 0.0)))
    with pytest.raises(L.LopeError) as ei:
        L.lope_batch_apply_noalloc(entries, 3, tdepth=1, rows=1)
    assert ei.value.code == _lib.LOPE_ERR_UNSUPPORTED
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert all(bool(torch.all(e[1].padded() == 7.0)) for e in entries)
    # the same grids in 64-row strips fit, and run
    idx = L.lope_batch_apply_noalloc(entries, 3, tdepth=1, rows=64)
    torch.cuda.synchronize()
    assert idx == 1 and bool(torch.all(entries[0][1].interior() == 1.0))


def test_capturing_stream_is_refused():
    rng = np.random.default_rng([synth.CFG_TEST, 703])
    entries = _entries(_batch(rng, 3, np.float32, 5, 40), np.float32)
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with pytest.raises(L.LopeError, match="captured"):
        with torch.cuda.graph(g):
            L.lope_batch_apply_noalloc(entries, 2)
    torch.cuda.synchronize()
