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
from tests.gpu_util import empty_grid, grid_from

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
