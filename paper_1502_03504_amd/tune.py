"""Autotuner: choose kernel variant (tile), sweeps per pass and chunk length.

For a grid/stencil class it times every compiled variant that fits, at each
candidate chunk length (the extent of the marched axis per workgroup), with
HIP events on the current stream, and registers the fastest per-sweep choice
in the library's table (lope_tune_set), which lope_iterate consults when its
tdepth argument is 0.  Results are kept in a JSON cache keyed by
(architecture, ndim, radius, dtype, star/box, size bucket = floor(log2 points),
requested depth, boundary-rule class) and by variant NAME, so a cache
survives rebuilds that renumber variants.
Batch plans are tuned the same way: every (sweeps per launch, rows per strip)
of a plan is timed and the fastest is registered for batches of its dtype and
size bucket (floor(log2 of the batch's interior points)), with the cache key
(architecture, "batch", dtype, bucket).
Tuning runs off the timed path.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import torch

from . import _lib
from ._lib import check, load

ARCH = "gfx950"
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")
MAX_REQUEST = 4   # the deepest tdepth a caller can request of lope_iterate
# the tuning table's boundary-rule classes (lope_tuning.rules)
RULE_NAMES = ("periodic", "dirichlet")


def _variant_table():
    from . import variants
    out = {}
    for vid, info in enumerate(variants(), start=1):
        f = dict(kv.split("=") for kv in info.split()[1:])
        f["name"] = info.split()[0]
        f["id"] = vid
        out[vid] = f
    return out


def _key(ndim, radius, dtype_code, star, points):
    bucket = int(math.floor(math.log2(points))) if points > 0 else 0
    return "%s|%d|%d|%s|%s|%d" % (ARCH, ndim, radius, "f64" if dtype_code == _lib.LOPE_F64 else "f32",
                                  "star" if star else "box", bucket)


def _is_star(coeffs) -> bool:
    import numpy as np
    c = np.asarray(coeffs)
    r = (c.shape[0] - 1) // 2
    for idx in zip(*np.nonzero(c)):
        if sum(1 for i in idx if i != r) > 1:
            return False
    return True


def candidates(grid, stencil):
    """Variant ids that fit this grid and stencil (all sweep depths)."""
    star = _is_star(stencil.coeffs if hasattr(stencil, "coeffs") else stencil)
    dt = "f64" if grid.dtype == torch.float64 else "f32"
    r = int(getattr(stencil, "radius", 0))
    out = []
    for vid, f in _variant_table().items():
        if int(f["ndim"]) != grid.ndim or int(f["radius"]) != r or f["dtype"] != dt:
            continue
        if f["shape"] == "star" and not star:
            continue
        out.append(vid)
    return out


def time_choice(a, b, stencil, bc, variant, chunk, sweeps, repeats=3):
    """Median seconds per sweep of lope_iterate_tuned with this choice."""
    from . import lope_iterate_tuned
    lope_iterate_tuned(a, b, stencil, bc, sweeps, variant=variant, chunk=chunk)
    s = torch.cuda.current_stream()
    times = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        lope_iterate_tuned(a, b, stencil, bc, sweeps, variant=variant, chunk=chunk)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3 / sweeps)
    times.sort()
    return times[len(times) // 2]


def autotune(a, b, stencil, bc, sweeps=24, chunks=(0, 16, 32, 64, 128), tdepths=None, repeats=3,
             register=True, cache_path=None, log=None):
    """Time every fitting (variant, chunk); register and cache the fastest.

    Returns (best, results) with results a list of dicts.
    """
    from . import lope_tune_set
    table = _variant_table()
    results = []
    for vid in candidates(a, stencil):
        td = int(table[vid]["tdepth"])
        if tdepths is not None and td not in tdepths:
            continue
        n = max(td, (sweeps // td) * td)
        for ch in chunks:
            t = time_choice(a, b, stencil, bc, vid, ch, n, repeats)
            pts = a.storage.numel() and math.prod(a.shape)
            rec = {"variant": table[vid]["name"], "id": vid, "tdepth": td, "chunk": ch, "s_per_sweep": t,
                   "gpts": pts / t / 1e9}
            results.append(rec)
            if log:
                log("%-40s chunk=%-4d %.3f ms/sweep %.1f GPt/s" % (rec["variant"], ch, t * 1e3, rec["gpts"]))
    if not results:
        return None, results
    best = min(results, key=lambda r: r["s_per_sweep"])
    # the overall best answers automatic requests (0); the best of each depth
    # answers explicit requests for that depth (requests go up to MAX_REQUEST;
    # deeper variants serve automatic requests only)
    choices = {0: best}
    for r in results:
        d = r["tdepth"]
        if d > MAX_REQUEST:
            continue
        if d not in choices or r["s_per_sweep"] < choices[d]["s_per_sweep"]:
            choices[d] = r
    if register:
        from . import rule_class
        rules = rule_class(bc, a.ndim)
        for req, r in choices.items():
            lope_tune_set(a, stencil, r["id"], req, r["chunk"], bc=bc)
        if cache_path:
            st = stencil.coeffs if hasattr(stencil, "coeffs") else stencil
            key = _key(a.ndim, int(getattr(stencil, "radius", 0)),
                       _lib.LOPE_F64 if a.dtype == torch.float64 else _lib.LOPE_F32, _is_star(st),
                       math.prod(a.shape))
            cache = load_cache_file(cache_path)
            for req, r in choices.items():
                cache["%s|%d|%s" % (key, req, RULE_NAMES[rules])] = {
                    "variant": r["variant"], "tdepth": r["tdepth"], "chunk": r["chunk"], "gpts": round(r["gpts"], 2)}
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
    return best, results


def load_cache_file(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def register_cache(path=None) -> int:
    """Register every cached choice whose variant the compiled library has; returns the count."""
    path = path or os.environ.get("LOPE_TUNE_CACHE", DEFAULT_CACHE)
    cache = load_cache_file(path)
    if not cache:
        return 0
    names = {f["name"]: vid for vid, f in _variant_table().items()}
    lib = load()
    count = 0
    for key, v in cache.items():
        parts = key.split("|")
        if len(parts) == 4 and parts[1] == "batch":
            arch, _, dt, bucket = parts
            if arch != ARCH:
                continue
            code = _lib.LOPE_F64 if dt == "f64" else _lib.LOPE_F32
            if lib.lope_batch_tune_set(code, 1 << int(bucket), int(v["tdepth"]), int(v["rows"])) == 0:
                count += 1
            continue
        if len(parts) == 6:
            parts.append("0")
        if len(parts) == 7:
            parts.append(RULE_NAMES[0])
        arch, ndim, radius, dt, shape, bucket, req, rules = parts
        if rules not in RULE_NAMES:
            continue
        req = int(req)
        if arch != ARCH or v["variant"] not in names:
            continue
        ndim, radius, bucket = int(ndim), int(radius), int(bucket)
        # a descriptor of the key's class: only its shape class is read
        g = _lib.lope_grid()
        g.ndim = ndim
        g.h = radius
        g.dtype = _lib.LOPE_F64 if dt == "f64" else _lib.LOPE_F32
        # a near-cube of 2^bucket points (planes small enough for every
        # family's offset limits)
        e = [0, 0, 0]
        for a in range(bucket):
            e[(ndim - 1 - a % ndim) if ndim > 1 else 0] += 1
        n = [1 << e[0], 1 << e[1], 1 << e[2]]
        for a in range(3):
            g.n[a] = n[a] if a < ndim else 1
        g.stride[0] = 1
        # strides and origin in whole 128-byte lines, like Grid.allocate, so
        # vector variants accept the descriptor
        g.stride[1] = ((g.n[0] + 2 * radius + 63) // 64) * 64 if ndim >= 2 else 0
        g.stride[2] = g.stride[1] * (g.n[1] + 2 * radius) if ndim >= 3 else 0
        g.origin = 0x100000
        w = 2 * radius + 1
        import numpy as np
        c = np.zeros((w,) * ndim)
        c[(radius,) * ndim] = 1.0
        if radius > 0:
            idx = [radius] * ndim
            idx[-1] = radius + 1
            c[tuple(idx)] = 0.5
            if shape == "box" and ndim >= 2:
                idx2 = [radius + 1] * ndim
                c[tuple(idx2)] = 0.25
        s = _lib.lope_stencil()
        s.ndim = ndim
        s.radius = radius
        s.coeffs = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        t = _lib.lope_tuning(names[v["variant"]], req, int(v["chunk"]), RULE_NAMES.index(rules))
        if lib.lope_tune_set(ctypes.byref(g), ctypes.byref(s), ctypes.byref(t)) == 0:
            count += 1
    return count


# The workloads the committed gfx950 table is tuned on: (name, case maker,
# candidate z- or row-chunk lengths).  The cases are the seeded synthetic
# inputs of the benchmark (package `synth` at the repository root).
def _workloads():
    import numpy as np
    import synth
    return [
        ("heat3d512", lambda: synth.case_heat3d(512, np.float32, 10), (0, 16, 32, 64, 128)),
        ("heat3d256f64", lambda: synth.case_heat3d(256, np.float64, 10), (0, 16, 32, 64, 128)),
        ("box9", lambda: synth.case_box9(8192, 10), (0, 32, 64, 128, 256)),
        ("heat3d512dir", lambda: synth.case_heat3d(512, np.float32, 10)._replace(
            bc=synth.Boundary((synth.DIRICHLET,) * 3, 0.0)), (0, 16, 32, 64, 128)),
        ("star25", lambda: synth.case_star25(512, 10), (0, 32, 64, 128)),
        ("heat2d", lambda: synth.case_heat2d(256, 10), (0, 2, 4, 8, 16, 32, 64)),
    ]


BATCH_ROWS = (32, 64, 128, 256)


def batch_key(dtype_code, points):
    bucket = int(math.floor(math.log2(points))) if points > 0 else 0
    return "%s|batch|%s|%d" % (ARCH, "f64" if dtype_code == _lib.LOPE_F64 else "f32", bucket)


def autotune_batch(plan, points, depths=range(1, 9), rows=BATCH_ROWS, repeats=3, register=True, cache_path=None,
                   log=None):
    """Time a batch plan's persistent launch at every (sweeps per pass, rows
    per strip) and register the fastest for batches of its dtype and size
    bucket (the tiling lope_batch_plan_create then starts with).  Returns
    (best, results)."""
    from . import lope_batch_tune_set
    s = torch.cuda.current_stream()
    results = []
    for td in depths:
        for r in rows:
            plan.set_tiles(td, r)
            plan.apply()              # first launch at this tiling (untimed)
            times = []
            for _ in range(repeats):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s)
                plan.apply()
                e1.record(s)
                e1.synchronize()
                times.append(e0.elapsed_time(e1) * 1e-3)
            t = sorted(times)[len(times) // 2]
            rec = {"tdepth": td, "rows": r, "s": t, "gpts": points * plan.n_steps / t / 1e9}
            results.append(rec)
            if log:
                log("batch tdepth=%d rows=%-4d %.3f ms %.1f GPt/s" % (td, r, t * 1e3, rec["gpts"]))
    best = min(results, key=lambda r: r["s"])
    dtype = plan.entries[0][0].dtype
    if register:
        lope_batch_tune_set(dtype, points, best["tdepth"], best["rows"])
        if cache_path:
            cache = load_cache_file(cache_path)
            code = _lib.LOPE_F64 if dtype == torch.float64 else _lib.LOPE_F32
            cache[batch_key(code, points)] = {"tdepth": best["tdepth"], "rows": best["rows"],
                                              "gpts": round(best["gpts"], 2)}
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
    plan.set_tiles(best["tdepth"], best["rows"])
    return best, results


def _tune_batch_workload(path, log=None):
    """The 512-grid batch of the benchmark (seeded synthetic grids)."""
    import synth
    from . import BatchPlan, Grid
    grids, steps = synth.case_batch()
    entries = [(Grid.from_array(g.field, 1), Grid.allocate(g.field.shape, 1, torch.float32), g.stencil, g.bc)
               for g in grids]
    points = sum(int(g.field.size) for g in grids)
    plan = BatchPlan(entries, steps)
    best, _ = autotune_batch(plan, points, cache_path=path, log=log)
    plan.close()
    del entries
    torch.cuda.empty_cache()
    return best


def tune_workloads(path, names=None, log=None):
    """Time every fitting (variant, chunk) on the benchmark workloads and write
    the choices to the JSON table at `path`: replaced when every workload is
    tuned; with `names`, only the keys those workloads write change.  Needs a
    GPU."""
    from . import Grid
    kept = {}
    if os.path.exists(path):
        if names:
            with open(path) as f:
                kept = json.load(f)
        os.remove(path)
    out = {}
    if not names or "batch" in names:
        if log:
            log("== batch")
        out["batch"] = _tune_batch_workload(path, log=log)
        if log:
            log("best: %s" % out["batch"])
    for name, make, chunks in _workloads():
        if names and name not in names:
            continue
        case = make()
        if log:
            log("== %s" % name)
        a = Grid.from_array(case.field, case.h)
        b = a.empty_like()
        best, _ = autotune(a, b, case.stencil, case.bc, sweeps=24, chunks=chunks, cache_path=path, log=log)
        out[name] = best
        if log:
            log("best: %s" % best)
        del a, b, case
        torch.cuda.empty_cache()
    if kept:
        fresh = {}
        if os.path.exists(path):
            with open(path) as f:
                fresh = json.load(f)
        kept.update(fresh)
        with open(path, "w") as f:
            json.dump(kept, f, indent=1, sort_keys=True)
    return out


if __name__ == "__main__":
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="re-tune the kernel table on the benchmark workloads")
    ap.add_argument("--out", default=DEFAULT_CACHE, help="table to write (default: the committed one)")
    ap.add_argument("names", nargs="*", help="workloads to tune (default: all)")
    args = ap.parse_args()
    tune_workloads(args.out, set(args.names) or None, log=lambda *m: print(*m, flush=True))
    sys.exit(0)
