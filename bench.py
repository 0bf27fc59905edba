#!/usr/bin/env python3
"""Throughput of the LOPe sweep on one MI355X.

Workload (one "step"): 1000 Jacobi sweeps of the 3D 7-point heat stencil
(r = 1/8, centre 1/4) over a 512^3 float32 periodic grid, halo h = 1, initial
field U[0,1) plus 4 seeded sine modes, double buffered.  Inputs are resident
in HBM before timing starts.  Prints ONE JSON line.

value = GPoint-updates/s = 512^3 * sweeps * steps / elapsed.  The roofline
object reports the dominant kernel's effective HBM bandwidth: 8 algorithmic
bytes per point-update (read 4 B, write 4 B) times the point-updates of one
launch, over the kernel's average duration measured with HIP events on the
stream the kernels run on.  The cpu_baseline object times the CPU oracle on a
bounded sample (a few full-size sweeps).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
VALU_LANE_OPS = 256 * 64 * 2.4e9   # fp32 lane operations per second, one per clock per lane


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measure_traffic_table():
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def measured_traffic(kernel, n, sweeps):
    """HBM bytes per launch from the committed counter runs (FETCH_SIZE and
    WRITE_SIZE, scaled by a known-size copy), if they were taken on this very
    kernel variant and workload; else None."""
    import hashlib
    key = "%s|heat3d_7pt_%d^3_f32_periodic" % (kernel, n)
    rec = measure_traffic_table().get(key)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["kernel_source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["kernel_source_sha256"]:
        return None          # the kernel changed since the counters were taken
    return rec["traffic_bytes_per_launch"]


def measure_adjoint(n=256, steps=200, every=20):
    """Per-step forward / reverse kernel times of the variable-coefficient
    diffusion step (256^3 float32, periodic), and the end-to-end checkpointed
    gradient (forward with checkpoint saves, then recompute + reverse)."""
    import numpy as np
    import torch

    import paper_1502_03504_amd as L
    import synth
    from paper_1502_03504_amd.autograd import diffusion

    c = synth.case_diffusion(n=n, steps=steps, k=every)
    bc = (("periodic",) * 3, 0.0)
    u = L.Grid.from_array(c.u0, 1)
    v = u.empty_like()
    kap = L.Grid.from_array(c.kappa, 1)
    lam = L.Grid.from_array(c.target, 1)
    lam2 = lam.empty_like()
    g32 = L.Grid.allocate(c.u0.shape, 0, torch.float32)
    s = torch.cuda.current_stream()

    def timed(fn, reps=7, calls=20):
        """Median over reps of the time per call of `calls` back-to-back calls
        (the host-side checks of each call overlap the previous kernels, as
        in the time loop of the gradient driver)."""
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(calls):
                fn()
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / calls)
        ts.sort()
        return ts[len(ts) // 2]

    fwd = timed(lambda: L.lope_apply_var(u, v, kap, c.dt, bc))
    # the reverse steps the gradient driver runs: two steps per fused pass
    adj = timed(lambda: L.lope_apply_var_adjoint2(lam, lam2, u, v, kap, c.dt, bc, g32)) / 2.0
    # context: one reverse step per call
    one = timed(lambda: L.lope_apply_var_adjoint(lam, lam2, u, kap, c.dt, bc, g32))
    u0 = torch.from_numpy(c.u0).cuda()
    k0 = torch.from_numpy(c.kappa).cuda()
    tg = torch.from_numpy(c.target).cuda()
    for rep in range(2):          # the first run warms the allocator; the second is timed
        uu = u0.clone().requires_grad_(True)
        kk = k0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uT = diffusion(uu, kk, c.dt, steps, every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        d = uT.double() - tg.double()
        (d * d).sum().backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del uT, d, uu, kk
    pts = n ** 3
    return {"workload": "diffusion_7pt_varcoef_%d^3_f32_periodic_%d_steps_checkpoint_%d" % (n, steps, every),
            "fwd_ms_per_step": round(fwd, 4), "adj_ms_per_step": round(adj, 4),
            "ratio_per_step": round(adj / fwd, 3),
            "fwd_GBs": round(12.0 * pts / (fwd * 1e-3) / 1e9, 1),
            "fwd_frac": round(12.0 * pts / (fwd * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "adj_GBs": round(14.0 * pts / (adj * 1e-3) / 1e9, 1),
            "adj_frac": round(14.0 * pts / (adj * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "one_step_ms": round(one, 4), "one_step_GBs": round(24.0 * pts / (one * 1e-3) / 1e9, 1),
            "ratio_one_step": round(one / fwd, 3),
            "fwd_total_ms": round((t1 - t0) * 1e3, 2), "bwd_total_ms": round((t2 - t1) * 1e3, 2),
            "ratio_end_to_end": round((t2 - t1) / (t1 - t0), 3)}


def measure_batch(reps=3, per_grid=True, by_depth_sweep=True):
    """512 uneven 2D float32 grids, 50 sweeps each: the single persistent
    launch (lope_batch_apply) and the graph of one launch per fused pass,
    against one launch per grid per sweep (median of reps, HIP events)."""
    import numpy as np
    import torch

    import paper_1502_03504_amd as L
    import synth

    grids, steps = synth.case_batch()
    entries = [(L.Grid.from_array(g.field, 1), L.Grid.allocate(g.field.shape, 1, torch.float32), g.stencil, g.bc)
               for g in grids]
    points = sum(int(g.field.size) for g in grids)
    plan = L.BatchPlan(entries, steps)
    s = torch.cuda.current_stream()

    def timed(fn, n=None, warm=2):
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(n or max(reps, 5)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        return ts[len(ts) // 2]

    # the plan's own tiling: the one the tuning table registers for this
    # batch's dtype and size (what lope_batch_apply does by default): every
    # pass of every grid in one persistent kernel launch
    depth, rows = plan.tiles()
    tb = timed(plan.apply, warm=20)   # the first launches after set-up run slower
    plan.check_persistent()
    # the same sweeps as one launch per fused pass (a recorded graph), at the
    # same tiling and at the tiling measured fastest for it (6 per pass,
    # 64-row strips)
    tpass = timed(plan.apply_passes)
    plan.set_tiles(6, 64)
    tpass6 = timed(plan.apply_passes)
    plan.set_tiles(depth, rows)
    tp = timed(plan.apply_per_grid, reps) if per_grid else None
    # context only: the persistent launch at every depth at the plan's rows
    by_depth = {}
    if by_depth_sweep:
        for td in range(1, 9):
            plan.set_depth(td)
            by_depth[td] = timed(plan.apply)
        plan.check_persistent()
    plan.close()
    upd = points * steps
    return {"workload": "batch_512_grids_2d_f32_50_sweeps", "points": points, "tdepth": depth, "rows": rows,
            "batched_ms": round(tb, 3), "per_grid_ms": round(tp, 3) if tp else None,
            "batched_GPts": round(upd / (tb * 1e-3) / 1e9, 1),
            "per_grid_GPts": round(upd / (tp * 1e-3) / 1e9, 1) if tp else None,
            "speedup": round(tp / tb, 2) if tp else None,
            "batched_ms_by_depth": {str(k): round(v, 3) for k, v in by_depth.items()} or None,
            "passes_ms": round(tpass, 3), "passes_ms_t6_rows64": round(tpass6, 3),
            "launches_batched": 1, "launches_passes": -(-steps // depth), "launches_per_grid": steps * len(grids)}


def measure_copy(mib=1024, reps=10):
    """Attainable-bandwidth reference: the library's streaming copy kernel
    (16-byte non-temporal loads and stores) over `mib` MiB, bytes read +
    written over its median time; torch's copy kernel beside it for context."""
    import torch

    import paper_1502_03504_amd as L
    n_el = mib * (1 << 20) // 4
    src = torch.ones(n_el, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()

    def timed(fn):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[reps // 2]

    ms = timed(lambda: L.lope_copy_stream(src, dst))
    ok = bool(torch.equal(src, dst))
    ms_t = timed(lambda: dst.copy_(src))
    del src, dst
    torch.cuda.empty_cache()
    gbs = lambda t: round(2 * mib * (1 << 20) / (t * 1e-3) / 1e9, 1)
    return {"MiB": mib, "kernel": "lope_copy_stream (16-byte non-temporal)", "ms": round(ms, 4), "GBs": gbs(ms),
            "frac": round(gbs(ms) / PEAK_HBM_GBS, 4), "copied_exactly": ok,
            "torch_copy_ms": round(ms_t, 4), "torch_copy_GBs": gbs(ms_t)}


def measure_workloads(reps=3):
    """The other sweep workloads at full size, each run with lope_iterate's
    default (tuned) kernel and depth: GPoint-updates/s and effective HBM
    bandwidth at 2*sizeof(T) algorithmic bytes per point-update (median of
    reps, HIP events around the whole sweep sequence)."""
    import numpy as np
    import torch

    import paper_1502_03504_amd as L
    import synth

    # (name, inputs, sweeps per pass requested: 0 = the tuned default)
    cases = [("heat3d_7pt_512^3_f32_periodic_1000_sweeps_one_sweep_per_pass",
              lambda: synth.case_heat3d(n=512, dtype=np.float32), 1),
             ("heat3d_7pt_512^3_f32_dirichlet_1000_sweeps",
              lambda: synth.case_heat3d(n=512, dtype=np.float32)._replace(
                  bc=synth.Boundary((synth.DIRICHLET,) * 3, 0.0)), 0),
             ("heat2d_5pt_256^2_f64_dirichlet_100_sweeps", synth.case_heat2d, 0),
             ("heat3d_7pt_256^3_f64_periodic_1000_sweeps", lambda: synth.case_heat3d(n=256, dtype=np.float64), 0),
             ("box9_8192^2_f32_periodic_1000_sweeps", synth.case_box9, 0),
             ("star25_r4_512^3_f32_dirichlet_500_sweeps", synth.case_star25, 0)]
    out = {}
    s = torch.cuda.current_stream()
    for name, make, td in cases:
        case = make()
        a = L.Grid.from_array(case.field, case.h)
        b = a.empty_like()
        pts, esize = int(case.field.size), case.field.dtype.itemsize
        case = case._replace(field=None)
        vid = L.lope_select_variant(a, case.stencil, td, bc=case.bc)
        info = L.lope_variant_info(vid) if vid > 0 else "generic"
        L.lope_iterate(a, b, case.stencil, case.bc, case.steps, tdepth=td)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            L.lope_iterate(a, b, case.stencil, case.bc, case.steps, tdepth=td)
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[reps // 2]
        upd = pts * case.steps / (ms * 1e-3)
        out[name] = {"ms": round(ms, 3), "GPts": round(upd / 1e9, 1),
                     "effective_GBs": round(upd * 2 * esize / 1e9, 1),
                     "frac": round(upd * 2 * esize / 1e9 / PEAK_HBM_GBS, 4), "kernel": info.split()[0]}
        if name.startswith("star25"):
            # both ceilings of one sweep per pass: HBM at 8 algorithmic bytes
            # per point-update; VALU at 25 fmas per point-update on 256 CUs x
            # 64 fp32 lanes per clock x 2.4 GHz (no packed fp32)
            taps = int(np.count_nonzero(case.stencil.coeffs))
            out[name]["ceilings_GPts"] = {"hbm_peak": round(PEAK_HBM_GBS / (2 * esize), 1),
                                          "valu": round(VALU_LANE_OPS / taps / 1e9, 1), "taps": taps}
        log("workload:", name, out[name])
        del a, b
        torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(field, st, bc, sweeps, n, threads=None):
    """The oracle's sweep timed on the host: `sweeps` full-size sweeps on one
    core, and as many again on slabs of planes run by a thread pool (numpy
    releases the GIL inside each slab's arithmetic; each slab carries one
    plane of its neighbours on each side, wrapped periodically, and keeps its
    own planes of the result)."""
    import concurrent.futures

    import numpy as np

    import oracle
    t = time.perf_counter()
    u = field
    for _ in range(sweeps):
        u = oracle.sweep(u, st.coeffs, bc.kinds, 0.0)
    one = time.perf_counter() - t
    threads = threads or max(1, min(16, os.cpu_count() or 1))
    nz = field.shape[0]
    bounds = [(k * nz // threads, (k + 1) * nz // threads) for k in range(threads)]

    def slab(u, z0, z1, out):
        idx = [z % nz for z in range(z0 - 1, z1 + 1)]
        res = oracle.sweep(u[idx], st.coeffs, bc.kinds, 0.0)
        out[z0:z1] = res[1:-1]

    t = time.perf_counter()
    v = field
    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        for _ in range(sweeps):
            w = np.empty_like(v)
            list(ex.map(lambda b: slab(v, b[0], b[1], w), bounds))
            v = w
    many = time.perf_counter() - t
    same = bool(np.array_equal(u, v))
    pts = n ** 3
    return {"value": pts * sweeps / one / 1e9, "unit": "GPoint-updates/s", "cores": 1, "kind": "oracle",
            "sample": "%d full-size sweeps of the %d^3 float32 grid (numpy, float64 arithmetic, single-threaded), "
                      "%.1f s" % (sweeps, n, one),
            "cpu_model": cpu_model(), "cpu_count": os.cpu_count(),
            "all_cores": {"value": pts * sweeps / many / 1e9, "cores": threads,
                          "sample": "the same sweeps on %d z-slabs run by %d threads, %.1f s (result identical "
                                    "to the single-threaded run: %s)" % (threads, threads, many, same)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--tdepth", type=int, default=0, help="sweeps fused per pass (0 = library default)")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--cpu-sweeps", type=int, default=3, help="full-size oracle sweeps timed (0 = skip)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="before timing, run the library's streaming copy over this many MiB (a "
                         "known-size reference for hardware byte counters)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratio measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-grids measurement")
    ap.add_argument("--no-workloads", action="store_true", help="skip the other full-size sweep workloads")
    ap.add_argument("--no-converge", action="store_true", help="skip the convergence-checked iteration")
    ap.add_argument("--no-stages", action="store_true", help="skip the two-stage (Heun) steps")
    ap.add_argument("--reps", type=int, default=3, help="timed repeats of the batch and workload runs")
    ap.add_argument("--no-per-grid", action="store_true",
                    help="skip the one-launch-per-grid comparison of the batched workload")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1502_03504_amd as L
    import synth

    torch.cuda.set_device(0)
    n, sweeps = args.n, args.sweeps
    t0 = time.time()
    case = synth.case_heat3d(n=n, dtype=np.float32, steps=sweeps)
    log("inputs generated in %.1fs" % (time.time() - t0))
    a = L.Grid.from_array(case.field, case.h)
    b = a.empty_like()
    field_cpu = case.field
    del case
    st = synth.heat_star(3, 0.125)
    bc = synth.Boundary(("periodic",) * 3, 0.0)

    vid = args.variant or L.lope_select_variant(a, st, args.tdepth, bc=bc)
    info = L.lope_variant_info(vid) if vid > 0 else "generic"
    td = int(dict(kv.split("=") for kv in info.split()[1:]).get("tdepth", 1)) if vid > 0 else 1
    log("kernel:", info)

    def run():
        if args.variant or args.chunk:
            return L.lope_iterate_tuned(a, b, st, bc, sweeps, variant=vid, chunk=args.chunk)
        return L.lope_iterate(a, b, st, bc, sweeps, tdepth=args.tdepth)

    if args.copy_mb > 0:
        n_el = args.copy_mb * (1 << 20) // 4
        c_src = torch.ones(n_el, dtype=torch.float32, device="cuda")
        c_dst = torch.empty_like(c_src)
        L.lope_copy_stream(c_src, c_dst)
        torch.cuda.synchronize()
        log("reference copy (k_copy16): %d MiB read, %d MiB written" % (args.copy_mb, args.copy_mb))
        del c_src, c_dst

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for k in range(args.steps):
        run()
        log("step %d/%d enqueued" % (k + 1, args.steps))
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    pts = n ** 3
    updates = pts * sweeps * args.steps
    value = updates / (ms * 1e-3) / 1e9
    passes_per_step = -(-sweeps // td)
    launch_s = ms * 1e-3 / (args.steps * passes_per_step)
    alg_bytes_per_launch = 8.0 * pts * td
    achieved = alg_bytes_per_launch / launch_s / 1e9

    converge = None
    if not args.no_converge:
        converge = {}
        scratch = torch.empty(1, dtype=torch.float64, device="cuda")
        for every in (10, 100):
            # tol < 0: never converged, so every run does all sweeps and all checks
            L.lope_iterate_until(a, b, st, bc, every, every, -1.0, scratch=scratch)
            t = time.perf_counter()
            _, done, _ = L.lope_iterate_until(a, b, st, bc, sweeps, every, -1.0, scratch=scratch)
            el = time.perf_counter() - t
            converge["check_every_%d" % every] = {"sweeps": done, "ms": round(el * 1e3, 2),
                                                  "GPts": round(pts * done / el / 1e9, 1),
                                                  "vs_plain": round(pts * done / el / 1e9 / value, 3)}
        log("converge:", converge)

    stages = None
    if not args.no_stages:
        # Heun's method for the same heat problem: v = S u, u' = u/2 + (S/2) v,
        # one fused pass per step, against the same two sweeps as two launches
        half = synth.Stencil(3, 1, 0.5 * st.coeffs)
        nst = 200
        L.lope_iterate_stages(a, b, st, half, 0.5, bc, 2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        L.lope_iterate_stages(a, b, st, half, 0.5, bc, nst)
        e1.record(stream)
        e1.synchronize()
        ms_f = e0.elapsed_time(e1)
        e0.record(stream)
        for _ in range(nst):
            L.lope_iterate(a, b, st, bc, 2, tdepth=1)
        e1.record(stream)
        e1.synchronize()
        ms_u = e0.elapsed_time(e1)
        stages = {"workload": "heun_7pt_%d^3_f32_periodic_%d_steps" % (n, nst), "ms": round(ms_f, 3),
                  "GPts_steps": round(pts * nst / (ms_f * 1e-3) / 1e9, 1),
                  "two_sweeps_ms": round(ms_u, 3), "speedup_vs_two_sweeps": round(ms_u / ms_f, 2)}
        log("stages:", stages)

    adjoint = None
    if not args.no_adjoint:
        del a, b
        torch.cuda.empty_cache()
        adjoint = measure_adjoint()
        log("adjoint:", adjoint)
    batch = None
    if not args.no_batch:
        torch.cuda.empty_cache()
        batch = measure_batch(reps=args.reps, per_grid=not args.no_per_grid)
        log("batch:", batch)
    copy_ref = measure_copy()
    log("copy:", copy_ref)
    workloads = None
    if not args.no_workloads:
        torch.cuda.empty_cache()
        workloads = measure_workloads(reps=args.reps)

    cpu = None
    if args.cpu_sweeps > 0:
        cpu = cpu_baseline(field_cpu, st, bc, args.cpu_sweeps, n)

    out = {
        "metric": "GPoint-updates/s, 3D 7-point heat stencil, 512^3 float32, periodic",
        "value": round(value, 3),
        "unit": "GPoint-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "heat3d_7pt_%d^3_f32_periodic_%d_sweeps" % (n, sweeps), "grid": [n, n, n],
                   "sweeps_per_step": sweeps, "halo": 1, "kernel": info.split()[0], "sweeps_per_pass": td},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(info.split()[0], n, sweeps)},
        "cpu_baseline": cpu,
        "converge": converge,
        "stages": stages,
        "adjoint_forward": adjoint,
        "batch": batch,
        "copy_reference": copy_ref,
        "workloads": workloads,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
