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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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
    ap.add_argument("--cpu-sweeps", type=int, default=2, help="full-size oracle sweeps timed (0 = skip)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
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

    vid = args.variant or L.lope_select_variant(a, st, args.tdepth)
    info = L.lope_variant_info(vid) if vid > 0 else "generic"
    td = int(dict(kv.split("=") for kv in info.split()[1:]).get("tdepth", 1)) if vid > 0 else 1
    log("kernel:", info)

    def run():
        if args.variant or args.chunk:
            return L.lope_iterate_tuned(a, b, st, bc, sweeps, variant=vid, chunk=args.chunk)
        return L.lope_iterate(a, b, st, bc, sweeps, tdepth=args.tdepth)

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

    cpu = None
    if args.cpu_sweeps > 0:
        import oracle
        t = time.perf_counter()
        u = field_cpu
        for _ in range(args.cpu_sweeps):
            u = oracle.sweep(u, st.coeffs, bc.kinds, 0.0)
        el = time.perf_counter() - t
        cpu = {"value": pts * args.cpu_sweeps / el / 1e9, "unit": "GPoint-updates/s", "cores": 1,
               "kind": "oracle",
               "sample": "%d full-size sweeps of the %d^3 float32 grid (numpy, float64 arithmetic, "
                         "single-threaded), %.1f s" % (args.cpu_sweeps, n, el)}

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
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
