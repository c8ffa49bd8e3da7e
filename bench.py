"""Throughput of the BSSN RK4 step on one MI355X.

One step = one classic RK4 step (4 right-hand sides + stage combinations) of
the whole patch.  Default workload: 128^3 interior points, 3 ghost zones,
4th-order upwinded finite differences, Kreiss-Oliger r=3, two-puncture
Brill-Lindquist data (synthetic, closed form), static ghosts, dt = h/4.

Prints one JSON line: grid-point updates per second (interior points x steps
/ GPU time), the roofline of the dominant kernel (the stage-2/3 kernel,
timed live with HIP events on the launch stream), and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2, choices=[2, 3])
    ap.add_argument("--n", type=int, default=0, help="override the interior edge (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}); the multi-GPU "
              "halo exchange is a design, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1307_6488_amd import chemora as C
    from paper_1307_6488_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = I.workload(args.workload, n_override=args.n or None)
    u0 = w.make_state()
    npts = w.grid.npoints
    P = C.Patch(w.params, w.grid, u0, device=dev)
    scratch = P.scratch()
    stream = torch.cuda.current_stream()
    sp = scratch.data_ptr()

    def step():
        for s in (1, 2, 3, 4):
            C.chemora_rk4_stage(P.params, P.patch, s, w.dt, sp, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for k in range(K):
        e = ev[k]
        e[0].record(stream)
        for s in (1, 2, 3, 4):
            C.chemora_rk4_stage(P.params, P.patch, s, w.dt, sp, stream)
            e[s].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    stage_ms = np.array([[ev[k][s - 1].elapsed_time(ev[k][s]) for s in (1, 2, 3, 4)] for k in range(K)])
    bad = C.chemora_check_finite(P.params, P.patch)
    if bad:
        print(f"warning: {bad} non-finite values after the run", file=sys.stderr)

    ms_per_step = total_ms / K
    value = npts * K / (total_ms * 1e-3)
    # dominant kernel: stages 2 and 3 (same kernel), 5 state transfers of 24 FP64 GFs per point
    t23 = float(np.mean(stage_ms[:, 1:3])) * 1e-3
    bytes23 = 5 * 24 * 8 * npts
    achieved = bytes23 / t23 / 1e9
    out = {
        "metric": "BSSN grid-point updates/s (one point advanced one full RK4 step), FP64",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (closed-form Brill-Lindquist two-puncture data)",
        "config": {
            "workload": w.name,
            "interior": list(w.grid.n),
            "ghost": w.params.ghost,
            "fd_order": w.params.fd_order,
            "upwind": bool(w.params.upwind),
            "ko_radius": w.params.ko_radius,
            "dt": w.dt,
            "boundary": "static",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "stage_kernel (RK4 stages 2/3)",
            "bytes_per_point": 960,
            "avg_launch_ms": t23 * 1e3,
        },
        "step_roofline": {
            "algorithmic_bytes_per_update": 3072,
            "hbm_frac": value * 3072 / (HBM_PEAK_GBS * 1e9),
        },
        "stage_ms": [float(x) for x in stage_ms.mean(axis=0)],
        "host_wall_s": wall,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, u0)
    print(json.dumps(out), flush=True)


def cpu_baseline(w, u0):
    """The CPU oracle (plain C++, OpenMP) timed on this host: one RK4 step of
    the same workload at full size."""
    root = os.path.dirname(os.path.abspath(__file__))
    if root not in sys.path:
        sys.path.insert(0, root)
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    t = time.perf_counter()
    oracle.rk4(w.params, w.grid, u0, w.dt, 1, nthreads=threads)
    dt = time.perf_counter() - t
    return {"value": w.grid.npoints / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"1 RK4 step of the same {w.grid.n[0]}x{w.grid.n[1]}x{w.grid.n[2]} workload "
                      f"({w.grid.npoints} point updates), {dt:.1f} s wall"}


if __name__ == "__main__":
    main()
