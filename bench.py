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
METRIC = "BSSN grid-point updates/s on 1 MI355X: FP64 vs batched vs split-FP32 (+% roofline)"

# Floating-point operations of one right-hand-side evaluation per point, as
# counted by the CPU oracle's counting scalar (+, -, *, / each one; no FMA):
# order 4 upwind / KO r=3 and order 8 upwind / KO r=5.  The RK4 combination
# adds 14 per grid function per step (2+2, 2+2, 2+2, 2).
RHS_FLOPS = {4: 6931, 8: 11821}
RK4_FLOPS = 24 * 14

# HBM bytes per launch of the stage-2/3 kernel, from rocprofv3 counter runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled by what the same
# counters read for a plain 2 GiB device copy (FETCH_SIZE reads half the
# bytes copied: x2.0; WRITE_SIZE reads them exactly: x1.0).  They hold only
# for the kernel sources and tile variant they were taken with (one record
# per tile variant the tuner picks on that workload: their times are within
# a few per cent, so its choice varies between runs); otherwise the bench
# reports traffic as null.
MEASURED_TRAFFIC = {
    "brill-lindquist-128^3-o4-upwind": {
        "32x8x2": {"sources_sha256": "79e7cda7a20ddb7ec670200d3c432ad267119d3662df178a315ef7f3d9e112b1",
            "fetch_kib": 1.0676e6, "write_kib": 8.1155e5, "fetch_scale": 2.0, "write_scale": 1.0},
        "32x4x4": {"sources_sha256": "79e7cda7a20ddb7ec670200d3c432ad267119d3662df178a315ef7f3d9e112b1",
            "fetch_kib": 1.2043e6, "write_kib": 8.1145e5, "fetch_scale": 2.0, "write_scale": 1.0},
        "32x16": {"sources_sha256": "79e7cda7a20ddb7ec670200d3c432ad267119d3662df178a315ef7f3d9e112b1",
            "fetch_kib": 1.1582e6, "write_kib": 8.1198e5, "fetch_scale": 2.0, "write_scale": 1.0},
    },
    "brill-lindquist-pert-192^3-o8-upwind": {
        "32x8": {"sources_sha256": "79e7cda7a20ddb7ec670200d3c432ad267119d3662df178a315ef7f3d9e112b1",
            "fetch_kib": 5.7693e6, "write_kib": 2.8619e6, "fetch_scale": 2.0, "write_scale": 1.0},
    },
}
KERNEL_SOURCES = ["stage_kernel.hpp", "stage_common.hpp", "fd_ops.hpp", "stage_o4.hip", "stage_o8.hip"]


def tile_name(C, variant):
    """A tile variant as 'TXxTY' (one plane) or 'TXxTYxTZ'."""
    tx, ty = C.chemora_tile_variant_shape(variant)
    tz = C.chemora_tile_variant_depth(variant)
    return f"{tx}x{ty}" + (f"x{tz}" if tz > 1 else "")


def set_tile(C, P, name):
    """Select the tile variant called `name` for the class of patch P."""
    v = 0
    while True:
        try:
            if tile_name(C, v) == name:
                C.chemora_set_tile_variant(P.params, P.patch, v)
                return v
        except C.ChemoraError:   # past the last variant id
            raise SystemExit(f"no tile variant {name}")
        v += 1


def kernel_sources_sha256():
    import hashlib
    root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1307_6488_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, tile):
    m = MEASURED_TRAFFIC.get(workload, {}).get(tile)
    if m is None or m["sources_sha256"] != kernel_sources_sha256():
        return None
    return (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2, choices=[2, 3])
    ap.add_argument("--n", type=int, default=0, help="override the interior edge (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="run the untuned default tile variant")
    ap.add_argument("--tile", default="", help="run the main workload with this tile variant (e.g. 32x16, "
                    "32x8x2) instead of the tuner's choice: counter runs per variant")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-patch batched form")
    ap.add_argument("--no-split", action="store_true", help="skip the 256^3 split-precision comparison")
    ap.add_argument("--no-rk3", action="store_true", help="skip the third-order Runge-Kutta form")
    ap.add_argument("--no-order8", action="store_true", help="skip the 192^3 order-8 workload")
    ap.add_argument("--split-steps", type=int, default=100, help="RK4 steps of the split-precision comparison")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters to bytes)")
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
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "launches": 3}), flush=True)
        return
    w = I.workload(args.workload, n_override=args.n or None)
    u0 = w.make_state()
    npts = w.grid.npoints
    P = C.Patch(w.params, w.grid, u0, device=dev)
    scratch = P.scratch()
    stream = torch.cuda.current_stream()
    sp = scratch.data_ptr()
    # the autotuner picks the tile variant of this patch's class (outside the
    # timed region; it times stage-2 launches of this patch)
    if args.tile:
        variant = set_tile(C, P, args.tile)
    else:
        variant = C.chemora_tile_variant(P.params, P.patch) if args.no_tune else \
            C.chemora_tune(P.params, P.patch, sp, None, stream)
    tile = tile_name(C, variant)

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
    # spread: 5 more repetitions of the same K steps (reported beside value)
    reps = []
    for _ in range(5):
        r0 = torch.cuda.Event(enable_timing=True)
        r1 = torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        for _k in range(K):
            step()
        r1.record(stream)
        torch.cuda.synchronize()
        reps.append(r0.elapsed_time(r1) / K)
    bad = C.chemora_check_finite(P.params, P.patch)
    if bad:
        print(f"warning: {bad} non-finite values after the run", file=sys.stderr)

    ms_per_step = total_ms / K
    value = npts * K / (total_ms * 1e-3)
    # dominant kernel: stages 2 and 3 (same kernel), 5 state transfers of 24 FP64 GFs per point
    t23 = float(np.mean(stage_ms[:, 1:3])) * 1e-3
    bytes23 = 5 * 24 * 8 * npts
    achieved = bytes23 / t23 / 1e9
    flops_update = 4 * RHS_FLOPS[w.params.fd_order] + RK4_FLOPS
    traffic = measured_traffic(w.name, tile)
    out = {
        "metric": METRIC,
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
            "tile": tile,
            "tuned": not args.no_tune,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "stage_kernel (RK4 stages 2/3)",
            "bytes_per_point": 960,
            "avg_launch_ms": t23 * 1e3,
        },
        "step_roofline": {
            "algorithmic_bytes_per_update": 3072,
            "hbm_frac": value * 3072 / (HBM_PEAK_GBS * 1e9),
            "flops_per_update": flops_update,
            "fp64_frac": value * flops_update / (FP64_PEAK_TFLOPS * 1e12),
            "stage23_traffic_over_algorithmic": None if traffic is None else traffic / bytes23,
        },
        "stage_ms": [float(x) for x in stage_ms.mean(axis=0)],
        "repeat_ms_per_step": {"reps": len(reps), "steps_each": K, "median": float(np.median(reps)),
                               "min": float(np.min(reps)), "max": float(np.max(reps))},
        "host_wall_s": wall,
    }
    out["roofline"]["achievable_copy_gbs"] = copy_bandwidth(torch)
    out["single_patch_plan"] = single_patch_plan_form(C, torch, w, u0, K, args.warmup)
    if not args.no_rk3:
        out["rk3"] = rk3_form(C, I, torch, w, u0)
        out["constraints"] = constraints_form(C, torch, P)
    del P, scratch
    torch.cuda.empty_cache()
    if not args.no_order8 and args.workload != 3:
        out["order8"] = order8_form(C, I, torch, args.no_tune)
    if not args.no_batched:
        out["batched"] = batched_form(C, I, torch, args.no_tune)
    if not args.no_split:
        out["split"] = split_form(C, I, torch, args.no_tune, steps=args.split_steps)
    if not args.no_rk3:
        out["bbh_share"] = bbh_share_form(C, I, torch, args.no_tune)
    if not args.no_batched:
        out["synced"] = synced_form(C, I, torch)
    out["boundary_and_psi4"] = boundary_psi4_form(C, I, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, u0, I)
    print(json.dumps(out), flush=True)


def single_patch_plan_form(C, torch, w, u0, steps, warmup):
    """The same patch and steps through a one-patch plan: the RK4 step
    replayed as a HIP graph, the static ghosts of the stage buffers prepared
    once at plan creation instead of at every step (chemora_rk4_step cannot
    assume its scratch kept them)."""
    B = C.Batch(w.params, [w.grid], [u0], courant=w.dt / w.grid.h)
    B.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    B.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    B.close()
    del B
    torch.cuda.empty_cache()
    return {"ms_per_step": ms, "value": w.grid.npoints / (ms * 1e-3), "unit": "updates/s",
            "calls": "chemora_batch_step on a plan of this one patch (graph replays)"}


def copy_bandwidth(torch, mib=2048, reps=5):
    """The achievable HBM bandwidth: a plain device-to-device copy of `mib` MiB
    (read + write bytes / time, best of `reps`)."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (best * 1e-3) / 1e9


def stage_timed_steps(C, torch, P, dt, sp, K):
    """K RK4 steps driven stage by stage with HIP events on the launch stream:
    (ms per step, mean stage-2/3 launch ms)."""
    import numpy as np
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(K)]
    torch.cuda.synchronize()
    for k in range(K):
        ev[k][0].record(stream)
        for s in (1, 2, 3, 4):
            C.chemora_rk4_stage(P.params, P.patch, s, dt, sp, stream)
            ev[k][s].record(stream)
    torch.cuda.synchronize()
    st = np.array([[ev[k][s - 1].elapsed_time(ev[k][s]) for s in (1, 2, 3, 4)] for k in range(K)])
    return float(st.sum(axis=1).mean()), float(st[:, 1:3].mean())


def order8_form(C, I, torch, no_tune, steps=5, warmup=1):
    """The 8th-order workload (192^3, 5 ghosts, partially upwinded order-8
    stencils, Kreiss-Oliger r=5, perturbed Brill-Lindquist data): rate and
    the stage-2/3 kernel's HBM fraction at 960 algorithmic bytes per point."""
    w = I.workload(3)
    P = C.Patch(w.params, w.grid, w.make_state())
    sp = P.scratch().data_ptr()
    stream = torch.cuda.current_stream()
    variant = C.chemora_tile_variant(P.params, P.patch) if no_tune else C.chemora_tune(P.params, P.patch, sp, None,
                                                                                         stream)
    tile = tile_name(C, variant)
    stage_timed_steps(C, torch, P, w.dt, sp, warmup)
    ms, t23 = stage_timed_steps(C, torch, P, w.dt, sp, steps)
    npts = w.grid.npoints
    gbs = 960 * npts / (t23 * 1e-3) / 1e9
    traffic = measured_traffic(w.name, tile)
    del P
    torch.cuda.empty_cache()
    return {"workload": w.name, "interior": list(w.grid.n), "fd_order": 8, "ghost": w.params.ghost,
            "steps": steps, "ms_per_step": ms, "value": npts / (ms * 1e-3), "unit": "updates/s",
            "tile": tile,
            "stage23": {"avg_launch_ms": t23, "achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                        "traffic": traffic},
            "step_hbm_frac": npts / (ms * 1e-3) * 3072 / (HBM_PEAK_GBS * 1e9),
            "fp64_frac": npts / (ms * 1e-3) * (4 * RHS_FLOPS[8] + RK4_FLOPS) / (FP64_PEAK_TFLOPS * 1e12)}


def batched_form(C, I, torch, no_tune, steps=10, warmup=2):
    """The batched form: 64 patches of 24-96 points per edge (h = 1/8 or
    1/16, Brill-Lindquist data on each patch's own domain, order 4 upwind,
    static ghosts, dt = h/4 per patch), one plan, one captured RK4 step per
    graph launch; the plan tunes the tile variant of every size class."""
    grids = I.patch_list()
    params = I.workload(2).params
    states = [I.brill_lindquist(g) for g in grids]
    npts = sum(g.npoints for g in grids)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def plan_ms(tune_cache_path, dispatch=C.DISPATCH_AUTO):
        B = C.Batch(params, grids, states, 0.25, tune_cache_path=tune_cache_path, dispatch=dispatch)
        B.step(warmup)
        torch.cuda.synchronize()
        e0.record()
        B.step(steps)
        e1.record()
        torch.cuda.synchronize()
        variants = sorted(set(B.variants()))
        chosen = B.dispatch()
        B.close()
        del B
        torch.cuda.empty_cache()
        return e0.elapsed_time(e1) / steps, variants, chosen
    # untuned first (no size class of these patches has a table entry yet:
    # every patch runs the default 32x8 tile), then the tuned plan
    ms_untuned = None if no_tune else plan_ms(None)[0]
    ms, variants, chosen = plan_ms(None if no_tune else _tune_cache())
    # the same tuned plan with each dispatch forced
    ms_pers = plan_ms(None if no_tune else _tune_cache(), C.DISPATCH_PERSISTENT)[0]
    ms_tiles = plan_ms(None if no_tune else _tune_cache(), C.DISPATCH_PER_TILE)[0]
    # the same patches and data stepped one chemora_rk4_step call each, with
    # the tile variants the plan's tuner recorded for their classes
    Ps = [C.Patch(params, g, s) for g, s in zip(grids, states)]
    stream = torch.cuda.current_stream()
    sps = [P.scratch().data_ptr() for P in Ps]

    def per_patch(n):
        for _ in range(n):
            for P, g, sp in zip(Ps, grids, sps):
                C.chemora_rk4_step(P.params, P.patch, 0.25 * g.h, sp, stream)
    per_patch(warmup)
    torch.cuda.synchronize()
    e0.record(stream)
    per_patch(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_pp = e0.elapsed_time(e1) / steps
    del Ps
    torch.cuda.empty_cache()
    # the same plan with the third-order SSP Runge-Kutta step captured
    B3 = C.Batch(params, grids, states, 0.25, tune_cache_path=None if no_tune else _tune_cache(), integrator="rk3")
    B3.step(warmup)
    torch.cuda.synchronize()
    e0.record()
    B3.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms3 = e0.elapsed_time(e1) / steps
    B3.close()
    return {"workload": "64 patches, 24-96 points per edge, order 4 upwind (batched plan)", "patches": len(grids),
            "points": npts, "steps": steps, "ms_per_step": ms, "value": npts / (ms * 1e-3),
            "unit": "updates/s", "tile_variants": [tile_name(C, v) for v in variants],
            "dispatch": ("persistent" if chosen == C.DISPATCH_PERSISTENT else "per-tile")
            + " (the plan's timed choice)",
            "persistent_dispatch": {"ms_per_step": ms_pers,
                                    "launch": "resident work-groups pulling tiles from per-XCD queues"},
            "per_tile_dispatch": {"ms_per_step": ms_tiles, "launch": "one work-group per tile"},
            "hbm_frac": npts / (ms * 1e-3) * 3072 / (HBM_PEAK_GBS * 1e9),
            "per_patch": {"ms_per_step": ms_pp, "value": npts / (ms_pp * 1e-3),
                          "calls": "one chemora_rk4_step per patch and step, same tile variants"},
            "speedup_vs_per_patch": ms_pp / ms,
            "untuned": None if ms_untuned is None else {
                "ms_per_step": ms_untuned, "tile_variants": ["32x8"], "tuned_speedup": ms_untuned / ms},
            "rk3": {"ms_per_step": ms3, "value": npts / (ms3 * 1e-3)}}


def constraints_form(C, torch, P, calls=20):
    """Algebraic-constraint enforcement (det gt = 1, gt^ij At_ij = 0) on the
    evolved 128^3 state: one pointwise launch reading and writing the 12
    conformal components, 192 algorithmic bytes per point; and the
    momentum-constraint diagnostic on the same state."""
    stream = torch.cuda.current_stream()
    C.chemora_enforce_constraints(P.params, P.patch, stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(calls):
        C.chemora_enforce_constraints(P.params, P.patch, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / calls
    npts = P.patch.n[0] * P.patch.n[1] * P.patch.n[2]
    gbs = npts * 192 / (ms * 1e-3) / 1e9
    # the momentum-constraint diagnostic on the same state: reads chi, gt, K,
    # At (14 grid functions, neighbours from L2) and writes 3: 136 B per point
    M = torch.empty(3 * P.grid.sf, dtype=torch.float64, device=P.u.device)
    C.chemora_momentum_constraint(P.params, P.patch, M.data_ptr(), stream)
    e0.record(stream)
    for _ in range(calls):
        C.chemora_momentum_constraint(P.params, P.patch, M.data_ptr(), stream)
    e1.record(stream)
    torch.cuda.synchronize()
    msm = e0.elapsed_time(e1) / calls
    return {"kernel": "enforce_kernel", "calls": calls, "ms_per_call": ms, "bytes_per_point": 192,
            "achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "momentum": {"kernel": "momentum_kernel", "ms_per_call": msm, "bytes_per_point": 136,
                         "achieved_gbs": npts * 136 / (msm * 1e-3) / 1e9}}


def rk3_form(C, I, torch, w, u0, steps=20, warmup=2):
    """The paper's integrator: third-order SSP Runge-Kutta steps (3 stage
    launches, 8 state transfers per point) on the same workload and data,
    tile variant as tuned for it; a step advances by the same dt."""
    P = C.Patch(w.params, w.grid, u0)
    P.rk3_step(w.dt, warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    P.rk3_step(w.dt, steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    npts = w.grid.npoints
    return {"workload": w.name, "integrator": "SSP RK3 (Shu-Osher)", "steps": steps, "ms_per_step": ms,
            "value": npts / (ms * 1e-3), "unit": "updates/s", "algorithmic_bytes_per_update": 8 * 24 * 8,
            "hbm_frac": npts / (ms * 1e-3) * 8 * 24 * 8 / (HBM_PEAK_GBS * 1e9)}


def split_form(C, I, torch, no_tune, steps=100, warmup=2):
    """Split precision (FP32 stencil combinations and algebra, FP64 state,
    RK combination and near-puncture chi terms, chi_split = 0.1) against FP64
    on the same 256^3 Brill-Lindquist data: throughput of each over `steps`
    RK4 steps (after `warmup` untimed ones, both runs advancing the same
    total), then on the 64^3 subsample i, j, k in {2, 6, ..., 254} the
    max-norm-normalised difference per GF of split against FP64 and the RMS
    of the Hamiltonian constraint of each state.  The FP64 reference is the
    GPU FP64 path (the oracle would need hours for 100 steps at 256^3; the
    parity tests hold the GPU FP64 path to the oracle)."""
    import numpy as np
    w = I.workload(5)
    u0 = w.make_state()
    g = w.grid.ghost
    sub = np.arange(2, w.grid.n[0], 4)
    res, st, ham = {}, {}, {}
    for name, prec in (("fp64", I.PREC_FP64), ("split", I.PREC_SPLIT)):
        p = I.Params(**vars(w.params))
        p.precision = prec
        P = C.Patch(p, w.grid, u0)
        stream = torch.cuda.current_stream()
        variant = C.chemora_tile_variant(P.params, P.patch) if no_tune else P.tune(None, stream)
        P.rk4_step(w.dt, warmup)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.rk4_step(w.dt, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = {"ms_per_step": ms, "value": w.grid.npoints / (ms * 1e-3), "tile": tile_name(C, variant)}
        ix = torch.as_tensor(g + sub, device=P.u.device)
        st[name] = P.u.index_select(1, ix).index_select(2, ix).index_select(3, ix).cpu().numpy()
        # H of the final state, evaluated in FP64 for both runs
        hp = I.Params(**vars(w.params))
        hp.precision = I.PREC_FP64
        H = C.Patch(hp, w.grid, P.u).hamiltonian()
        ham[name] = H.index_select(0, ix - g).index_select(1, ix - g).index_select(2, ix - g).cpu().numpy()
        del P, H
        torch.cuda.empty_cache()
    scale = np.max(np.abs(st["fp64"]), axis=(1, 2, 3))
    err = np.max(np.abs(st["split"] - st["fp64"]), axis=(1, 2, 3)) / np.where(scale > 0, scale, 1.0)
    worst = int(np.argmax(err))
    h64 = float(np.sqrt(np.mean(ham["fp64"] ** 2)))
    hsp = float(np.sqrt(np.mean(ham["split"] ** 2)))
    return {"workload": w.name, "interior": list(w.grid.n), "chi_split": w.params.chi_split,
            "steps": warmup + steps, "timed_steps": steps, "unit": "updates/s", "fp64": res["fp64"],
            "split": res["split"], "speedup": res["fp64"]["ms_per_step"] / res["split"]["ms_per_step"],
            "subsample": "64^3 points i,j,k in {2,6,...,254}",
            "reference": "GPU FP64 run on the same data and steps",
            "max_err_vs_fp64": float(err[worst]), "worst_gf": I.GF_NAMES[worst],
            "err_per_gf": {n: float(e) for n, e in zip(I.GF_NAMES, err)},
            "h_rms_fp64": h64, "h_rms_split": hsp, "h_rms_ratio": hsp / h64 if h64 > 0 else None}


def bbh_share_form(C, I, torch, no_tune, steps=20, warmup=2):
    """One GPU's share of the paper's production run: 90^3 interior points,
    5 ghost zones, 8th-order partially upwinded stencils, third-order
    Runge-Kutta (3 stage launches, 8 state transfers = 1536 algorithmic
    bytes per update), the share holding a puncture."""
    w = I.bbh_share()
    P = C.Patch(w.params, w.grid, w.make_state())
    stream = torch.cuda.current_stream()
    variant = C.chemora_tile_variant(P.params, P.patch) if no_tune else P.tune(None, stream)
    P.rk3_step(w.dt, warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    P.rk3_step(w.dt, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    npts = w.grid.npoints
    tile = tile_name(C, variant)
    del P
    torch.cuda.empty_cache()
    return {"workload": w.name, "interior": list(w.grid.n), "ghost": w.params.ghost, "fd_order": 8,
            "integrator": "SSP RK3", "steps": steps, "ms_per_step": ms, "value": npts / (ms * 1e-3),
            "unit": "updates/s", "tile": tile, "algorithmic_bytes_per_update": 1536,
            "hbm_frac": npts / (ms * 1e-3) * 1536 / (HBM_PEAK_GBS * 1e9)}


def _hierarchy(I, n0=48, nf=48, ghost=3):
    """A two-level grid hierarchy: the coarse level (h = 1/4) as a 2 x 2 x 2
    block split of a (2 n0)^3 grid, and one refined patch (h = 1/8) of nf^3
    points round each puncture of the Brill-Lindquist data (punctures at
    x = +-3)."""
    hc, hf = 0.25, 0.125
    L = 2 * n0 * hc
    o = -L / 2 + hc / 2
    grids = []
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                grids.append(I.Grid((n0, n0, n0), ghost, hc, (o + bx * n0 * hc, o + by * n0 * hc, o + bz * n0 * hc)))
    for cx in (3.0, -3.0):
        # fine origin on the fine lattice through the coarse origin
        k = round((cx - (nf - 1) * hf / 2 - o) / hf)
        ky = round((0.0 - (nf - 1) * hf / 2 - o) / hf)
        grids.append(I.Grid((nf, nf, nf), ghost, hf, (o + k * hf, o + ky * hf, o + ky * hf)))
    return grids


def synced_form(C, I, torch, steps=10, warmup=2):
    """A synchronised plan over a two-level hierarchy (8 coarse blocks of
    48^3 at h = 1/4, two refined 48^3 patches at h = 1/8 round the punctures;
    order 4 upwind, static outer ghosts, one dt = h_fine / 4): ghost exchange,
    prolongation after every RK4 stage and restriction after every step, all
    inside the captured graph.  Reported beside the same patches as an
    independent plan (no exchange) to show the synchronisation's cost."""
    grids = _hierarchy(I)
    params = I.workload(2).params
    states = [I.brill_lindquist(g) for g in grids]
    npts = sum(g.npoints for g in grids)
    dt = 0.25 * 0.125
    out = {"workload": "two-level hierarchy: 8 x 48^3 (h 1/4) + 2 x 48^3 (h 1/8), order 4 upwind, RK4",
           "patches": len(grids), "points": npts, "steps": steps}
    for name, kw in (("synced", {"synced_dt": dt}), ("independent", {"courant": dt / 0.125})):
        B = C.Batch(params, grids, states, **kw)
        B.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        B.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        B.close()
        out[name] = {"ms_per_step": ms, "value": npts / (ms * 1e-3)}
    out["unit"] = "updates/s"
    out["sync_overhead"] = out["synced"]["ms_per_step"] / out["independent"]["ms_per_step"] - 1.0
    torch.cuda.empty_cache()
    return out


def boundary_psi4_form(C, I, torch, reps=10):
    """The 128^3 workload's RK4 step with the radiative outer boundary (one
    extra launch per stage evolving the ghost points) against static ghosts,
    and the Psi4 diagnostic on the same state (ms per call)."""
    w = I.workload(2)
    u0 = w.make_state()
    out = {"workload": w.name}
    for name, bc in (("static", I.BC_STATIC), ("radiative", I.BC_RADIATIVE)):
        p = I.Params(**vars(w.params))
        p.bc = bc
        P = C.Patch(p, w.grid, u0)
        P.rk4_step(w.dt, 1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        P.rk4_step(w.dt, reps)
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"ms_per_step": e0.elapsed_time(e1) / reps}
        if bc == I.BC_STATIC:
            P.psi4()
            e0.record()
            for _ in range(reps):
                P.psi4()
            e1.record()
            torch.cuda.synchronize()
            out["psi4_ms_per_call"] = e0.elapsed_time(e1) / reps
        del P
        torch.cuda.empty_cache()
    out["radiative_overhead"] = out["radiative"]["ms_per_step"] / out["static"]["ms_per_step"] - 1.0
    return out


def _tune_cache():
    import tempfile
    return os.path.join(tempfile.gettempdir(), f"chemora_tiles_{os.getpid()}.json")


def cpu_baseline(w, u0, I, min_seconds=10.0, max_steps=20):
    """The CPU oracle (plain C++, OpenMP) timed on this host.  All host
    threads: RK4 steps of the same full-size workload; the first step (which
    also pages the buffers in) is timed alone and sets how many steps fill
    about min_seconds, and those are timed in one call whose step loop is
    clocked inside the oracle, without the allocation of its stage vectors.
    One thread: a 32^3 sample of the same workload (same data recipe,
    parameters and dt) for a per-core rate."""
    root = os.path.dirname(os.path.abspath(__file__))
    if root not in sys.path:
        sys.path.insert(0, root)
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    u1, t1 = oracle.rk4_timed(w.params, w.grid, u0, w.dt, 1, nthreads=threads)
    steps = int(max(1, min(max_steps, round(min_seconds / max(t1, 1e-3)))))
    _, t = oracle.rk4_timed(w.params, w.grid, u1, w.dt, steps, nthreads=threads)
    one = I.workload(2, n_override=32)
    _, t_one = oracle.rk4_timed(one.params, one.grid, one.make_state(), one.dt, 1, nthreads=1)
    return {"value": w.grid.npoints * steps / t, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} RK4 steps of the same {w.grid.n[0]}x{w.grid.n[1]}x{w.grid.n[2]} workload "
                      f"({w.grid.npoints * steps} point updates) in {t:.1f} s of step loop, after one "
                      f"step ({t1:.1f} s) that sizes the sample",
            "one_thread": {"value": one.grid.npoints / t_one, "unit": "updates/s", "cores": 1,
                           "sample": f"1 RK4 step of the 32^3 Brill-Lindquist workload, {t_one:.2f} s"}}


if __name__ == "__main__":
    main()
