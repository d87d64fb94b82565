"""Benchmark of the quantum-walk step engine on one MI355X.

Workload: continuous-time walk on the periodic 1024 x 1024 grid (N = 2^20
vertices, 4 * 2^20 arcs), H = -gamma A with gamma = 0.25, Taylor order 20,
dt = 0.1, started on the single vertex (512, 512).  One bench step is one
pass of the hot path: 1000 time steps (20 Horner stages each) plus the FP64
probability readout, on a state already resident in HBM.  The complex64 path
(FP64 reductions) is the reported value; the complex128 path is timed beside
it, and both are checked against the closed form (product of cycle Bessel
sums) at the end.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
L_SIDE = 1024
GAMMA = 0.25
DT = 0.1
K_ORDER = 20
STEPS_PER_PASS = 1000
METRIC = "arc-steps/s (c64 batched vs c128 plain, L2 err<=1e-4); p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--steps-per-pass", type=int, default=STEPS_PER_PASS,
                    help="time steps per pass (profiling runs shorten it; rates are per arc-step)")
    ap.add_argument("--dtypes", default="c64,c128")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    return ap.parse_args()


def copy_probe(mib):
    import torch
    n = mib * 2**20 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n * 8, "launches": 5}), flush=True)


def timed_passes(plan, psi, steps, warmup, spp):
    import torch
    for _ in range(warmup):
        plan.evolve(psi, spp, readout=True)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(steps):
        out = plan.evolve(psi, spp, readout=True)
        evs[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    return wall, per, out


def stage_launch_ms(plan, psi, reps=20):
    """Average duration of one Horner-stage launch: HIP events around
    single-step evolves (20 stage launches each) on the launch stream."""
    import torch
    plan.evolve(psi, 1)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.evolve(psi, 1)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / (reps * K_ORDER)


def pct(sorted_vals, q):
    if not sorted_vals:
        return None
    i = min(len(sorted_vals) - 1, max(0, int(math.ceil(q / 100.0 * len(sorted_vals))) - 1))
    return sorted_vals[i]


def cpu_baseline(g, v0, seconds):
    import numpy as np
    import oracle
    from paper_2406_08186_amd import inputs as I
    psi = I.ket_vertex(g.n, v0)
    t0 = time.perf_counter()
    psi = oracle.ctqw_evolve(g.row_ptr, g.col, psi, 1, gamma=GAMMA, dt=DT, K=K_ORDER)
    t1 = time.perf_counter() - t0
    n_more = max(1, int(seconds / max(t1, 1e-6)) - 1)
    t0 = time.perf_counter()
    psi = oracle.ctqw_evolve(g.row_ptr, g.col, psi, n_more, gamma=GAMMA, dt=DT, K=K_ORDER)
    el = time.perf_counter() - t0
    return {"value": g.n_arcs * n_more / el, "unit": "arc-steps/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{n_more} of the {STEPS_PER_PASS} time steps of one pass on the same "
                      f"{L_SIDE}x{L_SIDE} grid (FP64 power-form Taylor, K={K_ORDER})",
            "seconds": el}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py runs on one GPU only: the walk engine has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    spp = args.steps_per_pass
    dtypes = args.dtypes.split(",")
    import numpy as np
    import torch

    from oracle import closed_forms as cf
    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Plan

    g = I.torus(L_SIDE, L_SIDE)
    v0 = (L_SIDE // 2) * L_SIDE + L_SIDE // 2
    psi0 = I.ket_vertex(g.n, v0)
    res = {}
    for dtype in dtypes:
        pl = Plan(g, "ctqw", dtype=dtype, gamma=GAMMA, dt=DT, taylor_order=K_ORDER)
        psi = pl.state(psi0)
        wall, per, (p, norm, _) = timed_passes(pl, psi, args.steps, args.warmup, spp)
        total_steps = (args.steps + args.warmup) * spp
        state = psi.cpu().numpy().astype(np.complex128)
        launch_ms = stage_launch_ms(pl, pl.state(psi0))
        es = 8 if dtype == "c64" else 16
        bytes_per_launch = 3 * es * g.n  # read y, read psi, write y' (gathers ideally cached)
        res[dtype] = dict(plan=pl, wall=wall, per=per, norm=float(norm), state=state,
                          total_steps=total_steps, launch_ms=launch_ms,
                          bytes_per_launch=bytes_per_launch, structure=pl.structure)
        del psi
    t_final = res[dtypes[0]]["total_steps"] * DT
    ref1 = cf.cycle_ctqw(L_SIDE, GAMMA, t_final, L_SIDE // 2)
    ref = np.outer(ref1, ref1).reshape(-1)
    for r in res.values():
        r["l2"] = float(np.linalg.norm(r["state"] - ref))
    if "c64" not in res or "c128" not in res:
        r = res[dtypes[0]]
        print(json.dumps({"dtype": dtypes[0], "steps_per_pass": spp, "ms_per_step": r["wall"] / args.steps * 1e3,
                          "stage_launch_ms": r["launch_ms"], "l2_vs_closed_form": r["l2"]}), flush=True)
        return
    l2_64, l2_128 = res["c64"]["l2"], res["c128"]["l2"]
    l2_64_128 = float(np.linalg.norm(res["c64"]["state"] - res["c128"]["state"]))

    def rate(r):
        return g.n_arcs * spp * args.steps / r["wall"]

    r64, r128 = res["c64"], res["c128"]
    achieved = r64["bytes_per_launch"] / (r64["launch_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": rate(r64),
        "unit": "arc-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "ctqw_torus_1024x1024_gamma0.25_K20_dt0.1_1000steps",
                   "n": g.n, "arcs": g.n_arcs, "gamma": GAMMA, "dt": DT, "taylor_order": K_ORDER,
                   "steps_per_pass": spp, "start_vertex": v0,
                   "path": r64["structure"], "parallelism": "single-gpu"},
        "arc_spmv_per_s": rate(r64) * K_ORDER,
        "p50_ms": pct(r64["per"], 50), "p99_ms": pct(r64["per"], 99),
        "c128": {"value": rate(r128), "ms_per_step": r128["wall"] / args.steps * 1e3,
                 "p50_ms": pct(r128["per"], 50), "p99_ms": pct(r128["per"], 99),
                 "stage_launch_ms": r128["launch_ms"],
                 "stage_gbs": r128["bytes_per_launch"] / (r128["launch_ms"] * 1e-3) / 1e9,
                 "l2_vs_closed_form": l2_128},
        "speedup_c64_vs_c128": rate(r64) / rate(r128),
        "l2_c64_vs_closed_form": l2_64,
        "l2_c64_vs_c128": l2_64_128,
        "norm_drift_c64": abs(r64["norm"] - 1.0),
        "roofline": {"bound": "hbm", "kernel": "k_ctqw_struct<float2,TORUS> (one Horner stage)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": r64["bytes_per_launch"],
                     "launch_ms": r64["launch_ms"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(g, v0, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
