"""Benchmark of the quantum-walk step engine on one MI355X.

Default workload: a batch of 4096 continuous-time quantum-walk searches on
seeded random d-regular graphs (N log-uniform in [1e3, 2e5], d uniform in
3..8, gamma = 1/d, one uniformly drawn marked vertex, uniform start, total
time 2 sqrt(N); time step and Taylor order from the truncation rule at
rho <= 1 and tolerance 1e-8), all advanced together in complex64 by the
batched kernel with an FP64 p_marked history per step.  One bench step is a
fixed chunk of batch launches (--launches-per-step); each launch advances
every active walk by one Horner stage.  After the timed chunks every walk's
state holds its last completed time step; a seeded sample of walks is then
checked against the FP64 oracle (final-state L2 and norm drift), the same
walks are run alone on the single-walk path in complex64 (must equal the
batch bitwise) and complex128 (must match the oracle to 1e-12), and a
second sample is timed one walk at a time in both precisions (the plain
form the batch is compared with).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
    python bench.py --workload grid      # 1024^2 grid CTQW, complex64 and complex128

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
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a
# 256 MiB copy (x2.00 / x1.00).  Each entry holds only for the kernel version
# and launch configuration named in its key and source; any other reports None.
MEASURED_TRAFFIC = {
    # profiles/batch4096_ctqw_search_lds.md: mean over the 5120 timed launches of the
    # default command, FETCH_SIZE 3,088,620.9 KiB x 2.00 + WRITE_SIZE 1,164,456.9 KiB x 1.00
    # (768 threads x 9 rows, 19968-entry blocks staged by LDS-direct loads)
    "k_batch_ell_lds<float2,768,9,19968> batch4096 seed1 launches1280-6400": (3088620.9 * 2 + 1164456.9) * 1024,
    # profiles/ctqw_torus1024_sweep.md: the FP32 complex64 sweep, averaged over the four
    # launches of a step, FETCH_SIZE (4543.1 + 3 x 8942.0) / 4 KiB x 2.00 + WRITE_SIZE 8193.3 KiB
    "k_ctqw_torus_sweep<float2,5> 1024x1024": ((4543.1 + 3 * 8942.0) / 4 * 2 + 8193.3) * 1024,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--grid-side", type=int, default=L_SIDE,
                    help="side of the periodic grid (default 1024; 4096 gives an HBM-resident variant)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--steps-per-pass", type=int, default=STEPS_PER_PASS,
                    help="time steps per pass (profiling runs shorten it; rates are per arc-step)")
    ap.add_argument("--dtypes", default="c64,c128")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--workload", default="batch",
                    choices=["grid", "batch", "serve", "dense", "hypercube", "cycle", "snapshots", "staggered",
                             "lattice", "sparse", "streamed"],
                    help="batch: 4096 CTQW searches on random regular graphs in one batch (default); "
                         "grid: the 1024^2 CTQW; serve: the Poisson job stream")
    ap.add_argument("--batch-walks", type=int, default=4096)
    ap.add_argument("--batch-seed", type=int, default=1)
    ap.add_argument("--launches-per-step", type=int, default=256,
                    help="batch: launches (one Horner stage of every active walk each) per bench step")
    ap.add_argument("--graph-cache", default="",
                    help="batch: directory to read the drawn graphs from, or to write them to")
    ap.add_argument("--direct-launch", action="store_true",
                    help="batch: launch each stage directly instead of replaying captured hipGraphs")
    ap.add_argument("--stage-kernel", default="auto", choices=["auto", "lds", "gather"],
                    help="batch: kernel for the walks' Horner stages (auto: the autotuner's choice)")
    ap.add_argument("--oracle-walks", type=int, default=16, help="batch: walks checked against the oracle")
    ap.add_argument("--oracle-budget", type=float, default=2.5e10,
                    help="batch: bound on the oracle sample's work (time steps x K x arcs)")
    ap.add_argument("--plain-sample", type=int, default=16,
                    help="walks of the batch also run one at a time on the single-walk path (timed)")
    ap.add_argument("--stream-n", type=int, default=2**21, help="streamed workload: vertices")
    ap.add_argument("--stream-degree", type=int, default=32, help="streamed workload: mean degree")
    ap.add_argument("--stream-steps", type=int, default=3, help="streamed workload: timed time steps")
    ap.add_argument("--stream-budget-mib", type=int, default=64,
                    help="streamed workload: device MiB for the streamed graph beyond state and workspace")
    ap.add_argument("--progress", action="store_true", help="batch: a stderr line per timed step as it is enqueued")
    ap.add_argument("--gen-only", action="store_true",
                    help="batch: only draw the graphs into --graph-cache (no GPU) and exit")
    ap.add_argument("--serve-jobs", type=int, default=120)
    ap.add_argument("--serve-no-plain-saturated", action="store_true",
                    help="skip the plain form's saturated run (long streams split over several runs)")
    ap.add_argument("--serve-rates", default="0.5,0.9",
                    help="arrival rates as fractions of the measured saturated capacity")
    ap.add_argument("--serve-max-arcs", type=float, default=4e6)
    ap.add_argument("--serve-max-steps", type=int, default=5000)
    ap.add_argument("--serve-solo-arcs", type=float, default=2 ** 19,
                    help="jobs with at least this many arcs run in a solo lane")
    ap.add_argument("--serve-batch-arcs", type=float, default=2 ** 21,
                    help="cap on the arcs in the batch lane (0: none)")
    ap.add_argument("--serve-solo-slots", type=int, default=3, help="solo lanes running at once")
    ap.add_argument("--serve-no-idle-solo", action="store_true",
                    help="serve: never route a mid-size job to an idle solo lane while the batch is empty")
    ap.add_argument("--serve-solo-units", type=int, default=16384,
                    help="jobs needing at least this many launches (steps x K) run in a solo lane (0: none)")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--dense-n", type=int, default=15000)
    ap.add_argument("--dense-columns", default="1,8,32,128")
    ap.add_argument("--dense-dtype", default="c128")
    ap.add_argument("--snap-every", type=int, default=10, help="snapshots workload: steps between snapshots")
    ap.add_argument("--hypercube-layout", default="auto", choices=["auto", "csr"],
                    help="auto: index-free slot-major kernel; csr: the general CSR coined path")
    ap.add_argument("--hypercube-steps", type=int, default=0,
                    help="override the step count (profiling runs); 0 = ceil((pi/2) sqrt(N ln N))")
    ap.add_argument("--hypercube-dtypes", default="c64,c128")
    ap.add_argument("--stag-side", type=int, default=4096, help="staggered workload: side of the square lattice")
    ap.add_argument("--stag-steps", type=int, default=200, help="staggered workload: steps per timed pass")
    ap.add_argument("--stag-dtypes", default="c64,c128")
    ap.add_argument("--stag-layout", default="auto", choices=["auto", "csr"],
                    help="auto: the fused square-lattice kernel; csr: the per-tessellation polygon kernels")
    ap.add_argument("--lattice-side", type=int, default=2048, help="lattice workload: side of the periodic grid")
    ap.add_argument("--lattice-steps", type=int, default=200, help="lattice workload: steps per timed pass")
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


def stage_launch_ms(plan, per_pass_ms, steps_per_pass):
    """Average duration of one launch of the stage kernel over the timed
    region: the HIP-event time of the timed passes (recorded on the stream
    the kernels run on) over the number of stage launches they made
    (K / block_depth per time step).  The FP64 readout at the end of each
    pass, one small launch per thousands, is counted in."""
    launches = len(per_pass_ms) * steps_per_pass * (K_ORDER // max(1, plan.info.block_depth))
    return sum(per_pass_ms) / launches


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
    psi = oracle.ctqw_evolve(g.row_ptr, g.col, psi, 2, gamma=GAMMA, dt=DT, K=K_ORDER)  # warm-up
    n_more, chunk = 0, 25
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        psi = oracle.ctqw_evolve(g.row_ptr, g.col, psi, chunk, gamma=GAMMA, dt=DT, K=K_ORDER)
        n_more += chunk
    el = time.perf_counter() - t0
    return {"value": g.n_arcs * n_more / el, "unit": "arc-steps/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{n_more} time steps (dt={DT}) of the same walk from the same start vertex on the "
                      f"same {g.name} grid, run as oracle calls of {chunk} steps for about {seconds:g} s "
                      f"(FP64 power-form Taylor, K={K_ORDER})",
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
    if args.gen_only:
        batch_walks(args)
        return
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "dense":
        run_dense(args)
        return
    if args.workload == "hypercube":
        run_hypercube(args)
        return
    if args.workload == "cycle":
        run_cycle(args)
        return
    if args.workload == "snapshots":
        run_snapshots(args)
        return
    if args.workload == "staggered":
        run_staggered(args)
        return
    if args.workload == "lattice":
        run_lattice(args)
        return
    if args.workload == "sparse":
        run_sparse(args)
        return
    if args.workload == "grid":
        run_grid(args)
        return
    if args.workload == "streamed":
        run_streamed(args)
        return
    raise SystemExit(f"unknown workload {args.workload}")


def run_grid(args):
    """The 1024 x 1024 grid CTQW (gamma 0.25, K 20, dt 0.1, from vertex (512, 512)):
    passes of 1000 time steps plus the FP64 readout, complex64 and complex128,
    both checked against the closed form (product of cycle Bessel sums)."""
    spp = args.steps_per_pass
    dtypes = args.dtypes.split(",")
    import numpy as np
    import torch

    from oracle import closed_forms as cf
    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Plan

    side = args.grid_side
    g = I.torus(side, side)
    v0 = (side // 2) * side + side // 2
    psi0 = I.ket_vertex(g.n, v0)
    res = {}
    for dtype in dtypes:
        pl = Plan(g, "ctqw", dtype=dtype, gamma=GAMMA, dt=DT, taylor_order=K_ORDER)
        psi = pl.state(psi0)
        wall, per, (p, norm, _) = timed_passes(pl, psi, args.steps, args.warmup, spp)
        total_steps = (args.steps + args.warmup) * spp
        state = psi.cpu().numpy().astype(np.complex128)
        launch_ms = stage_launch_ms(pl, per, spp)
        es = 8 if dtype == "c64" else 16
        # algorithmic bytes of one row-stage of the matrix-free grid stencil: read y,
        # read psi, write y' (3 S); one launch runs block_depth stages of every row
        depth = int(pl.info.block_depth)
        # bytes a launch must move: read y_in and psi, write y_out (3 S per row);
        # the first launch of a time step reads psi as y_in (2 S).  Averaged over
        # the K / depth launches of a step.
        lps = max(1, K_ORDER // depth)
        bytes_per_launch = (3 * lps - 1) / lps * es * g.n
        stage_model_bytes = depth * 3 * es * g.n
        res[dtype] = dict(plan=pl, wall=wall, per=per, norm=float(norm), state=state,
                          total_steps=total_steps, launch_ms=launch_ms,
                          bytes_per_launch=bytes_per_launch, stage_model_bytes=stage_model_bytes,
                          structure=pl.structure,
                        depth=depth)
        del psi
    t_final = res[dtypes[0]]["total_steps"] * DT
    ref1 = cf.cycle_ctqw(side, GAMMA, t_final, side // 2)
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
    kname = (f"k_ctqw_torus_sweep<float2,{r64['depth']}>" if r64["depth"] > 1
             else "k_ctqw_struct<float2,TORUS>")
    traffic = MEASURED_TRAFFIC.get(f"{kname} {side}x{side}")
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
        "config": {"workload": f"ctqw_torus_{side}x{side}_gamma0.25_K20_dt0.1_{spp}steps"
                               + ("" if side == L_SIDE else "_supplementary"),
                   "n": g.n, "arcs": g.n_arcs, "gamma": GAMMA, "dt": DT, "taylor_order": K_ORDER,
                   "steps_per_pass": spp, "start_vertex": v0,
                   "path": r64["structure"], "stages_per_launch": r64["depth"], "parallelism": "single-gpu"},
        "arc_spmv_per_s": rate(r64) * K_ORDER,
        "p50_ms": pct(r64["per"], 50), "p99_ms": pct(r64["per"], 99),
        "c128": {"value": rate(r128), "ms_per_step": r128["wall"] / args.steps * 1e3,
                 "p50_ms": pct(r128["per"], 50), "p99_ms": pct(r128["per"], 99),
                 "stage_launch_ms": r128["launch_ms"],
                 "launch_gbs": r128["bytes_per_launch"] / (r128["launch_ms"] * 1e-3) / 1e9,
                 "launch_frac": r128["bytes_per_launch"] / (r128["launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "l2_vs_closed_form": l2_128},
        "speedup_c64_vs_c128": rate(r64) / rate(r128),
        "l2_c64_vs_closed_form": l2_64,
        "l2_c64_vs_c128": l2_64_128,
        "norm_drift_c64": abs(r64["norm"] - 1.0),
        "roofline": {"bound": "hbm",
                     "kernel": kname + (f" ({r64['depth']} Horner stages per launch)" if r64["depth"] > 1
                                        else " (one Horner stage)"),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": r64["bytes_per_launch"],
                     "launch_ms": r64["launch_ms"],
                     "stage_model_gbs": r64["stage_model_bytes"] / (r64["launch_ms"] * 1e-3) / 1e9,
                     "note": ("achieved counts the bytes one launch must move (psi and y_in read, y_out "
                              "written; psi doubles as y_in in the first launch of a step); "
                              "stage_model_gbs counts 3 S per row for every stage the launch runs, "
                              "which several stages per launch in registers avoid moving")},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(g, v0, args.cpu_seconds)
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- batch workload (default)

def _gen_regular(spec):
    from paper_2406_08186_amd import inputs as I
    g = I.random_regular(spec["n"], spec["d"], spec["graph_seed"])
    return g.row_ptr, g.col


def batch_csrs(args, specs):
    """CSR arrays of the batch's graphs: drawn from their seeds in worker
    processes, or read back from --graph-cache when that directory holds this
    batch (it is written there after drawing).  Returns (list of (row_ptr,
    col), source)."""
    import multiprocessing as mp

    import numpy as np
    key = {"walks": len(specs), "seed": args.batch_seed, "format": 1}
    cache = args.graph_cache
    if cache and os.path.exists(os.path.join(cache, "meta.json")):
        with open(os.path.join(cache, "meta.json")) as f:
            meta = json.load(f)
        if meta.get("key") == key:
            rp_all = np.load(os.path.join(cache, "row_ptr.npy"), mmap_mode="r")
            col_all = np.load(os.path.join(cache, "col.npy"), mmap_mode="r")
            ro, co = meta["rp_off"], meta["col_off"]
            return [(np.asarray(rp_all[ro[i]:ro[i + 1]]), np.asarray(col_all[co[i]:co[i + 1]]))
                    for i in range(len(specs))], "cache"
    if args.workers <= 1:
        csrs = [_gen_regular(sp) for sp in specs]
    else:
        with mp.get_context("fork").Pool(min(args.workers, os.cpu_count() or 1)) as pool:
            csrs = pool.map(_gen_regular, specs, chunksize=4)
    if cache:
        os.makedirs(cache, exist_ok=True)
        ro = np.cumsum([0] + [rp.size for rp, _ in csrs]).tolist()
        co = np.cumsum([0] + [c.size for _, c in csrs]).tolist()
        np.save(os.path.join(cache, "row_ptr.npy"), np.concatenate([rp.astype(np.int64) for rp, _ in csrs]))
        np.save(os.path.join(cache, "col.npy"), np.concatenate([c.astype(np.int32) for _, c in csrs]))
        with open(os.path.join(cache, "meta.json"), "w") as f:
            json.dump({"key": key, "rp_off": ro, "col_off": co}, f)
    return csrs, "generated"


def batch_walks(args):
    """Specs, graphs and (K, dt, steps) schedules of the batch."""
    from paper_2406_08186_amd import _lib as L
    from paper_2406_08186_amd import inputs as I
    specs = I.batch_regular_specs(args.batch_walks, seed=args.batch_seed)
    t0 = time.perf_counter()
    csrs, src = batch_csrs(args, specs)
    gen_s = time.perf_counter() - t0
    print(f"[batch] {len(specs)} graphs {src} in {gen_s:.1f} s", file=sys.stderr, flush=True)
    graphs = [I.Graph(n=sp["n"], row_ptr=rp, col=cl, name=f"rr{i}") for i, (sp, (rp, cl)) in
              enumerate(zip(specs, csrs))]
    sched = []
    for sp in specs:
        # ||H||_inf = gamma d + 1 (the marked vertex); rho <= 1, tolerance 1e-8 over the whole walk
        K, dt, steps = L.qw_taylor_plan(sp["gamma"] * sp["d"] + 1.0, sp["t_final"], 1.0, 1e-8)
        sched.append((K, dt, steps))
    return specs, graphs, sched, gen_s


def _walk_plan(graph, spec, sched, dtype, upload=True):
    from paper_2406_08186_amd.walk import Plan
    K, dt, _ = sched
    return Plan(graph, "ctqw", dtype=dtype, layout="structured", gamma=spec["gamma"], dt=dt,
                taylor_order=K, marked=[spec["marked"]], upload=upload)


def oracle_sample(args, graphs, sched, done_steps):
    """Seeded sample of walks for the oracle check, bounded by an estimate of
    the oracle's work (steps x K x arcs summed over the sample)."""
    import numpy as np
    rng = np.random.default_rng(args.batch_seed + 7)
    budget = args.oracle_budget
    out = []
    for i in rng.permutation(len(graphs)).tolist():
        cost = done_steps[i] * sched[i][0] * max(1, graphs[i].n_arcs)
        if done_steps[i] > 0 and cost <= budget:
            out.append(i)
            budget -= cost
        if len(out) >= args.oracle_walks:
            break
    return out


def run_batch(args):
    """The default bench line: the 4096-walk CTQW search batch (module docstring)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    specs, graphs, sched, gen_s = batch_walks(args)

    import torch

    import oracle
    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Batch

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max(1, args.workers)) as ex:
        plans = list(ex.map(lambda i: _walk_plan(graphs[i], specs[i], sched[i], "c64", upload=False),
                            range(len(specs))))
    plan_s = time.perf_counter() - t0
    total_rows = sum(g.n for g in graphs)
    # tiles at 256 rows or more, plus the XCD padding (8 lists, each about the mean plus the
    # largest walk's tiles under longest-first placement by load), with a tenth to spare
    max_tiles = int(1.1 * (total_rows // 256 + len(graphs) + 8 * (max(g.n for g in graphs) // 256 + 1) + 64))
    batch = Batch(capacity=len(plans), max_tiles=max_tiles, dtype="c64")
    states, hists = [], []
    for i, pl in enumerate(plans):
        pl.upload()
        psi = pl.state(I.uniform(graphs[i].n))
        hist = torch.zeros(sched[i][2], dtype=torch.float64, device="cuda")
        batch.set_slot(i, pl, psi, sched[i][2], hist=hist)
        states.append(psi)
        hists.append(hist)
    if args.stage_kernel != "auto":
        batch.set_stage_kernel(args.stage_kernel)
    batch.commit()
    if args.direct_launch:
        batch.set_replay(False)
    if args.stage_kernel == "auto":
        rows, xcd, _ = batch.autotune(reps=2)
    sched_now = batch.schedule()
    rows, xcd, stage_kernel = sched_now["rows_per_tile"], sched_now["xcd_aware"], sched_now["stage_kernel"]
    torch.cuda.synchronize()
    print(f"[batch] plans built in {plan_s:.1f} s; schedule {rows} rows/tile, xcd {bool(xcd)}",
          file=sys.stderr, flush=True)

    units = np.array([batch.remaining(i) for i in range(len(plans))], dtype=np.int64)
    Ks = np.array([s[0] for s in sched], dtype=np.int64)
    A = np.array([g.n_arcs for g in graphs], dtype=np.float64)
    Nv = np.array([g.n for g in graphs], dtype=np.float64)
    D = np.array([sp["d"] for sp in specs], dtype=np.float64)
    CH = args.launches_per_step
    total = int(units.max())
    if (args.warmup + args.steps) * CH > total:
        CH = max(1, total // (args.warmup + args.steps))
        print(f"[batch] launches per step cut to {CH} to stay inside one pass", file=sys.stderr, flush=True)

    def finished_between(la, lb):
        return [i for i in range(len(plans)) if la < units[i] <= lb]

    for w in range(args.warmup):
        la = batch.launches
        batch.run(CH)
        for i in finished_between(la, batch.launches):
            batch.readout(i)
        print(f"[batch] warm-up step {w + 1}/{args.warmup} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    La = batch.launches
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        la = batch.launches
        ev[k][0].record()
        batch.run(CH)
        ev[k][1].record()
        for i in finished_between(la, batch.launches):  # fused-path readout of walks that just ended
            batch.readout(i)
        ev[k][2].record()
        if args.progress:
            print(f"[batch] step {k + 1}/{args.steps} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    Lb = batch.launches
    print(f"[batch] timed launches {La}..{Lb} in {wall:.2f} s", file=sys.stderr, flush=True)
    run_ms = sum(e[0].elapsed_time(e[1]) for e in ev)
    per = sorted(e[0].elapsed_time(e[2]) for e in ev)
    stages = np.clip(Lb, 0, units) - np.clip(La, 0, units)
    arc_steps = float((A * stages / Ks).sum())
    alg_bytes = float((Nv * (4 * D + 24) * stages).sum())
    active_start = int((units > La).sum())
    active_end = int((units > Lb).sum())
    launches = args.steps * CH
    launch_ms = run_ms / launches

    # ---- parity on a seeded sample: oracle (FP64), the walk alone in c64 and c128
    done = np.minimum(Lb, units) // Ks
    sample = oracle_sample(args, graphs, sched, done)
    l2s, drifts, c128_err, c64_alone_diff, oracle_s, oracle_as = [], [], [], [], 0.0, 0.0
    for i in sample:
        g, sp, (K, dt, _) = graphs[i], specs[i], sched[i]
        c = int(done[i])
        got = states[i].cpu().numpy().astype(np.complex128)
        t1 = time.perf_counter()
        ref = oracle.ctqw_evolve(g.row_ptr, g.col, I.uniform(g.n), c, gamma=sp["gamma"], dt=dt, K=K,
                                 marked=[sp["marked"]])
        oracle_s += time.perf_counter() - t1
        oracle_as += g.n_arcs * c
        l2s.append(float(np.linalg.norm(got - ref)))
        drifts.append(abs(float(np.sum(np.abs(got) ** 2)) - 1.0))
        for dtype in ("c64", "c128"):
            pl = _walk_plan(g, sp, sched[i], dtype)
            x = pl.state(I.uniform(g.n))
            pl.evolve(x, c)
            if dtype == "c64":
                c64_alone_diff.append(float((x - states[i]).abs().max()))
            else:
                c128_err.append(float(np.abs(x.cpu().numpy() - ref).max()))
            del x
            pl.close()

    print(f"[batch] parity on {len(sample)} walks; oracle {oracle_s:.1f} s", file=sys.stderr, flush=True)

    # ---- the plain form: one walk at a time on the single-walk path, whole walks
    stride = max(1, len(plans) // max(1, args.plain_sample))
    psample = list(range(0, len(plans), stride))[:args.plain_sample]
    plain = {}
    for dtype in ("c64", "c128"):
        as_, secs = 0.0, 0.0
        for i in psample:
            pl = _walk_plan(graphs[i], specs[i], sched[i], dtype)
            x = pl.state(I.uniform(graphs[i].n))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            pl.evolve(x, sched[i][2])
            torch.cuda.synchronize()
            secs += time.perf_counter() - t1
            as_ += graphs[i].n_arcs * sched[i][2]
            del x
            pl.close()
        print(f"[batch] plain form {dtype}: {len(psample)} walks in {secs:.1f} s", file=sys.stderr, flush=True)
        plain[dtype] = {"value": as_ / secs if secs > 0 else None, "unit": "arc-steps/s",
                        "walks": len(psample), "seconds": secs}

    value = arc_steps / wall
    l2_max = max(l2s) if l2s else None
    kname = "k_batch_ell_lds<float2,768,9,19968>" if stage_kernel == "lds" else "k_batch_stage<float2>"
    traffic_key = f"{kname} batch{len(plans)} seed{args.batch_seed} launches{La}-{Lb}"
    traffic = MEASURED_TRAFFIC.get(traffic_key)
    line = {
        "metric": METRIC, "value": value, "unit": "arc-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"batch_{len(plans)}_ctqw_search_random_regular_c64",
                   "walks": len(plans), "n_range": [1e3, 2e5], "degree_range": [3, 8],
                   "total_vertices": total_rows, "total_arcs": int(A.sum()),
                   "launches_per_step": CH, "launches_per_pass": total,
                   "timed_launches": [La, Lb], "walks_active_at_start": active_start,
                   "walks_active_at_end": active_end,
                   "path": sorted({pl.structure for pl in plans}), "stage_kernel": stage_kernel,
                   "rows_per_tile": rows,
                   "xcd_aware": bool(xcd), "replay": "direct" if args.direct_launch else "hipgraph",
                   "graph_gen_s": gen_s, "plan_build_s": plan_s, "parallelism": "single-gpu"},
        "arc_spmv_per_s": float((A * stages).sum()) / wall,
        "p50_ms": pct(per, 50), "p99_ms": pct(per, 99),
        "parity": {"walks": len(sample), "steps_checked": [int(done[i]) for i in sample],
                   "l2_vs_oracle_max": l2_max, "l2_gate": 1e-4,
                   "l2_gate_pass": l2_max is not None and l2_max <= 1e-4,
                   "norm_drift_max": max(drifts) if drifts else None,
                   "c64_alone_vs_batch_max_abs_diff": max(c64_alone_diff) if c64_alone_diff else None,
                   "c128_plain_vs_oracle_max_abs": max(c128_err) if c128_err else None,
                   "c128_gate": 1e-12},
        "c128_plain": plain["c128"], "c64_plain": plain["c64"],
        "speedup_vs_c128_plain": value / plain["c128"]["value"] if plain["c128"]["value"] else None,
        "speedup_vs_c64_plain": value / plain["c64"]["value"] if plain["c64"]["value"] else None,
        "roofline": {"bound": "hbm", "kernel": kname,
                     "achieved": alg_bytes / (run_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg_bytes / (run_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": alg_bytes / launches, "launch_ms": launch_ms,
                     "note": "algorithmic bytes per row-stage on the ELL layout: 4d neighbour indices + "
                             "8 (the gathered vector once) + 8 (psi) + 8 (y out); launch_ms from HIP events "
                             "around the timed batch launches on their stream"},
    }
    if not args.no_cpu_baseline and sample:
        line["cpu_baseline"] = {
            "value": oracle_as / oracle_s, "unit": "arc-steps/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{len(sample)} walks of the batch (seeded choice), each from the uniform state for the "
                      f"time steps it completed in the GPU run ({sum(int(done[i]) for i in sample)} steps, "
                      f"{oracle_as:.3g} arc-steps): FP64 power-form Taylor, the same K and dt",
            "seconds": oracle_s}
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- serving stream

def _gen_job(args_tuple):
    from paper_2406_08186_amd.serve import make_job
    import numpy as np
    i, seed, max_arcs, max_steps = args_tuple
    return make_job(i, np.random.default_rng(seed), arc_range=(1e3, max_arcs), steps_range=(100, max_steps))


def run_serve(args):
    """Poisson stream of mixed coined / CTQW jobs served (continuous batch for
    small jobs, solo lane for large ones), against the plain one-job-at-a-time
    form on the same GPU with the same arrivals."""
    import copy
    import multiprocessing as mp

    import numpy as np
    t0 = time.perf_counter()
    tasks = [(i, 1000 + i, args.serve_max_arcs, args.serve_max_steps) for i in range(args.serve_jobs)]
    if args.workers <= 1:
        base_jobs = [_gen_job(t) for t in tasks]
    else:
        with mp.get_context("fork").Pool(min(args.workers, os.cpu_count() or 1)) as pool:
            base_jobs = pool.map(_gen_job, tasks)
    print(f"[serve] generated {len(base_jobs)} jobs in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    import torch

    from paper_2406_08186_amd.serve import WalkServer, latency_stats, poisson_arrivals, serve_sequential, serve_stream

    def arc_work(jobs):
        return sum(j.arcs * j.steps for j in jobs if j.status == "done")

    def report(done, seconds):  # progress of a long stream
        print(f"[serve]   {done} jobs done at {seconds:.1f} s", file=sys.stderr, flush=True)

    def fresh():
        return [copy.copy(j) for j in base_jobs]

    def served(jobs):
        srv = WalkServer(capacity=64, chunk=64, dtype="c64", workers=args.workers,
                         solo_arcs=int(args.serve_solo_arcs), solo_slots=args.serve_solo_slots,
                         solo_units=args.serve_solo_units or None, idle_solo=not args.serve_no_idle_solo,
                         batch_arcs=int(args.serve_batch_arcs) if args.serve_batch_arcs > 0 else None)
        t1 = time.perf_counter()
        done = serve_stream(srv, jobs, time_limit=900, progress=report)
        el = time.perf_counter() - t1
        srv.close()
        return done, el, srv.cycles

    def plain(jobs):
        t1 = time.perf_counter()
        serve_sequential(jobs, time_limit=1800, progress=report)
        return jobs, time.perf_counter() - t1

    # warm-up (kernel loading, graph capture): a few jobs, untimed
    warm = fresh()[:8]
    for j in warm:
        j.arrival = 0.0
    served(warm)
    # saturated capacity: every job at t = 0
    jobs = fresh()
    for j in jobs:
        j.arrival = 0.0
    done, sat_s, _ = served(jobs)
    cap_jobs_s = len(done) / sat_s
    cap_rate = arc_work(done) / sat_s
    print(f"[serve] saturated: {len(done)} jobs in {sat_s:.1f} s", file=sys.stderr, flush=True)
    plain_sat = None
    if not args.serve_no_plain_saturated:
        jobs = fresh()
        for j in jobs:
            j.arrival = 0.0
        pdone, psat_s = plain(jobs)
        plain_sat = {"jobs_per_s": len(pdone) / psat_s, "arc_steps_per_s": arc_work(pdone) / psat_s}
        print(f"[serve] plain saturated: {len(pdone)} jobs in {psat_s:.1f} s", file=sys.stderr, flush=True)
    results = []
    for k, frac in enumerate(float(x) for x in args.serve_rates.split(",")):
        lam = frac * cap_jobs_s
        arrivals = poisson_arrivals(len(base_jobs), lam, np.random.default_rng(7 + k))
        jobs = fresh()
        for j, a in zip(jobs, arrivals):
            j.arrival = float(a)
        done, el, cycles = served(jobs)
        st = latency_stats(done)
        print(f"[serve] load {frac}: served {len(done)} jobs in {el:.1f} s", file=sys.stderr, flush=True)
        jobs = fresh()
        for j, a in zip(jobs, arrivals):
            j.arrival = float(a)
        pdone, pel = plain(jobs)
        pst = latency_stats(pdone)

        def tail(js):  # the five slowest jobs: latency, lane, kind, arcs, steps
            return [[round(j.latency, 3), j.lane, j.kind, j.arcs, j.steps]
                    for j in sorted(js, key=lambda j: -j.latency)[:5]]
        results.append({"load": frac, "rate_jobs_per_s": lam, "arc_steps_per_s": arc_work(done) / el,
                        **st, "cycles": cycles, "slowest": tail(done),
                        "plain": {"arc_steps_per_s": arc_work(pdone) / pel, **pst, "slowest": tail(pdone)}})
        print(f"[serve] load {frac}: p50 {st['p50_s']:.3f} s p99 {st['p99_s']:.3f} s; plain p50 "
              f"{pst['p50_s']:.3f} s p99 {pst['p99_s']:.3f} s", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": cap_rate, "unit": "arc-steps/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": sat_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"serve_{len(base_jobs)}_mixed_jobs", "jobs": len(base_jobs),
                   "arcs_range": [1e3, args.serve_max_arcs], "steps_range": [100, args.serve_max_steps],
                   "slots": 64, "chunk": 64, "solo_lane_arcs": int(args.serve_solo_arcs),
                   "batch_arcs_cap": int(args.serve_batch_arcs), "solo_lanes": args.serve_solo_slots,
                   "solo_lane_units": args.serve_solo_units, "idle_solo": not args.serve_no_idle_solo,
                   "parallelism": "single-gpu"},
        "saturated_jobs_per_s": cap_jobs_s,
        "plain_saturated": plain_sat,
        "speedup_saturated_vs_plain": cap_rate / plain_sat["arc_steps_per_s"] if plain_sat else None,
        "loads": results,
    }
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- dense H on MFMA

def run_dense(args):
    """CTQW search on the complete graph K_n through the dense-H path: every
    Horner stage is an n x n by n x 2B real GEMM on the matrix cores, for B
    walks sharing H (n = 15000 is the dense vector-matrix size the paper times,
    Sec. 4.6.1).  Reports per-stage time, GB/s of H streamed and MFMA TFLOP/s."""
    import numpy as np
    import torch

    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Plan
    n = args.dense_n
    g = I.complete(n)
    es = 8 if args.dense_dtype == "c128" else 4
    peak_tf = 78.6 if args.dense_dtype == "c128" else 157.3
    out = []
    for cols in [int(x) for x in args.dense_columns.split(",")]:
        pl = Plan(g, "ctqw", dtype=args.dense_dtype, layout="dense", gamma=1.0 / n, dt=0.5, taylor_order=16,
                  marked=[7], columns=cols)
        u = np.full(n * cols, 1 / math.sqrt(n), dtype=np.complex128)
        psi = pl.state(u)
        pl.evolve(psi, 1)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        a.record()
        pl.evolve(psi, reps)
        b.record()
        torch.cuda.synchronize()
        ms_stage = a.elapsed_time(b) / (reps * 16)
        flops = 2.0 * n * n * 2 * cols
        hbytes = float(n) * n * es
        out.append({"columns": cols, "ms_per_stage": ms_stage, "tflops": flops / (ms_stage * 1e-3) / 1e12,
                    "mfma_frac": flops / (ms_stage * 1e-3) / 1e12 / peak_tf,
                    "h_gbs": hbytes / (ms_stage * 1e-3) / 1e9,
                    "hbm_frac": hbytes / (ms_stage * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "arc_steps_per_s": g.n_arcs * cols * reps / (a.elapsed_time(b) * 1e-3)})
        pl.close()
        del psi
    print(json.dumps({"workload": f"dense_complete_{n}", "dtype": args.dense_dtype, "taylor_order": 16,
                      "points": out}), flush=True)


# ---------------------------------------------------------------- hypercube search

def run_hypercube(args):
    """Coined Grover search on the dimension-20 hypercube (2^20 vertices,
    20 * 2^20 arcs), coin -I at vertex 0, uniform arc state, ceil((pi/2)
    sqrt(N ln N)) = 5989 steps; complex64 and complex128, checked against the
    symmetric-subspace closed form."""
    import numpy as np
    import torch

    from oracle import closed_forms as cf
    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Plan
    dim = 20
    n = 1 << dim
    steps = args.hypercube_steps or math.ceil(math.pi / 2 * math.sqrt(n * math.log(n)))
    g = I.hypercube(dim)
    o, _, _ = cf.hypercube_search_reduced(dim, steps)
    ref = cf.hypercube_search_state(dim, steps, g.row_ptr, g.col)
    res = {}
    for dtype in args.hypercube_dtypes.split(","):
        pl = Plan(g, "coined", dtype=dtype, marked=[0], layout=args.hypercube_layout)
        psi0 = np.full(g.n_arcs, 1 / math.sqrt(g.n_arcs), dtype=np.complex128)
        psi = pl.state(psi0)
        pl.evolve(psi, 2)
        torch.cuda.synchronize()
        psi = pl.state(psi0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record()
        p, norm, pm = pl.evolve(psi, steps, readout=True)
        b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = a.elapsed_time(b)
        es = 8 if dtype == "c64" else 16
        # algorithmic bytes per arc-step: read and write the state (2S); the
        # general CSR path also reads rev (4 B) and row_ptr (4/d B)
        per_arc = 2 * es + (0 if pl.structure == "hypercube" else 4 + 4 / dim)
        got = psi.cpu().numpy().astype(np.complex128)
        res[dtype] = {"value": g.n_arcs * steps / (ms * 1e-3), "ms": ms, "wall_s": wall,
                      "step_us": ms * 1e3 / steps, "bytes_per_arc_step": per_arc,
                      "step_gbs": per_arc * g.n_arcs / (ms * 1e-3 / steps) / 1e9,
                      "frac": per_arc * g.n_arcs / (ms * 1e-3 / steps) / 1e9 / HBM_PEAK_GBS,
                      "p_marked": float(pm), "p_marked_ref": float(abs(o[0]) ** 2),
                      "l2_vs_closed_form": float(np.linalg.norm(got - ref)), "norm": float(norm),
                      "path": pl.structure}
        del psi
        pl.close()
    print(json.dumps({"workload": "coined_search_hypercube20", "steps": steps, "arcs": g.n_arcs,
                      "unit": "arc-steps/s", "layout": args.hypercube_layout,
                      **{k: v for k, v in res.items()}}), flush=True)


# ---------------------------------------------------------------- streamed snapshots

def run_snapshots(args):
    """The 1024 x 1024 grid CTQW pass (1000 steps, complex64) with a snapshot
    every --snap-every steps brought to host memory: compute alone, the naive
    form (evolve, then a synchronous copy per snapshot), the streamed form
    (qw_copy_to_host: a copy kernel on the walk's stream writes each snapshot
    into its pinned host buffer), for states and for FP64 distributions, and
    the runtime-copy form (device ring, hipMemcpyAsync on a second stream)
    beside it."""
    import numpy as np
    import torch

    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd import _lib as L
    from paper_2406_08186_amd.walk import Plan, stream_snapshots
    g = I.torus(L_SIDE, L_SIDE)
    v0 = (L_SIDE // 2) * L_SIDE + L_SIDE // 2
    psi0 = I.ket_vertex(g.n, v0)
    pl = Plan(g, "ctqw", dtype="c64", gamma=GAMMA, dt=DT, taylor_order=K_ORDER)
    every = args.snap_every
    snaps = list(range(every, STEPS_PER_PASS + 1, every))

    def timed(fn):
        psi = pl.state(psi0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn(psi)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out, psi

    def compute(psi):
        pl.evolve(psi, STEPS_PER_PASS)

    def naive(psi):
        out, at = [], 0
        for k in snaps:
            pl.evolve(psi, k - at)
            at = k
            out.append(psi.cpu().numpy())
        return out

    pinned_s = [torch.empty(g.n, dtype=torch.complex64, pin_memory=True) for _ in snaps]
    pinned_p = [torch.empty(g.n, dtype=torch.float64, pin_memory=True) for _ in snaps]
    timed(compute)                                  # warm-up
    t_comp, _, ref = timed(compute)
    t_naive, out_n, _ = timed(naive)
    t_ce, out_ce, _ = timed(lambda psi: stream_snapshots(pl, psi, snaps, "state", host=pinned_s, via="memcpy"))
    out_ce = [x.copy() for x in out_ce]             # the buffers are reused below
    t_ce_prob, _, _ = timed(lambda psi: stream_snapshots(pl, psi, snaps, "probability", host=pinned_p,
                                                         via="memcpy"))
    t_state, out_s, _ = timed(lambda psi: stream_snapshots(pl, psi, snaps, "state", host=pinned_s))
    t_prob, out_p, _ = timed(lambda psi: stream_snapshots(pl, psi, snaps, "probability", host=pinned_p))
    same = all(np.array_equal(a, b) for a, b in zip(out_n, out_s))
    same_ce = all(np.array_equal(a, b) for a, b in zip(out_ce, out_s))
    final_ok = np.array_equal(out_s[-1], ref.cpu().numpy())
    # each transfer's rate alone: the same device-to-pinned copies, nothing
    # else running (this overwrites the pinned buffers, so it comes last)
    src = pl.state(psi0)
    cs = int(torch.cuda.current_stream().cuda_stream)
    rates = {}
    for via in ("memcpy", "link"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for h in pinned_s:
            if via == "link":
                L.qw_copy_to_host(h.data_ptr(), src.data_ptr(), g.n * 8, cs)
            else:
                h.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        rates[via] = time.perf_counter() - t0
    t_d2h, t_link = rates["memcpy"], rates["link"]
    mb_state = len(snaps) * g.n * 8 / 1e6
    mb_prob = len(snaps) * g.n * 8 / 1e6
    print(json.dumps({
        "workload": f"ctqw_torus_{L_SIDE}x{L_SIDE}_c64_{STEPS_PER_PASS}steps_snapshot_every_{every}",
        "snapshots": len(snaps), "compute_only_ms": t_comp * 1e3,
        "naive_states_ms": t_naive * 1e3, "streamed_states_ms": t_state * 1e3,
        "streamed_probabilities_ms": t_prob * 1e3,
        "streamed_overhead_vs_compute": t_state / t_comp - 1.0,
        "naive_overhead_vs_compute": t_naive / t_comp - 1.0,
        "states_MB": mb_state, "probabilities_MB": mb_prob,
        "streamed_states_GBps": mb_state / 1e3 / t_state, "link_copy_alone_GBps": mb_state / 1e3 / t_link,
        "memcpy_states_ms": t_ce * 1e3, "memcpy_probabilities_ms": t_ce_prob * 1e3,
        "memcpy_alone_GBps": mb_state / 1e3 / t_d2h,
        "streamed_equals_naive": same, "memcpy_equals_streamed": same_ce,
        "final_equals_unsnapshotted": final_ok,
        "arc_steps_per_s_streamed": g.n_arcs * STEPS_PER_PASS / t_state}), flush=True)


# ---------------------------------------------------------------- staggered lattice search

def run_staggered(args):
    """Staggered-walk search on the periodic L x L square lattice (default
    L = 4096, 2^24 vertices): two tessellations of 2 x 2 squares (corners at
    even and at odd coordinates), uniform amplitudes, reflection form, the
    centre vertex marked, uniform start.  One timed pass is --stag-steps steps
    (two steps per launch on the square-lattice kernels, the marked flip
    applied at every step), timed with HIP events on the launch stream; the
    readout follows outside the timed region.  3 steps from a random state are checked against the
    oracle at full size."""
    import numpy as np
    import torch

    import oracle
    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Plan
    side = args.stag_side
    g, tess = I.stag_lattice(side)
    marked = [(side // 2) * side + side // 2]
    steps = args.stag_steps
    psi0 = I.uniform(g.n)
    # the check starts from a random state: from the uniform one every
    # amplitude stays a short dyadic fraction and any path would be exact
    chk0 = I.random_state(g.n, 1)
    ref3 = oracle.staggered_evolve(g.n, tess, chk0, 3, marked=marked)
    res = {}
    for dtype in args.stag_dtypes.split(","):
        pl = Plan(g, "staggered", dtype=dtype, marked=marked, tessellations=tess, layout=args.stag_layout)
        psi = pl.state(chk0)
        pl.evolve(psi, 3)
        torch.cuda.synchronize()
        got3 = psi.cpu().numpy().astype(np.complex128)
        err3 = float(np.abs(got3 - ref3).max()) if dtype == "c128" else float(np.linalg.norm(got3 - ref3))
        psi = pl.state(psi0)
        pl.evolve(psi, 5)
        psi = pl.state(psi0)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        pl.evolve(psi, steps)
        b.record()
        p, norm, pm = pl.probabilities(psi)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        es = 8 if dtype == "c64" else 16
        if pl.structure == "stag_lattice":
            # the fused square-lattice kernels: per step, read and write every
            # amplitude once (2 S), no index; two steps run per launch, so the
            # DRAM traffic is half of this model and frac can pass 0.5 of it
            per_vertex = 2 * es
        else:
            # one launch per tessellation: read and write every amplitude (2 S)
            # and read its vertex index (4 B; the squares are one size, so no
            # polygon pointers and no amplitudes are stored), twice per step
            per_vertex = 2 * (2 * es + 4)
        step_ms = ms / steps
        gbs = per_vertex * g.n / (step_ms * 1e-3) / 1e9
        res[dtype] = {"vertex_steps_per_s": g.n * steps / (ms * 1e-3), "ms": ms, "step_us": step_ms * 1e3,
                      "bytes_per_vertex_step": per_vertex, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
                      "p_marked": float(pm), "norm": float(norm), "path": pl.structure,
                      ("max_abs_err_3_steps" if dtype == "c128" else "l2_err_3_steps"): err3}
        res[dtype]["state"] = psi
        pl.close()
    out = {k: {kk: vv for kk, vv in v.items() if kk != "state"} for k, v in res.items()}
    if "c64" in res and "c128" in res:
        out["l2_c64_vs_c128"] = float(torch.linalg.norm(res["c64"]["state"].to(torch.complex128)
                                                        - res["c128"]["state"]).item())
    print(json.dumps({"workload": f"staggered_lattice_{side}x{side}_squares_{steps}steps", "n": g.n,
                      "tessellations": len(tess), "unit": "vertex-steps/s", **out}), flush=True)


# ---------------------------------------------------------------- lattice walk (position-coin notation)

def run_lattice(args):
    """Coined walk on the periodic L x L grid (default L = 2048, 2^22
    vertices, 2^24 arcs) in position-coin notation: rows in direction order
    (c+1, c-1, r+1, r-1), the 4 x 4 Fourier coin and the persistent shift,
    started with amplitude 1/2 on the four arcs of the centre vertex.  One
    timed pass is --lattice-steps steps (one launch each, plus the layout
    permutation in and out of the call), timed with HIP events on the launch
    stream.  3 steps from a random state are checked against the oracle at
    full size."""
    import numpy as np
    import torch

    import oracle
    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Coined
    side = args.lattice_side
    g = I.torus_directed(side, side)
    steps = args.lattice_steps
    v0 = (side // 2) * side + side // 2
    psi0 = np.zeros(g.n_arcs, dtype=np.complex128)
    psi0[g.row_ptr[v0]:g.row_ptr[v0 + 1]] = 0.5
    chk0 = I.random_state(g.n_arcs, 2)
    ref3 = oracle.coined_evolve_general(g.row_ptr, g.col, chk0, 3, coin="fourier", shift="persistent",
                                        dims=(side, side))
    res = {}
    for dtype in ("c64", "c128"):
        w = Coined(g, shift="persistent", coin="fourier", dtype=dtype)
        pl = w.plan
        x = pl.state(chk0)
        pl.evolve(x, 3)
        torch.cuda.synchronize()
        got3 = x.cpu().numpy().astype(np.complex128)
        err3 = float(np.abs(got3 - ref3).max()) if dtype == "c128" else float(np.linalg.norm(got3 - ref3))
        del x
        psi = pl.state(psi0)
        pl.evolve(psi, 4)
        psi = pl.state(psi0)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        pl.evolve(psi, steps)
        b.record()
        p, norm, _ = pl.probabilities(psi)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        es = 8 if dtype == "c64" else 16
        # algorithmic bytes per arc-step of the slot-major kernel: read and write
        # the state (2S); the coin is 16 complex numbers read by every workgroup
        step_ms = ms / steps
        gbs = 2 * es * g.n_arcs / (step_ms * 1e-3) / 1e9
        res[dtype] = {"arc_steps_per_s": g.n_arcs * steps / (ms * 1e-3), "ms": ms, "step_us": step_ms * 1e3,
                      "bytes_per_arc_step": 2 * es, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
                      "norm": float(norm), "path": pl.structure,
                      ("max_abs_err_3_steps" if dtype == "c128" else "l2_err_3_steps"): err3}
        del psi
        pl.close()
    print(json.dumps({"workload": f"coined_fourier_persistent_grid_{side}x{side}_{steps}steps", "n": g.n,
                      "arcs": g.n_arcs, "unit": "arc-steps/s", **res}), flush=True)


# ---------------------------------------------------------------- CTQW on random sparse graphs

def run_sparse(args):
    """CTQW search on two random sparse graphs of 2^20 vertices through the
    general kernels: Erdos-Renyi G(N, 8/(N-1)) (irregular: CSR rows, lanes per
    row by mean degree) and a random 6-regular graph (column-major neighbour
    table, no row pointers).  gamma = 1/mean degree, dt = 1/||H||_inf, K from
    the truncation rule (tolerance 1e-8 over the pass), vertex 0 marked,
    uniform start, 50 steps per timed pass (HIP events on the launch stream).
    2 steps from a random state are checked against the oracle at full size.
    Algorithmic bytes per row-stage: 4 (row pointer, CSR only) + 4 d (column
    indices) + 3 S (gathered y, psi, y out), with each gathered value counted
    once; random neighbours make each gather move a whole cache line."""
    import numpy as np
    import torch

    import oracle
    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Plan
    n = 1 << 20
    steps = 50
    graphs = [("er", I.erdos_renyi(n, 8 / (n - 1), seed=3), 8.0), ("rr6", I.random_regular(n, 6, seed=4), 6.0)]
    out = {}
    for name, g, dbar in graphs:
        dmax = int(np.diff(g.row_ptr).max())
        gamma = 1.0 / dbar
        dt = 1.0 / (gamma * dmax + 1.0)
        chk0 = I.random_state(g.n, 5)
        res = {"arcs": g.n_arcs, "max_degree": dmax}
        for dtype in ("c64", "c128"):
            pl = Plan(g, "ctqw", dtype=dtype, gamma=gamma, dt=dt, taylor_order=0, trunc_tol=1e-8,
                      horizon_steps=steps, marked=[0], layout="auto")
            K = int(pl.info.taylor_order)
            if dtype == "c128":
                ref2 = oracle.ctqw_evolve(g.row_ptr, g.col, chk0, 2, gamma=gamma, dt=dt, K=K, marked=[0])
                x = pl.state(chk0)
                pl.evolve(x, 2)
                torch.cuda.synchronize()
                res["max_abs_err_2_steps"] = float(np.abs(x.cpu().numpy() - ref2).max())
                del x
            psi = pl.state(I.uniform(g.n))
            pl.evolve(psi, 2)
            psi = pl.state(I.uniform(g.n))
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            pl.evolve(psi, steps)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            es = 8 if dtype == "c64" else 16
            per_launch = (4 * g.n if pl.structure == "general" else 0) + 4 * g.n_arcs + 3 * es * g.n
            launch_ms = ms / (steps * K)
            gbs = per_launch / (launch_ms * 1e-3) / 1e9
            res[dtype] = {"path": pl.structure, "K": K, "arc_steps_per_s": g.n_arcs * steps / (ms * 1e-3),
                          "arc_spmv_per_s": g.n_arcs * steps * K / (ms * 1e-3), "stage_us": launch_ms * 1e3,
                          "bytes_per_stage": per_launch, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
            del psi
            pl.close()
        out[name] = res
    print(json.dumps({"workload": "ctqw_search_sparse_random_2^20", "steps": steps, **out}), flush=True)


# ---------------------------------------------------------------- out-of-core (streamed) CTQW

def run_streamed(args):
    """Out-of-core CTQW: a CTQW search on G(N, d/(N-1)) whose neighbour table
    (4 bytes per arc) stays in pinned host memory, under a device budget of the
    state and workspace plus --stream-budget-mib, in both modes: direct (the
    device keeps what fits of the table, the stage kernel reads the rest from
    host memory itself) and ring (the table streams through a ring of device
    slots at every Horner stage, the copies overlapping the stage kernels).
    Timed beside the same walk in core (stage kernels only) and the ring's
    copies alone (same tiles, same count)."""
    import numpy as np
    import torch

    import oracle
    from paper_2406_08186_amd import _lib as L
    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Plan

    n, dbar, steps = args.stream_n, args.stream_degree, args.stream_steps
    t0 = time.perf_counter()
    g = I.erdos_renyi(n, dbar / (n - 1), seed=11)
    print(f"[streamed] graph n={g.n} arcs={g.n_arcs} in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    gamma = 1.0 / dbar
    dmax = int(np.diff(g.row_ptr).max())
    dt = 1.0 / (gamma * dmax + 1.0)
    K = L.qw_taylor_order(1.0, steps, 1e-8)
    params = dict(gamma=gamma, dt=dt, taylor_order=K, marked=[0])
    psi0 = I.uniform(g.n)
    stages = steps * K
    host_ms = {}

    def timed(pl, psi):
        pl.evolve(psi, 1)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        t1 = time.perf_counter()
        pl.evolve(psi, steps)
        host_ms[id(pl)] = (time.perf_counter() - t1) * 1e3  # enqueue time on the host
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    core = Plan(g, "ctqw", dtype="c64", layout="csr", **params)
    x = core.state(psi0)
    ms_core = timed(core, x)
    core.evolve(x, 0)
    ref_gpu = x.cpu().numpy()
    walk = core.info.state_bytes + core.info.work_bytes
    core.close()
    del core
    budget = walk + args.stream_budget_mib * 2**20
    modes = {}
    states = {}
    for mode in ("direct", "ring"):
        pl = Plan(g, "ctqw", dtype="c64", layout="csr", upload=False, **params)
        sizes = pl.upload_streamed(budget, mode=mode)
        y = pl.state(psi0)
        ms = timed(pl, y)
        states[mode] = y
        modes[mode] = {"sizes": sizes, "ms": ms, "host_ms": host_ms[id(pl)],
                       "diff_vs_in_core": float(np.abs(y.cpu().numpy() - ref_gpu).max()), "plan": pl}
    # direct: every stage reads the table's host part across the link
    d = modes["direct"]
    host_part = 4 * (g.n_arcs - d["sizes"]["device_arcs"])
    # ring: the tiles the streamed call copies, in the same sizes, from pinned memory to
    # a device ring.  The call copies every tile at its first stage; each later stage
    # starts with the tiles the ring still holds (alternating tile order) and copies the
    # others.
    r = modes["ring"]
    tiles = r["sizes"]["tiles"]
    hits = min(3, tiles)
    copies = tiles + (stages - 1) * (tiles - hits)
    tile_bytes = 4 * g.n_arcs // max(1, tiles)
    ring = torch.empty(3 * max(tile_bytes, 256), dtype=torch.uint8, device="cuda")
    host = r["plan"].h_graph
    cs = torch.cuda.Stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(cs):
        a.record()
        for st in range(stages):
            for t in range(tiles if st == 0 else tiles - hits):
                lo = t * tile_bytes
                hi = min(4 * g.n_arcs, lo + tile_bytes)
                ring[(t % 3) * tile_bytes:(t % 3) * tile_bytes + (hi - lo)].copy_(host[lo:hi], non_blocking=True)
        b.record()
    torch.cuda.synchronize()
    ms_copy = a.elapsed_time(b)
    # parity: both streamed states against the oracle (c64 L2), and against each other
    t1 = time.perf_counter()
    ref = oracle.ctqw_evolve(g.row_ptr, g.col, psi0, steps + 1, **{k: v for k, v in params.items()
                                                                     if k != "taylor_order"}, K=K)
    l2 = {m: float(np.linalg.norm(states[m].cpu().numpy().astype(np.complex128) - ref)) for m in states}
    copied = copies * tile_bytes  # tiles of about the average size
    line = {"workload": f"ctqw_search_er_{g.n}_d{dbar}_out_of_core", "dtype": "c64", "n": g.n, "arcs": g.n_arcs,
            "K": K, "steps": steps, "device_budget_bytes": budget, "table_bytes_in_host_memory": 4 * g.n_arcs,
            "stage_ms_in_core": ms_core / stages,
            "direct": {"device_graph_bytes": d["sizes"]["device_bytes"],
                       "device_arcs": d["sizes"]["device_arcs"], "workgroup_tiles": d["sizes"]["tiles"],
                       "host_bytes_read_per_stage": host_part,
                       "stage_ms": d["ms"] / stages, "stage_ms_host_enqueue": d["host_ms"] / stages,
                       "host_read_gbs": host_part * stages / (d["ms"] * 1e-3) / 1e9,
                       "table_gbs": 4 * g.n_arcs * stages / (d["ms"] * 1e-3) / 1e9,
                       "arc_steps_per_s": g.n_arcs * steps / (d["ms"] * 1e-3),
                       "max_abs_diff_vs_in_core": d["diff_vs_in_core"], "l2_vs_oracle": l2["direct"]},
            "ring": {"device_graph_bytes": r["sizes"]["device_bytes"], "tiles_per_stage": tiles,
                     "stage_ms": r["ms"] / stages, "stage_ms_copies_only": ms_copy / stages,
                     "stage_ms_host_enqueue": r["host_ms"] / stages,
                     "tile_copies_per_call": copies, "tiles_held_by_the_ring": hits,
                     "h2d_bytes_per_stage_approx": copied / stages,
                     "table_gbs": 4 * g.n_arcs * stages / (r["ms"] * 1e-3) / 1e9,
                     "h2d_gbs": copied / (r["ms"] * 1e-3) / 1e9,
                     "h2d_gbs_copies_only": copied / (ms_copy * 1e-3) / 1e9,
                     "arc_steps_per_s": g.n_arcs * steps / (r["ms"] * 1e-3),
                     "max_abs_diff_vs_in_core": r["diff_vs_in_core"], "l2_vs_oracle": l2["ring"]},
            "direct_equals_ring_bitwise": bool(torch.equal(states["direct"], states["ring"])),
            "arc_steps_per_s_in_core": g.n_arcs * steps / (ms_core * 1e-3),
            "oracle_s": time.perf_counter() - t1}
    for m in modes.values():
        m["plan"].close()
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- 64-cycle latency

def run_cycle(args):
    """The 64-cycle Hadamard walk from (|0,0> + i|0,1>)/sqrt2, 100 steps, complex128,
    with the FP64 readout: one call runs the whole walk in one workgroup's LDS.
    Reports the per-call latency distribution (host clock around a synchronised call,
    and HIP events on the stream)."""
    import numpy as np
    import torch

    from paper_2406_08186_amd import inputs as I
    from paper_2406_08186_amd.walk import Plan
    g, psi0 = I.cycle_hadamard_state(64)
    pl = Plan(g, "coined", coin="hadamard", dtype="c128")
    psi = pl.state(psi0)
    for _ in range(50):
        psi.copy_(pl.state(psi0))
        pl.evolve(psi, 100, readout=True)
    torch.cuda.synchronize()
    host, dev = [], []
    reps = 1000
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record()
        pl.evolve(psi, 100, readout=True)
        b.record()
        b.synchronize()
        host.append((time.perf_counter() - t0) * 1e3)
        dev.append(a.elapsed_time(b))
    host.sort()
    dev.sort()
    print(json.dumps({"workload": "coined_hadamard_cycle64_100steps", "dtype": "c128", "path": pl.structure,
                      "calls": reps, "host_p50_ms": pct(host, 50), "host_p99_ms": pct(host, 99),
                      "device_p50_ms": pct(dev, 50), "device_p99_ms": pct(dev, 99),
                      "arc_steps_per_s_p50": g.n_arcs * 100 / (pct(dev, 50) * 1e-3)}), flush=True)


if __name__ == "__main__":
    main()
