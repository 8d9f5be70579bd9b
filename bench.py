"""Benchmark of the MacLABSWE step on one MI355X.

Workload: subcritical flow over a Gaussian bump in a 4096 x 4096 channel
(dx = 1 m, 2 m still depth, inflow discharge 4.42 m^2/s on the west edge,
fixed 2 m depth on the east edge, walls north and south), FP32 fields.
One "step" is one MacLABSWE time step over the whole lattice.

Prints one JSON line: MLUPS (million lattice updates per second), the HBM
roofline block of the step kernel and the FP64 oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published peak
BYTES_PER_LUP = 28             # read eta, qx, qy, H; write eta, qx, qy (FP32) once per launch
# FP32 vector peak usable by these kernels: 256 CUs x 64 lanes x 2 (FMA) x 2.4 GHz.
# (The published 157.3 TFLOP/s counts packed FP32, which this build does not emit.)
FP32_PEAK_TFLOPS = 78.6
# Algorithmic FP32 operations per node update (FMA = 2, rcp / sqrt = 1 each):
# derive 48 (41 without bed friction), row partial sums 8, links 12, update 34,
# carried link sums 2.
FLOP_PER_LUP = {True: 104, False: 97}
FLOP_IMPLICIT = 5              # implicit link depth: scale the increment, correct qx and qy (two FMAs)
KERNEL_SRC = os.path.join(ROOT, "paper_1902_02999_amd", "csrc", "mlb_kernels.hip")
TRAFFIC_FILES = {1: os.path.join(ROOT, "profiles", "step_kernel_bump4096_traffic.json"),
                 2: os.path.join(ROOT, "profiles", "step2_kernel_bump4096_traffic.json"),
                 "implicit": os.path.join(ROOT, "profiles", "step_kernel_implicit_bump4096_traffic.json"),
                 "implicit2": os.path.join(ROOT, "profiles", "step2_kernel_implicit_bump4096_traffic.json"),
                 "dish4096": os.path.join(ROOT, "profiles", "step_kernel_masked_dish4096_traffic.json"),
                 "dish4096_2": os.path.join(ROOT, "profiles", "step2_kernel_masked_dish4096_traffic.json"),
                 "ensemble": os.path.join(ROOT, "profiles", "step2_kernel_closed_ensemble512_traffic.json"),
                 "elab": os.path.join(ROOT, "profiles", "elab_step_kernel_lake4096_traffic.json")}


def roofline_of(bytes_per_launch: float, flop_per_launch: float, launch_s: float, traffic):
    """Roofline of the dominant kernel from its algorithmic bytes and FP32
    operations per launch: HBM-bound where the arithmetic intensity lies
    below the ridge point (peak FP32 rate over peak HBM rate, 9.8 FLOP/B),
    ALU-bound above it.  Also returns the achieved FP32 rate in TFLOP/s."""
    gbs = bytes_per_launch / launch_s / 1e9
    tfl = flop_per_launch / launch_s / 1e12
    if flop_per_launch / bytes_per_launch < FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9):
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic}
    else:
        r = {"bound": "alu", "achieved": round(tfl, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
             "frac": round(tfl / FP32_PEAK_TFLOPS, 4), "traffic": traffic}
    return r, round(tfl, 2)


def traffic_rate(traffic, launch_s: float):
    """HBM rate [GB/s] of the measured bytes per launch (None without a
    counter summary for this kernel and size)."""
    return None if traffic is None else round(traffic / launch_s / 1e9, 1)


def measured_traffic(nodes: int, key, tile_rows=None):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summaries, or None when none was taken on this kernel
    source, problem size and (where the summary records it) tile height."""
    from paper_1902_02999_amd.profiling import kernel_sha
    files = TRAFFIC_FILES.get(key)
    for path in ([files] if isinstance(files, str) else files or []):
        try:
            with open(path) as f:
                t = json.load(f)
            src = os.path.join(ROOT, "paper_1902_02999_amd", "csrc", t.get("kernel_source", "mlb_kernels.hip"))
            sha = kernel_sha(src)
        except (OSError, ValueError, KeyError):
            continue
        if t.get("kernel_sha") != sha or t.get("nodes") != nodes:
            continue
        if tile_rows is not None and t.get("tile_rows") not in (None, tile_rows):
            continue
        return t.get("bytes_per_launch")
    return None


def timed_steps(ctx, obj, warmup: int, steps: int):
    """W warm-up steps, the timed call's plan warmed up untimed (a call of the
    same length: its graph of passes is captured there), then exactly `steps`
    steps timed between synchronisations.  Returns the wall time, the HIP
    event time of the whole call [ms] and (ms per pass, passes, steps per
    pass) of its bulk passes timed alone on the library stream (None when the
    call has no bulk pass)."""
    import torch
    if warmup:
        obj.step(warmup)
    obj.step(steps)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obj.step(steps)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ctx.last_step_ms()
    try:
        bulk = ctx.last_pass_ms()
    except Exception:
        bulk = None
    return wall, ev_ms, bulk


def cpu_baseline(spec, budget_s: float = 12.0):
    """The FP64 oracle (as is) on the host cores: steps of the same workload
    until the time budget is spent, on all cores (the reported value) and then
    on one thread for a third of the budget."""
    import oracle

    def rate(threads, budget):
        b = oracle.from_spec(spec)
        b.threads = threads
        t0 = time.perf_counter()
        n = 0
        while True:
            b.run(1)
            n += 1
            if time.perf_counter() - t0 >= budget:
                break
        return n, time.perf_counter() - t0

    threads = oracle.default_threads()
    n, dt = rate(threads, budget_s)
    n1, dt1 = rate(1, budget_s / 3)
    return {"value": round(spec.nodes * n / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": "%d step(s) of the %dx%d workload, FP64, %.1f s" % (n, spec.nx, spec.ny, dt),
            "value_1_thread": round(spec.nodes * n1 / dt1 / 1e6, 3),
            "sample_1_thread": "%d step(s), %.1f s" % (n1, dt1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=4096, help="lattice side")
    ap.add_argument("--tile-rows", type=int, default=15)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-warm", action="store_true",
                    help="bump: skip the small warm-vs-cold start measurement added to the default line")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run the plain copy kernel on this many MiB and print GB/s")
    ap.add_argument("--blocks-per-cu", type=int, default=3)
    ap.add_argument("--persistent", type=int, default=0, choices=[0, 1, 2],
                    help="when not autotuning: 0 one launch per pass, 1 cooperative grid barrier, 2 work queue")
    ap.add_argument("--tblock", type=int, default=1, choices=[1, 2],
                    help="steps per kernel pass when not autotuning")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (by default it picks tile rows and the CU cap before timing)")
    ap.add_argument("--workload", default="bump",
                    choices=["bump", "ensemble", "lake_steady", "warm_start", "dish", "dish4096", "hump", "elab",
                             "net"],
                    help="bump: 4096^2 channel (default line); ensemble: 512 basins 64^2..512^2 in "
                         "one launch per step; lake_steady: 256^2 wind lake to residual 1e-6; "
                         "warm_start: learned warm start vs cold start on held-out 256^2 basins; "
                         "dish: the paper's circular wind-driven basin (200^2, node mask) with its "
                         "time to steady state; dish4096: the same basin on 4096^2 nodes; "
                         "hump: the paper's 2D hump channel (200^2) with its time to steady state; "
                         "elab: the eLABSWE baseline (nine stored distributions) against the streaming-only "
                         "step on a closed 4096^2 basin; net: the warm-start network's forward pass and "
                         "training step (256^2, batch 8) against the BF16 MFMA roofline")
    ap.add_argument("--implicit", action="store_true",
                    help="bump: the implicit link depth (new-time depth at the node; 12 more bytes per node "
                         "per pass, 5 more FP32 operations per update)")
    ap.add_argument("--compensated", action="store_true",
                    help="bump: surface stored as a compensated FP32 pair (one step per pass, 8 more bytes per node)")
    ap.add_argument("--elab-tile-rows", type=int, default=0,
                    help="elab: tile rows of the eLABSWE baseline (0: the fastest of 6, 9, 12, 15)")
    ap.add_argument("--pcie", action="store_true",
                    help="bump: also time the same steps with the state handed over in host memory "
                         "(FP64 upload before, download after) and report that rate in config; "
                         "value stays the HBM-resident rate")
    ap.add_argument("--net", default=None, help="warm_start: load this trained net instead of training")
    ap.add_argument("--ws-train", type=int, default=512, help="warm_start: training basins")
    ap.add_argument("--ws-epochs", type=int, default=40, help="warm_start: training epochs")
    ap.add_argument("--ws-held-out", type=int, default=20, help="warm_start: held-out basins timed")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the step runs on a single MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1902_02999_amd import mlb, workloads as wl

    ctx = mlb.Context(0)
    if args.copy_probe_mib:
        gbps = ctx.copy_probe(args.copy_probe_mib << 20, reps=5)
        print(json.dumps({"copy_probe_bytes": args.copy_probe_mib << 20, "GBps": round(gbps, 1)}), flush=True)
        ctx.close()
        return
    copy_gbps = ctx.copy_probe(1 << 30, reps=10)
    if args.workload == "ensemble":
        return bench_ensemble(args, ctx, copy_gbps)
    if args.workload == "lake_steady":
        return bench_lake_steady(args, ctx)
    if args.workload == "warm_start":
        return bench_warm_start(args, ctx)
    if args.workload in ("dish", "dish4096", "hump"):
        return bench_geometry(args, ctx, copy_gbps)
    if args.workload == "elab":
        return bench_elab(args, ctx, copy_gbps)
    if args.workload == "net":
        return bench_net(args, ctx)
    spec = wl.bump_channel(args.n)
    spec.hbar_implicit = args.implicit
    spec.compensated = args.compensated
    grid = mlb.grid_from_spec(ctx, spec)
    grid.set_exec_opts(tile_rows=args.tile_rows, use_graph=not args.no_graph, graph_chunk=100,
                       blocks_per_cu=args.blocks_per_cu, tblock=args.tblock, persistent=args.persistent)
    tuned = None if args.no_autotune else grid.autotune(steps=40)

    wall, ev_ms, bulk = timed_steps(ctx, grid, args.warmup, args.steps)
    d = grid.diag()
    if d["nonfinite"]:
        print("bench.py: non-finite state after the timed steps", file=sys.stderr)
        sys.exit(1)

    nodes = spec.nodes
    mlups = nodes * args.steps / wall / 1e6
    pcie = None
    if args.pcie:
        # host FP64 state in, the same steps, host FP64 state out
        h0, qx0, qy0 = spec.initial()
        ctx.sync()
        t1 = time.perf_counter()
        grid.set_state(h0, qx0, qy0)
        ctx.sync()
        t2 = time.perf_counter()
        grid.step(args.steps)
        ctx.sync()
        t3 = time.perf_counter()
        grid.get_state()
        t4 = time.perf_counter()
        pcie = {"MLUPS": round(nodes * args.steps / (t4 - t1) / 1e6, 1), "upload_ms": round((t2 - t1) * 1e3, 2),
                "steps_ms": round((t3 - t2) * 1e3, 2), "download_ms": round((t4 - t3) * 1e3, 2)}
    # Dominant kernel: the call's bulk passes (one or two steps each), timed
    # alone on the library stream; without them, the whole call per step.
    if bulk is not None:
        launch_s, tb = bulk[0] / 1e3, bulk[2]
    else:
        tb = 1
        launch_s = ev_ms / 1e3 / args.steps
    # + 1/(1+kappa), kappa_x, kappa_y; + the low part of eta read and written
    bpl = BYTES_PER_LUP + (12 if args.implicit else 0) + (8 if args.compensated else 0)
    gbs = bpl * nodes / launch_s / 1e9
    traffic = None if args.compensated else measured_traffic(nodes, ("implicit" if tb == 1 else "implicit2")
                                                             if args.implicit else tb, grid.exec_opts().tile_rows)
    flop = FLOP_PER_LUP[spec.chezy > 0] + (FLOP_IMPLICIT if args.implicit else 0)
    roofline, tfl = roofline_of(bpl * nodes, flop * tb * nodes, launch_s, traffic)
    out = {
        "metric": "MLUPS",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "nodes": nodes, "dx_m": spec.dx, "dt_s": spec.dx / (6 * spec.nu / spec.dx),
                   "tile_rows": grid.exec_opts().tile_rows, "blocks_per_cu": grid.exec_opts().blocks_per_cu,
                   "tblock": grid.exec_opts().tblock, "hbar": "implicit" if args.implicit else "eq_h-bar",
                   "surface": "compensated" if args.compensated else "fp32",
                   "autotuned": tuned is not None, "graph": not args.no_graph, "fp32_TFLOPs": tfl,
                   # per-step bytes of the one-step formulation x update rate
                   "effective_GBps": round(mlups * 1e6 * bpl / 1e9, 1),
                   "launch_GBps": round(gbs, 1), "traffic_GBps": traffic_rate(traffic, launch_s),
                   "launch_us": round(launch_s * 1e6, 3),
                   "bulk_passes": None if bulk is None else bulk[1], "call_event_ms": round(ev_ms, 4),
                   "copy_probe_GBps": round(copy_gbps, 1)},
        "roofline": roofline,
    }
    if pcie is not None:
        out["config"]["host_state_inclusive"] = pcie
    grid.close()
    ctx.close()
    if not args.no_warm:
        out["config"]["warm_vs_cold"] = warm_vs_cold_small()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def warm_vs_cold_small():
    """The other half of the metric at a size that fits the default run
    (about ten seconds): a three-level warm-start net trained from scratch
    here, by the library's kernels, on the steady states of 128 closed 128^2
    basins of the ensemble distributions (seed 2999), then wall seconds to
    R <= 1e-6 warm (inference included) against cold on 12 held-out basins
    (seed 3000).  The full-size experiment is --workload warm_start."""
    from paper_1902_02999_amd import mlb, warmstart as ws, workloads as wl
    ctx = mlb.Context(0)
    n = 128
    net = mlb.Net(ctx, n, n, base_ch=32, levels=3, in_ch=32, max_batch=8, seed=2999)
    t0 = time.perf_counter()
    data = ws.build_dataset(ctx, net, wl.learned_set(128, 2999, n=n), 1e-6, log=lambda *a: None)
    for g in data.grids:
        g.close()
    data.grids = []
    losses = ws.train(net, data, ws.TrainSpec(epochs=40, batch=8, lr=2e-3, lr_min=1e-5, warmup_steps=20),
                      log=lambda *a: None)
    train_s = time.perf_counter() - t0
    del data
    rows = ws.evaluate(ctx, net, wl.learned_set(12, 3000, n=n), 1e-6, log=lambda *a: None)
    sm = ws.summary(rows)
    net.close()
    ctx.close()
    return {"workload": "learned_warm_start_128 (3-level net, 128 training basins, 40 epochs, 12 held-out)",
            "cold_s": round(sm["cold_s_total"], 4), "warm_s": round(sm["warm_s_total"], 4),
            "speedup": round(sm["speedup_total"], 3), "cold_steps_median": sm["cold_steps_median"],
            "warm_steps_median": sm["warm_steps_median"], "fallbacks": sm["fallbacks"],
            "train_s": round(train_s, 1), "loss": [round(losses[0], 4), round(losses[-1], 4)]}


def bench_ensemble(args, ctx, copy_gbps):
    """512 closed basins (sizes 64^2..512^2, seed 1902) in one launch per step."""
    import torch
    from paper_1902_02999_amd import mlb, workloads as wl
    specs = wl.ensemble(512, 1902)
    grids = [mlb.grid_from_spec(ctx, s) for s in specs]
    nodes = sum(s.nodes for s in specs)
    b = mlb.Batch(ctx, grids)
    b.set_exec_opts(tile_rows=args.tile_rows, use_graph=not args.no_graph, graph_chunk=100,
                    blocks_per_cu=args.blocks_per_cu, tblock=args.tblock, persistent=args.persistent)
    tuned = None if args.no_autotune else b.autotune(steps=30)
    opts = tuned or {"tile_rows": args.tile_rows, "tblock": args.tblock, "use_graph": int(not args.no_graph),
                     "graph_chunk": 100, "blocks_per_cu": args.blocks_per_cu, "persistent": args.persistent}
    wall, ev_ms, bulk = timed_steps(ctx, b, args.warmup, args.steps)
    ok, diags = b.run_steady(0.0, 1, 1)   # one checked step: finiteness of every basin
    bad = sum(d["nonfinite"] for d in diags)
    b.close()
    for g in grids:
        g.close()
    ctx.close()
    mlups = nodes * args.steps / wall / 1e6
    if bulk is not None:
        launch_s, tb = bulk[0] / 1e3, bulk[2]
    else:
        tb = 1
        launch_s = ev_ms / 1e3 / args.steps
    gbs = BYTES_PER_LUP * nodes / launch_s / 1e9
    traffic = measured_traffic(nodes, "ensemble", opts["tile_rows"]) if tb == 2 else None
    roofline, tfl = roofline_of(BYTES_PER_LUP * nodes, FLOP_PER_LUP[True] * tb * nodes, launch_s, traffic)
    print(json.dumps({
        "metric": "MLUPS", "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ensemble_512_basins_64-512_seed1902", "basins": len(specs), "nodes": nodes,
                   "exec": opts, "autotuned": tuned is not None, "nonfinite": bad, "copy_probe_GBps": round(copy_gbps, 1),
                   "effective_GBps": round(mlups * 1e6 * BYTES_PER_LUP / 1e9, 1), "launch_GBps": round(gbs, 1),
                   "traffic_GBps": traffic_rate(traffic, launch_s),
                   "launch_us": round(launch_s * 1e6, 3), "fp32_TFLOPs": tfl},
        "roofline": roofline,
        "cpu_baseline": None if args.no_cpu else cpu_baseline_ensemble(specs, args.cpu_seconds)}), flush=True)


def cpu_baseline_ensemble(specs, budget_s: float = 12.0):
    """The FP64 oracle on a fixed sample of the ensemble's basins (every
    32nd, 16 basins of the same size distribution), stepped round-robin until
    the budget is spent, on all cores and then on one thread."""
    import oracle
    sample = specs[::32]
    nodes = sum(sp.nodes for sp in sample)

    def rate(threads, budget):
        bs = [oracle.from_spec(sp) for sp in sample]
        for bb in bs:
            bb.threads = threads
        t0 = time.perf_counter()
        n = 0
        while True:
            for bb in bs:
                bb.run(1)
            n += 1
            if time.perf_counter() - t0 >= budget:
                break
        return n, time.perf_counter() - t0

    threads = oracle.default_threads()
    n, dt = rate(threads, budget_s)
    n1, dt1 = rate(1, budget_s / 3)
    return {"value": round(nodes * n / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d step(s) of %d of the 512 basins (every 32nd, %d nodes), FP64, %.1f s"
                      % (n, len(sample), nodes, dt),
            "value_1_thread": round(nodes * n1 / dt1 / 1e6, 3),
            "sample_1_thread": "%d step(s), %.1f s" % (n1, dt1)}


def bench_geometry(args, ctx, copy_gbps):
    """The paper's own geometries (Section 4).  Throughput of `steps` steps
    counted over the water nodes (SOLID nodes of the circular basin's mask
    are not updated), the dominant kernel's HBM roofline at 28 B per water
    node plus 1 B per node kind read, and for the 200^2 cases the wall time
    from rest to a per-step residual of 1e-6."""
    import numpy as np
    import torch
    from paper_1902_02999_amd import mlb, workloads as wl
    if args.workload == "hump":
        spec = wl.hump_channel()
    else:
        n = 4096 if args.workload == "dish4096" else 200
        spec = wl.circular_dish(n, 400.0 / n)
    water = spec.nodes if spec.kind is None else int((spec.kind != wl.SOLID).sum())
    kind_bytes = 0 if spec.kind is None else 1
    g = mlb.grid_from_spec(ctx, spec)
    g.set_exec_opts(tile_rows=args.tile_rows, use_graph=not args.no_graph, graph_chunk=100,
                    blocks_per_cu=args.blocks_per_cu, tblock=args.tblock)
    tuned = None if args.no_autotune else g.autotune(steps=40)
    wall, ev_ms, bulk = timed_steps(ctx, g, args.warmup, args.steps)
    d = g.diag()
    opts = g.exec_opts().as_dict()
    g.close()
    if bulk is not None:
        launch_s, tb = bulk[0] / 1e3, bulk[2]
    else:
        tb = 1
        launch_s = ev_ms / 1e3 / args.steps
    bpl = (BYTES_PER_LUP + kind_bytes) * water
    traffic = (measured_traffic(water, args.workload if tb == 1 else "dish4096_2", opts["tile_rows"])
               if args.workload == "dish4096" else None)
    roofline, tfl = roofline_of(bpl, FLOP_PER_LUP[spec.chezy > 0] * tb * water, launch_s, traffic)
    steady = None
    if spec.nodes <= 200 * 200:
        g = mlb.grid_from_spec(ctx, spec)
        if tuned is not None:
            g.set_exec_opts(**{k: opts[k] for k in ("tile_rows", "tblock", "blocks_per_cu", "persistent")})
        g.set_exec_opts(graph_chunk=100)
        ctx.sync()
        t1 = time.perf_counter()
        ok, ds = g.run_steady(1e-6, 5_000_000, 2000)
        steady = {"converged": ok, "wall_s": round(time.perf_counter() - t1, 3), "steps": ds["step"],
                  "t_model_s": round(ds["t"], 1), "residual": ds["residual"], "max_speed": ds["max_speed"]}
        g.close()
    ctx.close()
    out = {"metric": "MLUPS", "value": round(water * args.steps / wall / 1e6, 1), "unit": "MLUPS",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(wall * 1e3 / args.steps, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": spec.name, "nodes": spec.nodes, "water_nodes": water, "dx_m": spec.dx,
                      "nu": spec.nu, "exec": opts, "autotuned": tuned is not None, "nonfinite": d["nonfinite"],
                      "launch_us": round(launch_s * 1e6, 3), "traffic_GBps": traffic_rate(traffic, launch_s),
                      "copy_probe_GBps": round(copy_gbps, 1), "fp32_TFLOPs": tfl, "steady_1e-6": steady},
           "roofline": roofline}
    out["cpu_baseline"] = None if args.no_cpu else cpu_baseline(spec, args.cpu_seconds)
    if out["cpu_baseline"] is not None and water != spec.nodes:
        cb = out["cpu_baseline"]
        cb["value"] = round(cb["value"] * water / spec.nodes, 3)
        cb["sample"] += " (water nodes only)"
    print(json.dumps(out), flush=True)


ELAB_BYTES_PER_LUP = 76   # read nine distributions and H, write nine (FP32)


def bench_elab(args, ctx, copy_gbps):
    """The storage claim on one GPU: the eLABSWE baseline (Eq. lb.1, nine
    FP32 distributions per node, tau = 1) and the streaming-only step on the
    same closed 4096^2 wind-driven basin, same tiles.  `value` is the
    baseline's rate; the streaming-only rate (autotuned, two steps per pass)
    and the ratio are in config."""
    import torch
    from paper_1902_02999_amd import mlb, workloads as wl
    spec = wl.wind_lake(args.n)
    g = mlb.grid_from_spec(ctx, spec)
    tuned = None if args.no_autotune else g.autotune(steps=40)
    g.step(args.warmup)
    ctx.sync()
    t0 = time.perf_counter()
    g.step(args.steps)
    ctx.sync()
    mac_wall = time.perf_counter() - t0
    # the streaming-only step with one step per pass (same tiles as the baseline's walk)
    g.set_exec_opts(tblock=1, tile_rows=15)
    g.step(args.warmup)
    ctx.sync()
    t0 = time.perf_counter()
    g.step(args.steps)
    ctx.sync()
    mac1_wall = time.perf_counter() - t0
    # tile rows of the baseline: the fastest of a few (50 steps each)
    tried = {}
    for tr in ((args.elab_tile_rows,) if args.elab_tile_rows else (6, 9, 12, 15)):
        g.set_exec_opts(tile_rows=tr)
        el = mlb.Elab(g, 1.0)
        el.step(10)
        ctx.sync()
        t1 = time.perf_counter()
        el.step(50)
        ctx.sync()
        tried[tr] = round((time.perf_counter() - t1) / 50 * 1e6, 2)
        el.close()
    best_tr = min(tried, key=tried.get)
    g.set_exec_opts(tile_rows=best_tr)
    tried = tried if len(tried) > 1 else None
    el = mlb.Elab(g, 1.0)
    el.step(args.warmup)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    el.step(args.steps)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ctx.last_step_ms()
    h, qx, qy = el.get_state()
    el.close()
    g.close()
    ctx.close()
    import numpy as np
    if not (np.isfinite(h).all() and np.isfinite(qx).all() and (h > 0).all()):
        print("bench.py: non-finite eLABSWE state", file=sys.stderr)
        sys.exit(1)
    nodes = spec.nodes
    launch_s = ev_ms / 1e3 / args.steps
    gbs = ELAB_BYTES_PER_LUP * nodes / launch_s / 1e9
    mlups = nodes * args.steps / wall / 1e6
    mac = nodes * args.steps / mac_wall / 1e6
    out = {"metric": "MLUPS", "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "elab_tau1_" + spec.name, "nodes": nodes, "tile_rows": best_tr,
                      "tile_rows_us_per_step": tried,
                      "streaming_only_MLUPS": round(mac, 1), "streaming_only_exec": tuned,
                      "streaming_only_over_elab": round(mac / mlups, 3),
                      "streaming_only_one_step_MLUPS": round(nodes * args.steps / mac1_wall / 1e6, 1),
                      "elab_bytes_per_node": ELAB_BYTES_PER_LUP, "launch_us": round(launch_s * 1e6, 2),
                      "copy_probe_GBps": round(copy_gbps, 1)},
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(nodes, "elab")},
           "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_lake_steady(args, ctx):
    """256^2 wind-driven dish lake from rest to a per-step residual of 1e-6."""
    from paper_1902_02999_amd import mlb, workloads as wl
    spec = wl.wind_lake(256)
    g = mlb.grid_from_spec(ctx, spec)
    tuned = None if args.no_autotune else g.autotune(steps=40)
    g.set_exec_opts(graph_chunk=98)
    ctx.sync()
    t0 = time.perf_counter()
    ok, d = g.run_steady(1e-6, 3_000_000, 100)
    wall = time.perf_counter() - t0
    g_opts = g.exec_opts().as_dict()
    g.close()
    ctx.close()
    print(json.dumps({"metric": "wall_s_to_residual_1e-6", "value": round(wall, 4), "unit": "s",
                      "higher_is_better": False, "converged": ok, "steps": d["step"],
                      "residual": d["residual"], "t_model_s": d["t"],
                      "config": {"workload": spec.name, "nodes": spec.nodes, "exec": g_opts}}), flush=True)


BF16_PEAK_TFLOPS = 2500.0       # MI355X dense BF16 MFMA, published


def net_layers(h: int, w: int, in_ch: int = 32, base_ch: int = 32, levels: int = 4, out_ch: int = 3):
    """(pixels, cin, cout, k) of every layer of the warm-start network in
    forward order: two 3x3 convolutions per encoder level, then per decoder
    level one after the upsampling and two after the skip concatenation, and
    the 1x1 head."""
    ch = [base_ch << l for l in range(levels)]
    px = [(h >> l) * (w >> l) for l in range(levels)]
    out, cin = [], in_ch
    for l in range(levels):
        out += [(px[l], cin, ch[l], 3), (px[l], ch[l], ch[l], 3)]
        cin = ch[l]
    for l in range(levels - 2, -1, -1):
        out += [(px[l], ch[l + 1], ch[l], 3), (px[l], 2 * ch[l], ch[l], 3), (px[l], ch[l], ch[l], 3)]
    out.append((px[0], ch[0], out_ch, 1))
    return out


def bench_net(args, ctx):
    """Forward pass and AdamW training step of the warm-start network at
    256^2, batch 8, random weights and inputs.  FLOPs count the
    convolutions' multiply-adds (2 per MAC); the roofline floor of a pass is
    the sum over layers of max(FLOPs / BF16 MFMA peak, activation bytes /
    HBM peak), activations in BF16, read once and written once."""
    import torch
    from paper_1902_02999_amd import mlb
    n, hw = 8, 256
    net = mlb.Net(ctx, hw, hw, base_ch=32, levels=4, in_ch=32, max_batch=n, seed=1)
    gen = torch.Generator().manual_seed(0)
    x = torch.randn((n, hw, hw, mlb.NET_FEATURES), generator=gen).cuda()
    t = torch.randn((n, hw, hw, 3), generator=gen).cuda()
    y = torch.empty((n, hw, hw, 3), device="cuda")
    torch.cuda.synchronize()
    for _ in range(3):
        net.forward(x, n, y)
    ctx.sync()
    reps = max(10, args.steps // 100)
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(x, n, y)
    ctx.sync()
    fwd = (time.perf_counter() - t0) / reps
    net.train(x, t, n, 1, n, 1e-4)
    ctx.sync()
    t0 = time.perf_counter()
    net.train(x, t, n, reps, n, 1e-4)
    ctx.sync()
    step = (time.perf_counter() - t0) / reps
    net.close()
    ctx.close()
    flop, floor = 0.0, 0.0
    for px, ci, co, k in net_layers(hw, hw):
        f = 2.0 * n * px * k * k * ci * co
        b = 2.0 * n * px * (ci + co)
        flop += f
        floor += max(f / (BF16_PEAK_TFLOPS * 1e12), b / (HBM_PEAK_GBS * 1e9))
    tfl = flop / fwd / 1e12
    print(json.dumps({
        "metric": "TFLOP/s", "value": round(tfl, 1), "unit": "TFLOP/s", "n_gpus": 1, "steps": reps,
        "warmup": 3, "ms_per_step": round(fwd * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 (fp32 accumulation)", "data": "synthetic",
        "config": {"workload": "warm_start_net_256_batch8", "forward_gflop": round(flop / 1e9, 1),
                   "forward_ms": round(fwd * 1e3, 3), "train_step_ms": round(step * 1e3, 3),
                   "roofline_floor_ms": round(floor * 1e3, 4), "of_floor": round(floor / fwd, 4)},
        "roofline": {"bound": "mfma", "achieved": round(tfl, 1), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tfl / BF16_PEAK_TFLOPS, 4), "traffic": None},
        "cpu_baseline": None}), flush=True)


def bench_warm_start(args, ctx):
    """Wall seconds to R <= 1e-6 on held-out 256^2 basins (seed 3000): cold
    start from rest vs the learned warm start (inference included), one basin
    at a time in graph mode, both under the same stall rule."""
    from paper_1902_02999_amd import mlb, warmstart as ws, workloads as wl
    spec = ws.NetSpec()
    net = mlb.Net(ctx, spec.n, spec.n, base_ch=spec.base_ch, levels=spec.levels, in_ch=spec.in_ch,
                  max_batch=spec.max_batch, seed=2999)
    train = {}
    if args.net:
        net.load(args.net)
        train["loaded"] = os.path.basename(args.net)
    else:
        data = ws.build_dataset(ctx, net, wl.learned_set(args.ws_train, 2999, n=spec.n), 1e-6,
                                log=lambda *a: print(*a, file=sys.stderr, flush=True))
        for g in data.grids:
            g.close()
        data.grids = []
        t0 = time.perf_counter()
        losses = ws.train(net, data, ws.TrainSpec(epochs=args.ws_epochs), log=lambda *a: None)
        train = {"basins": args.ws_train, "epochs": args.ws_epochs, "solve_s": round(data.solve_s, 1),
                 "train_s": round(time.perf_counter() - t0, 1), "loss_first": round(losses[0], 4),
                 "loss_last": round(losses[-1], 4)}
        del data
    rows = ws.evaluate(ctx, net, wl.learned_set(args.ws_held_out, 3000, n=spec.n), 1e-6,
                       log=lambda *a: None)
    sm = ws.summary(rows)
    net.close()
    ctx.close()
    print(json.dumps({"metric": "wall_s_to_residual_1e-6_warm", "value": round(sm["warm_s_total"], 3), "unit": "s",
                      "higher_is_better": False, "cold_s": round(sm["cold_s_total"], 3),
                      "speedup": round(sm["speedup_total"], 3), "speedup_median": round(sm["speedup_median"], 3),
                      "n_gpus": 1, "dtype": "f32 step, bf16 net (fp32 accumulation)", "data": "synthetic",
                      "config": {"workload": "learned_warm_start_256", "held_out": args.ws_held_out,
                                 "train": train, "summary": sm}}), flush=True)


if __name__ == "__main__":
    main()
