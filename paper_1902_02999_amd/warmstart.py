"""Learned warm start for steady-state runs: data, normalisation, training,
evaluation of warm against cold starts.

Every numerical step runs in the library's kernels (the step, the network's
MFMA forward / backward, AdamW, feature and target extraction, inference and
the warm-started run with its fallback); this module only orders the calls,
holds the device tensors and keeps the bookkeeping.

Data: closed square basins drawn from the ensemble distributions (random
bumps, wind speed and heading, Chezy coefficient), solved from rest to a
per-step discharge residual <= tol in one batched launch per step.  Inputs:
still-water depth, wind stress direction and magnitude, bed coefficient,
node position; targets: the steady (eta, hu, hv) divided per basin by the
stress magnitude (set-up and circulation grow with it) and by the spread of
the training set.
"""
from __future__ import annotations

import json
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import mlb
from . import workloads as wl


@dataclass
class NetSpec:
    n: int = 256
    base_ch: int = 32
    levels: int = 4
    in_ch: int = 32
    max_batch: int = 8


@dataclass
class TrainSpec:
    epochs: int = 40
    batch: int = 8
    lr: float = 1e-3
    lr_min: float = 1e-5
    warmup_steps: int = 100
    weight_decay: float = 1e-4
    seed: int = 2999


@dataclass
class Dataset:
    specs: List[wl.Spec]
    grids: List[mlb.Grid]
    steps: List[int]
    solve_s: float
    x: object = None      # torch CUDA [n, h, w, mlb.NET_FEATURES]
    t: object = None      # torch CUDA [n, h, w, 3]
    norm: dict = field(default_factory=dict)


def solve_steady(ctx: mlb.Context, specs: List[wl.Spec], tol: float = 1e-6, max_steps: int = 2_000_000,
                 check_every: int = 200, group: int = 1024):
    """Grids of `specs` run from rest to residual <= tol, `group` basins per
    batched launch.  Returns (grids, steps per basin, wall seconds)."""
    grids, steps = [], []
    t0 = time.perf_counter()
    for i in range(0, len(specs), group):
        gs = [mlb.grid_from_spec(ctx, s) for s in specs[i:i + group]]
        b = mlb.Batch(ctx, gs)
        ok, diags = b.run_steady(tol, max_steps, check_every)
        b.close()
        if not ok:
            raise RuntimeError("training basins did not reach the tolerance in %d steps" % max_steps)
        grids += gs
        steps += [int(d["step"]) for d in diags]
    ctx.sync()
    return grids, steps, time.perf_counter() - t0


def _fill(ctx, net, grids, x, t):
    import torch
    torch.cuda.synchronize()
    for i, g in enumerate(grids):
        net.features(g, x[i])
        net.targets(g, t[i])
    ctx.sync()


def fit_norm(ctx: mlb.Context, net: mlb.Net, grids: List[mlb.Grid], x, t, sub: int = 4,
             stress_scaled: bool = True) -> dict:
    """Normalisation from raw features / targets of the training grids:
    identity normalisation first (raw H, tau_x, tau_y, |tau|, C_b in channels
    0..4), statistics of a strided host copy.  With stress_scaled, targets
    are divided per basin by |tau| / tau_ref (tau_ref = mean |tau|) before
    their spread is taken."""
    net.set_norm([0] * 5, [1] * 5, 1.0, 1.0, 0.0)
    _fill(ctx, net, grids, x, t)
    xs = x[:, ::sub, ::sub, :5].cpu().numpy().astype(np.float64)
    mean = [float(xs[..., k].mean()) for k in range(5)]
    std = [float(max(xs[..., k].std(), 1e-12)) for k in range(5)]
    tau_ref = float(max(xs[..., 3].mean(), 1e-12)) if stress_scaled else 0.0
    net.set_norm(mean, std, 1.0, 1.0, tau_ref)
    _fill(ctx, net, grids, x, t)
    ts = t[:, ::sub, ::sub, :].cpu().numpy().astype(np.float64)
    s_eta = float(max(ts[..., 0].std(), 1e-12))
    s_q = float(max(ts[..., 1:].std(), 1e-12))
    norm = {"in_mean": mean, "in_std": std, "s_eta": s_eta, "s_q": s_q, "tau_ref": tau_ref}
    net.set_norm(mean, std, s_eta, s_q, tau_ref)
    return norm


def build_dataset(ctx: mlb.Context, net: mlb.Net, specs: List[wl.Spec], tol: float = 1e-6,
                  check_every: int = 200, norm: Optional[dict] = None, stress_scaled: bool = True,
                  log=print) -> Dataset:
    import torch
    grids, steps, solve_s = solve_steady(ctx, specs, tol, check_every=check_every)
    log("solved %d basins in %.1f s (steps %d..%d)" % (len(specs), solve_s, min(steps), max(steps)))
    n, h, w = len(specs), specs[0].ny, specs[0].nx
    x = torch.empty((n, h, w, mlb.NET_FEATURES), dtype=torch.float32, device="cuda")
    t = torch.empty((n, h, w, 3), dtype=torch.float32, device="cuda")
    if norm is None:
        norm = fit_norm(ctx, net, grids, x, t, stress_scaled=stress_scaled)
    else:
        net.set_norm(norm["in_mean"], norm["in_std"], norm["s_eta"], norm["s_q"], norm.get("tau_ref", 0.0))
    _fill(ctx, net, grids, x, t)
    return Dataset(specs, grids, steps, solve_s, x, t, norm)


def train(net: mlb.Net, data: Dataset, ts: TrainSpec, log=print) -> List[float]:
    """One mlb_net_train call per epoch: step size constant within an epoch,
    cosine decay from lr to lr_min across epochs, linear warm-up over the
    first warmup_steps steps; a fresh sample order per epoch."""
    t0 = time.perf_counter()
    losses = []
    for e in range(ts.epochs):
        lr_e = ts.lr_min + 0.5 * (ts.lr - ts.lr_min) * (1.0 + np.cos(np.pi * e / ts.epochs))
        el = net.train(data.x, data.t, len(data.specs), 1, ts.batch, lr_e, lr_e,
                       ts.warmup_steps if e == 0 else 0, weight_decay=ts.weight_decay, seed=ts.seed + e)
        losses.append(float(el[0]))
        log("epoch %d/%d loss %.4g lr %.2e (%.1f s)" % (e + 1, ts.epochs, losses[-1], lr_e,
                                                      time.perf_counter() - t0))
    net.ctx.sync()
    log("trained %d epochs in %.1f s; loss %.4g -> %.4g" % (ts.epochs, time.perf_counter() - t0, losses[0],
                                                           losses[-1]))
    return losses


def evaluate(ctx: mlb.Context, net: mlb.Net, specs: List[wl.Spec], tol: float = 1e-6,
             max_steps: int = 2_000_000, check_every: int = 100, stall_checks: int = 100,
             log=print) -> List[dict]:
    """Per basin: cold run from rest (mlb_run_steady) and warm run
    (mlb_warm_start_run, inference included), single-basin graph mode.  Both
    stop at R <= tol or under the same stall rule (`stall_checks` checks
    without a new lowest residual: the FP32 noise floor of a weak flow)."""
    ctx.set_stall_checks(stall_checks)
    # launch options tuned once for the basin shape, used by both runs
    g = mlb.grid_from_spec(ctx, specs[0])
    opts = g.autotune(steps=40)
    g.close()
    log("exec options %s" % json.dumps(opts))
    out = []
    for s in specs:
        g = mlb.grid_from_spec(ctx, s)
        g.set_exec_opts(**opts)
        ctx.sync()
        t0 = time.perf_counter()
        ok_c, dc = g.run_steady(tol, max_steps, check_every)
        cold_s = time.perf_counter() - t0
        g.close()
        g = mlb.grid_from_spec(ctx, s)
        g.set_exec_opts(**opts)
        ctx.sync()
        ok_w, rep = net.warm_start_run(g, tol, max_steps, check_every)
        g.close()
        r = {"name": s.name, "cold_s": cold_s, "cold_steps": int(dc["step"]), "cold_ok": ok_c,
             "cold_stalled": dc["stalled"], "cold_residual": dc["residual"],
             "warm_s": rep["wall_s"], "warm_steps": int(rep["steps_total"]), "warm_ok": ok_w,
             "warm_stalled": rep["stalled"], "warm_residual": rep["diag"]["residual"],
             "used_guess": int(rep["used_guess"]), "fallback": int(rep["fallback"]),
             "infer_ms": rep["infer_ms"], "r0_guess": rep["r0_guess"], "r0_cold": rep["r0_cold"],
             "guess_err": rep["guess_err"]}
        log(json.dumps(r))
        out.append(r)
    return out


def summary(rows: List[dict]) -> dict:
    cold = np.array([r["cold_s"] for r in rows])
    warm = np.array([r["warm_s"] for r in rows])
    ge = np.array([r["guess_err"] for r in rows], dtype=np.float64)
    return {"basins": len(rows), "cold_s_total": float(cold.sum()), "warm_s_total": float(warm.sum()),
            "speedup_total": float(cold.sum() / warm.sum()),
            "speedup_median": float(np.median(cold / warm)),
            "cold_steps_median": float(np.median([r["cold_steps"] for r in rows])),
            "warm_steps_median": float(np.median([r["warm_steps"] for r in rows])),
            "fallbacks": int(sum(1 for r in rows if not r["used_guess"])),
            "stalled_cold": int(sum(1 for r in rows if r["cold_stalled"])),
            "stalled_warm": int(sum(1 for r in rows if r["warm_stalled"])),
            "guess_err_median": [float(v) for v in np.nanmedian(ge, axis=0)],
            "infer_ms_median": float(np.median([r["infer_ms"] for r in rows]))}


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="train and evaluate the learned warm start")
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--held-out", type=int, default=200)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--save", default=None, help="write the trained net here")
    ap.add_argument("--load", default=None, help="skip training: load this net (its normalisation included)")
    ap.add_argument("--out", default=None, help="write the JSON summary here")
    ap.add_argument("--global-scales", action="store_true",
                    help="scale targets by global spreads only (no per-basin stress scaling)")
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, flush=True)

    ctx = mlb.Context(0)
    ns = NetSpec(n=args.n)
    net = mlb.Net(ctx, ns.n, ns.n, base_ch=ns.base_ch, levels=ns.levels, in_ch=ns.in_ch, max_batch=ns.max_batch,
                  seed=2999)
    result = {"net_params": net.nparam}
    if args.load:
        net.load(args.load)
    else:
        data = build_dataset(ctx, net, wl.learned_set(args.train, 2999, n=args.n), args.tol,
                             stress_scaled=not args.global_scales, log=log)
        result["train_solve_s"] = data.solve_s
        result["train_steps_median"] = float(np.median(data.steps))
        result["norm"] = data.norm
        for g in data.grids:
            g.close()
        data.grids = []
        result["epoch_loss"] = train(net, data, TrainSpec(epochs=args.epochs, lr=args.lr), log=log)
        del data
        if args.save:
            net.save(args.save)
    rows = evaluate(ctx, net, wl.learned_set(args.held_out, 3000, n=args.n), args.tol, log=log)
    result["eval"] = summary(rows)
    log(json.dumps(result["eval"]))
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": result, "rows": rows}, f, indent=1)
    net.close()
    ctx.close()
    return result


if __name__ == "__main__":
    main()
