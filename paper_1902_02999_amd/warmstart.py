"""Learned warm start for steady-state runs: data, normalisation, training,
evaluation of warm against cold starts.

Every numerical step runs in the library's kernels (the step, the network's
MFMA forward / backward, AdamW, feature and target extraction, inference and
the warm-started run with its fallback); this module only orders the calls,
holds the device tensors and keeps the bookkeeping.

Data: closed square basins drawn from the ensemble distributions (random
bumps, wind speed and heading, Chezy coefficient), solved from rest to a
per-step discharge residual <= tol in one batched launch per step.  Inputs:
still-water depth, wind stress over density, bed coefficient, node position;
targets: the steady (eta, hu, hv), each normalised by statistics of the
training set.
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
    x: object = None      # torch CUDA [n, h, w, 6]
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


def fit_norm(ctx: mlb.Context, net: mlb.Net, grids: List[mlb.Grid], x, t, sub: int = 4) -> dict:
    """Normalisation from raw features / targets of the training grids
    (identity normalisation first, statistics of a strided host copy)."""
    net.set_norm([0, 0, 0, 0], [1, 1, 1, 1], 1.0, 1.0)
    _fill(ctx, net, grids, x, t)
    xs = x[:, ::sub, ::sub, :4].cpu().numpy().astype(np.float64)
    ts = t[:, ::sub, ::sub, :].cpu().numpy().astype(np.float64)
    mean = [float(xs[..., k].mean()) for k in range(4)]
    std = [float(max(xs[..., k].std(), 1e-12)) for k in range(4)]
    s_eta = float(max(ts[..., 0].std(), 1e-12))
    s_q = float(max(ts[..., 1:].std(), 1e-12))
    norm = {"in_mean": mean, "in_std": std, "s_eta": s_eta, "s_q": s_q}
    net.set_norm(mean, std, s_eta, s_q)
    return norm


def build_dataset(ctx: mlb.Context, net: mlb.Net, specs: List[wl.Spec], tol: float = 1e-6,
                  check_every: int = 200, norm: Optional[dict] = None, log=print) -> Dataset:
    import torch
    grids, steps, solve_s = solve_steady(ctx, specs, tol, check_every=check_every)
    log("solved %d basins in %.1f s (steps %d..%d)" % (len(specs), solve_s, min(steps), max(steps)))
    n, h, w = len(specs), specs[0].ny, specs[0].nx
    x = torch.empty((n, h, w, 6), dtype=torch.float32, device="cuda")
    t = torch.empty((n, h, w, 3), dtype=torch.float32, device="cuda")
    if norm is None:
        norm = fit_norm(ctx, net, grids, x, t)
    else:
        net.set_norm(norm["in_mean"], norm["in_std"], norm["s_eta"], norm["s_q"])
    _fill(ctx, net, grids, x, t)
    return Dataset(specs, grids, steps, solve_s, x, t, norm)


def train(net: mlb.Net, data: Dataset, ts: TrainSpec, log=print) -> List[float]:
    t0 = time.perf_counter()
    losses = net.train(data.x, data.t, len(data.specs), ts.epochs, ts.batch, ts.lr, ts.lr_min, ts.warmup_steps,
                       weight_decay=ts.weight_decay, seed=ts.seed)
    net.ctx.sync()
    log("trained %d epochs in %.1f s; loss %.4g -> %.4g" % (ts.epochs, time.perf_counter() - t0, losses[0],
                                                           losses[-1]))
    return [float(v) for v in losses]


def evaluate(ctx: mlb.Context, net: mlb.Net, specs: List[wl.Spec], tol: float = 1e-6,
             max_steps: int = 2_000_000, check_every: int = 100, log=print) -> List[dict]:
    """Per basin: cold run from rest (mlb_run_steady) and warm run
    (mlb_warm_start_run, inference included), single-basin graph mode."""
    out = []
    for s in specs:
        g = mlb.grid_from_spec(ctx, s)
        ctx.sync()
        t0 = time.perf_counter()
        ok_c, dc = g.run_steady(tol, max_steps, check_every)
        cold_s = time.perf_counter() - t0
        g.close()
        g = mlb.grid_from_spec(ctx, s)
        ctx.sync()
        ok_w, rep = net.warm_start_run(g, tol, max_steps, check_every)
        g.close()
        r = {"name": s.name, "cold_s": cold_s, "cold_steps": int(dc["step"]), "cold_ok": ok_c,
             "warm_s": rep["wall_s"], "warm_steps": int(rep["steps_total"]), "warm_ok": ok_w,
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
        data = build_dataset(ctx, net, wl.learned_set(args.train, 2999, n=args.n), args.tol, log=log)
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
