"""Learned warm start on the GPU: training API, the warm-started steady run
and its fallbacks (forced from the host with a non-finite or garbage net).

Properties checked: training is reproducible bit for bit and lowers the
loss; a warm run converges to the cold run's steady state within the distance
the residual tolerance implies and with the same volume; a fallback run is the
cold run exactly (same steps, same bits); the reported guess error is the
relative L2 distance of the guess the net writes to the converged state.
"""
import sys

import numpy as np
import pytest

from paper_1902_02999_amd import workloads as wl

pytestmark = pytest.mark.gpu

N = 64
TOL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1902_02999_amd import mlb
    c = mlb.Context(0)
    yield c
    c.close()


def small_net(ctx, seed=11):
    from paper_1902_02999_amd import mlb
    return mlb.Net(ctx, N, N, base_ch=32, levels=2, in_ch=32, max_batch=4, seed=seed)


@pytest.fixture(scope="module")
def trained(ctx):
    """A two-level net trained briefly on 24 basins of 64^2."""
    from paper_1902_02999_amd import warmstart as ws
    net = small_net(ctx)
    data = ws.build_dataset(ctx, net, wl.learned_set(24, 77, n=N), TOL, log=say)
    for g in data.grids:
        g.close()
    losses = ws.train(net, data, ws.TrainSpec(epochs=30, batch=4, lr=2e-3, lr_min=1e-4, warmup_steps=10), log=say)
    yield net, data, losses
    net.close()


def test_training_lowers_loss_and_is_reproducible(ctx, trained):
    from paper_1902_02999_amd import warmstart as ws
    net, data, losses = trained
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], losses
    other = small_net(ctx)
    other.set_norm(data.norm["in_mean"], data.norm["in_std"], data.norm["s_eta"], data.norm["s_q"],
                   data.norm["tau_ref"])
    l2 = ws.train(other, data, ws.TrainSpec(epochs=30, batch=4, lr=2e-3, lr_min=1e-4, warmup_steps=10), log=say)
    assert l2 == losses
    assert np.array_equal(other.get_params(), net.get_params())
    other.close()


def test_training_rejects_bad_settings(ctx, trained):
    from paper_1902_02999_amd import mlb
    net, data, _ = trained
    with pytest.raises(mlb.MlbError):
        net.train(data.x, data.t, len(data.specs), 1, 5, 1e-3)   # batch above max_batch
    with pytest.raises(mlb.MlbError):
        net.train(data.x, data.t, len(data.specs), 0, 4, 1e-3)


def cold_run(ctx, spec):
    from paper_1902_02999_amd import mlb
    g = mlb.grid_from_spec(ctx, spec)
    ok, d = g.run_steady(TOL, 2_000_000, 100)
    st = g.get_state()
    g.close()
    assert ok
    return d, st


def test_warm_run_reaches_the_cold_steady_state(ctx, trained):
    from paper_1902_02999_amd import mlb
    net = trained[0]
    for spec in wl.learned_set(3, 3000, n=N):
        dc, (hc, qxc, qyc) = cold_run(ctx, spec)
        g = mlb.grid_from_spec(ctx, spec)
        ok, rep = net.warm_start_run(g, TOL, 2_000_000, 100)
        h, qx, qy = g.get_state()
        dw = g.diag()
        g.close()
        say(spec.name, "cold steps", dc["step"], "warm", rep["steps_total"], "used", rep["used_guess"],
            "fallback", rep["fallback"], "guess err", rep["guess_err"], "r0", rep["r0_guess"], rep["r0_cold"])
        assert ok
        assert rep["steps_total"] >= rep["steps"] >= 1
        assert rep["infer_ms"] > 0 and rep["wall_s"] > 0
        assert rep["diag"]["residual"] <= TOL
        # steady states agree within the residual-implied distance; the volume is the still-water volume
        qn = np.sqrt((qxc ** 2 + qyc ** 2).sum())
        assert np.sqrt(((qx - qxc) ** 2 + (qy - qyc) ** 2).sum()) <= 2e-2 * qn
        eta_c, eta_w = hc - spec.H, h - spec.H
        assert np.sqrt(((eta_w - eta_c) ** 2).sum()) <= 2e-2 * np.sqrt((eta_c ** 2).sum())
        assert abs(dw["mass"] - dc["mass"]) <= 1e-9 * dc["mass"] + 1e-6


def test_guess_error_is_distance_of_written_guess(ctx, trained):
    from paper_1902_02999_amd import mlb
    net = trained[0]
    spec = wl.learned_set(1, 3001, n=N)[0]
    g = mlb.grid_from_spec(ctx, spec)
    net.infer(g)
    hg, qxg, qyg = g.get_state()
    g.close()
    g = mlb.grid_from_spec(ctx, spec)
    ok, rep = net.warm_start_run(g, TOL, 2_000_000, 100)
    h, qx, qy = g.get_state()
    g.close()
    assert ok and rep["used_guess"] == 1
    H = spec.H
    exp = [np.linalg.norm((hg - H) - (h - H)) / np.linalg.norm(h - H),
           np.linalg.norm(qxg - qx) / np.linalg.norm(qx), np.linalg.norm(qyg - qy) / np.linalg.norm(qy)]
    say("guess err", rep["guess_err"], "host", exp)
    for a, b in zip(rep["guess_err"], exp):
        assert abs(a - b) <= 1e-5 * b + 1e-7


@pytest.mark.parametrize("kind", ["nan_weights", "huge_surface"])
def test_fallback_is_the_cold_run(ctx, trained, kind):
    from paper_1902_02999_amd import mlb
    net0, data, _ = trained
    bad = small_net(ctx, seed=3)
    nm = data.norm
    if kind == "nan_weights":
        bad.set_params(np.full(bad.nparam, np.nan, np.float32))
        bad.set_norm(nm["in_mean"], nm["in_std"], nm["s_eta"], nm["s_q"], nm["tau_ref"])
    else:
        bad.set_params(net0.get_params())
        bad.set_norm(nm["in_mean"], nm["in_std"], 5000.0 * max(nm["s_eta"], 0.01), nm["s_q"], nm["tau_ref"])
    spec = wl.learned_set(1, 3002, n=N)[0]
    dc, (hc, qxc, qyc) = cold_run(ctx, spec)
    g = mlb.grid_from_spec(ctx, spec)
    ok, rep = bad.warm_start_run(g, TOL, 2_000_000, 100)
    h, qx, qy = g.get_state()
    g.close()
    bad.close()
    say(kind, rep["fallback"], rep["r0_guess"], rep["r0_cold"], rep["steps"], dc["step"])
    assert ok
    assert rep["used_guess"] == 0 and rep["fallback"] in (mlb.WARM_NONFINITE_GUESS, mlb.WARM_WORSE_THAN_COLD,
                                                         mlb.WARM_DIVERGING)
    if kind == "nan_weights":
        assert rep["fallback"] == mlb.WARM_NONFINITE_GUESS
    assert rep["steps"] == dc["step"]
    assert np.array_equal(h, hc) and np.array_equal(qx, qxc) and np.array_equal(qy, qyc)


def test_steady_cold_start_returns_at_once(ctx, trained):
    from paper_1902_02999_amd import mlb
    net = trained[0]
    spec = wl.learned_set(1, 3003, n=N)[0]
    g = mlb.grid_from_spec(ctx, spec)
    ok, _ = g.run_steady(TOL * 0.5, 2_000_000, 100)
    assert ok
    ok, rep = net.warm_start_run(g, TOL, 1000, 100)
    g.close()
    assert ok and rep["used_guess"] == 0 and rep["fallback"] == mlb.WARM_NONE and rep["steps"] == 1


def test_warm_run_argument_errors(ctx, trained):
    from paper_1902_02999_amd import mlb
    net = trained[0]
    spec = wl.learned_set(1, 3004, n=128)[0]
    g = mlb.grid_from_spec(ctx, spec)
    with pytest.raises(mlb.MlbError):
        net.warm_start_run(g, TOL, 1000, 100)   # grid size differs from the net's
    g.close()
    g = mlb.grid_from_spec(ctx, wl.learned_set(1, 3004, n=N)[0])
    with pytest.raises(mlb.MlbError):
        net.warm_start_run(g, TOL, 1000, 0)
    b = mlb.Batch(ctx, [g])
    with pytest.raises(mlb.MlbError):
        net.warm_start_run(g, TOL, 1000, 100)    # grid inside a live batch
    b.close()
    g.close()


def test_stall_rule_stops_at_the_noise_floor(ctx, trained):
    """A tolerance under FP32's noise floor (but within the stall band of it)
    stalls instead of running to max_steps; the warm run reports the stall
    without falling back.  The floor is measured first: the lowest residual
    of 50 checks once the flow has settled.  The tolerance is a quarter of
    it: runs from other starts settle into other FP32 cycles whose floors
    differ by up to about 2x (the warm run's lowest residual has been 1.7x
    the cold run's), and the stall band reaches 10x the tolerance."""
    from paper_1902_02999_amd import mlb
    net = trained[0]
    spec = wl.learned_set(1, 3005, n=N)[0]
    g = mlb.grid_from_spec(ctx, spec)
    ok, d = g.run_steady(1e-6, 500_000, 100)
    assert ok
    res = []
    for _ in range(50):
        ok, d = g.run_steady(0.0, 100, 100)
        res.append(d["residual"])
    g.close()
    tol = min(res) / 4.0
    say("floor", min(res), max(res), "tol", tol)
    ctx.set_stall_checks(20)
    try:
        g = mlb.grid_from_spec(ctx, spec)
        ok, d = g.run_steady(tol, 500_000, 100)
        say("cold stall at", d["step"], d["residual"])
        assert not ok and d["stalled"] and d["step"] < 500_000
        g.close()
        g = mlb.grid_from_spec(ctx, spec)
        ok, rep = net.warm_start_run(g, tol, 500_000, 100)
        say("warm stall at", rep["steps_total"], rep["diag"]["residual"])
        assert not ok and rep["stalled"] and rep["used_guess"] == 1 and rep["fallback"] == mlb.WARM_NONE
        assert rep["steps_total"] < 500_000
        g.close()
        # a tolerance far below the floor never enters the band: plain max_steps
        g = mlb.grid_from_spec(ctx, spec)
        ok, d = g.run_steady(1e-12, 20_000, 100)
        assert not ok and not d["stalled"] and d["step"] == 20_000
        g.close()
    finally:
        ctx.set_stall_checks(0)
    with pytest.raises(mlb.MlbError):
        ctx.set_stall_checks(-1)


def test_trained_network_gains_over_cold_start(ctx):
    """What the trained network gains: a two-level net trained on the steady
    states of 128 basins of 64^2 (solved by the step itself, 40 epochs)
    against cold starts on 12 held-out basins, each run to R <= 1e-6 (same
    launch options and stall rule for both): the median number of steps is
    at least 15 % lower warm than cold, most basins take fewer steps, and the
    total wall time, inference included, is lower."""
    from paper_1902_02999_amd import mlb, warmstart as ws
    net = mlb.Net(ctx, N, N, base_ch=32, levels=2, in_ch=32, max_batch=8, seed=21)
    data = ws.build_dataset(ctx, net, wl.learned_set(128, 2999, n=N), TOL, log=say)
    for g in data.grids:
        g.close()
    data.grids = []
    losses = ws.train(net, data, ws.TrainSpec(epochs=40, batch=8, lr=2e-3, lr_min=1e-5, warmup_steps=20),
                      log=lambda *a: None)
    say("trained: loss", losses[0], "->", losses[-1])
    rows = ws.evaluate(ctx, net, wl.learned_set(12, 3000, n=N), TOL, log=say)
    sm = ws.summary(rows)
    ctx.set_stall_checks(0)
    net.close()
    say("summary", sm)
    assert all(r["cold_ok"] and r["warm_ok"] for r in rows)
    assert sm["fallbacks"] <= 1
    assert sm["warm_steps_median"] <= 0.85 * sm["cold_steps_median"]
    assert sum(1 for r in rows if r["warm_steps"] < r["cold_steps"]) >= 9
    assert sm["warm_s_total"] < sm["cold_s_total"]
