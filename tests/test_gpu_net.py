"""Warm-start network on the GPU (BF16 MFMA convolutions, FP32 masters)
through the C ABI against the FP64 oracle network.

Weights are rounded to BF16 on the host before they are set and the inputs
are BF16-exact, so both sides start from identical operands; what remains is
the BF16 rounding of activations between layers (8-bit significand, relative
step 2^-8) and FP32 accumulation order.  Bars, relative L2 over the whole
tensor: forward output 1e-2, loss 2e-3, gradient 2e-2 overall and 8e-2 per
layer; AdamW (pure FP32 arithmetic) 1e-6 relative per element.
"""
import sys

import numpy as np
import pytest

from oracle import nn_ref as R
from paper_1902_02999_amd import workloads as wl

pytestmark = pytest.mark.gpu

NF = 8   # input features per pixel (MLB_NET_FEATURES)

# the last is the warm start's own architecture (4 levels, 32 to 256 channels)
# on a 64 x 256 input, batch 1
CFGS = [dict(H=64, W=64, in_ch=32, base=32, levels=2, N=2),
        dict(H=32, W=128, in_ch=32, base=32, levels=3, N=3),
        dict(H=64, W=256, in_ch=32, base=32, levels=4, N=1)]
IDS = ["L2_64x64", "L3_32x128", "L4_64x256"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_1902_02999_amd import mlb
    c = mlb.Context(0)
    yield c
    c.close()


def bf16_round(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).float().numpy()


def make_net(ctx, cfg, seed=5, max_batch=None):
    from paper_1902_02999_amd import mlb
    net = mlb.Net(ctx, cfg["H"], cfg["W"], base_ch=cfg["base"], levels=cfg["levels"], in_ch=cfg["in_ch"],
                  max_batch=max_batch or cfg["N"], seed=seed)
    rng = np.random.default_rng(seed)
    th = net.get_params().astype(np.float64)
    # nonzero biases so the bias paths are exercised, then BF16-exact weights
    th += 0.02 * rng.standard_normal(th.size)
    th = bf16_round(th).astype(np.float32)
    net.set_params(th)
    return net, th.astype(np.float64)


def inputs(cfg, seed=7):
    rng = np.random.default_rng(seed)
    N, H, W = cfg["N"], cfg["H"], cfg["W"]
    x6 = bf16_round(rng.standard_normal((N, H, W, NF))).astype(np.float64)
    t = rng.standard_normal((N, H, W, 3))
    mask = (rng.uniform(size=(N, H, W)) > 0.25).astype(np.float64)
    xo = np.zeros((N, H, W, cfg["in_ch"]))
    xo[..., :NF] = x6
    return x6, xo, t, mask


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


def okw(cfg):
    return dict(in_ch=cfg["in_ch"], out_ch=3, base=cfg["base"], levels=cfg["levels"])


@pytest.mark.parametrize("cfg", CFGS, ids=IDS)
def test_param_count_and_layout(ctx, cfg):
    net, th = make_net(ctx, cfg)
    assert net.nparam == R.param_count(**okw(cfg))
    # get/set round trip is exact
    assert np.array_equal(net.get_params().astype(np.float64), th)
    net.close()


@pytest.mark.parametrize("cfg", CFGS, ids=IDS)
def test_forward_matches_oracle(ctx, cfg):
    import torch
    say("net forward", cfg)
    net, th = make_net(ctx, cfg)
    x6, xo, _, _ = inputs(cfg)
    xd = dev(x6)
    yd = torch.empty((cfg["N"], cfg["H"], cfg["W"], 3), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    net.forward(xd, cfg["N"], yd)
    ctx.sync()
    y = yd.cpu().numpy().astype(np.float64)
    ref = R.forward(th, xo, **okw(cfg))
    err = rel_l2(y, ref)
    say("forward rel L2", err)
    assert np.isfinite(y).all()
    assert err <= 1e-2, err
    # a smaller batch gives the same per-sample outputs
    if cfg["N"] > 1:
        y1 = torch.empty((1, cfg["H"], cfg["W"], 3), dtype=torch.float32, device="cuda")
        net.forward(xd[1:2].contiguous(), 1, y1)
        ctx.sync()
        assert np.array_equal(y1.cpu().numpy()[0], y[1].astype(np.float32))
    net.close()


@pytest.mark.parametrize("cfg", CFGS, ids=IDS)
def test_loss_and_gradient_match_oracle(ctx, cfg):
    import torch
    say("net loss/grad", cfg)
    net, th = make_net(ctx, cfg)
    x6, xo, t, mask = inputs(cfg)
    torch.cuda.synchronize()
    loss, g = net.loss_grad(dev(x6), dev(t), cfg["N"], mask=dev(mask), mask_count=float(mask.sum()),
                            want_grad=True)
    Lr, Gr, _ = R.loss_and_grad(th, xo, t, mask, **okw(cfg))
    gr = R.pack(Gr, **okw(cfg))
    say("loss", loss, Lr, "grad rel L2", rel_l2(g, gr))
    assert abs(loss - Lr) <= 2e-3 * abs(Lr)
    assert np.isfinite(g).all()
    assert rel_l2(g.astype(np.float64), gr) <= 2e-2
    o = 0
    for name, co, ci, k in R.layer_shapes(**okw(cfg)):
        nw = co * ci * k * k
        ew = rel_l2(g[o:o + nw].astype(np.float64), gr[o:o + nw])
        eb = rel_l2(g[o + nw:o + nw + co].astype(np.float64), gr[o + nw:o + nw + co])
        say("  %-8s dW %.2e db %.2e" % (name, ew, eb))
        assert ew <= 8e-2 and eb <= 8e-2, (name, ew, eb)
        o += nw + co
    # no mask = all ones
    loss2, _ = net.loss_grad(dev(x6), dev(t), cfg["N"])
    L2r = R.loss_and_grad(th, xo, t, np.ones_like(mask), **okw(cfg))[0]
    assert abs(loss2 - L2r) <= 2e-3 * abs(L2r)
    net.close()


def test_gradient_is_deterministic(ctx):
    import torch
    cfg = CFGS[1]
    net, _ = make_net(ctx, cfg)
    x6, _, t, mask = inputs(cfg)
    xd, td, md = dev(x6), dev(t), dev(mask)
    torch.cuda.synchronize()
    a = net.loss_grad(xd, td, cfg["N"], mask=md, mask_count=float(mask.sum()), want_grad=True)
    b = net.loss_grad(xd, td, cfg["N"], mask=md, mask_count=float(mask.sum()), want_grad=True)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])
    net.close()


def test_adamw_matches_oracle(ctx):
    import torch
    cfg = CFGS[0]
    net, th = make_net(ctx, cfg)
    x6, _, t, mask = inputs(cfg)
    xd, td, md = dev(x6), dev(t), dev(mask)
    torch.cuda.synchronize()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    ref = th.copy()
    hp = dict(lr=1e-3, beta1=0.9, beta2=0.99, eps=1e-8, wd=0.01)
    for step in (1, 2, 3):
        _, g = net.loss_grad(xd, td, cfg["N"], mask=md, mask_count=float(mask.sum()), want_grad=True)
        net.adamw(hp["lr"], hp["beta1"], hp["beta2"], hp["eps"], hp["wd"])
        got = net.get_params().astype(np.float64)
        ref, m, v = R.adamw_step(ref, g.astype(np.float64), m, v, step, **hp)
        err = np.abs(got - ref).max()
        say("adamw step", step, "max err", err)
        assert err <= 1e-6 * np.abs(ref).max() + 1e-9, err
        ref = got  # carry the GPU's FP32 parameters on (its m, v are FP32 too)
    net.close()


def test_training_reduces_loss(ctx):
    import torch
    cfg = CFGS[0]
    net, _ = make_net(ctx, cfg)
    x6, _, t, mask = inputs(cfg)
    # a learnable target: a smooth function of the inputs
    t = np.stack([x6[..., 0] * 0.5, x6[..., 1] - x6[..., 2], np.tanh(x6[..., 3])], axis=-1)
    xd, td = dev(x6), dev(t)
    torch.cuda.synchronize()
    first = None
    for it in range(60):
        loss, _ = net.loss_grad(xd, td, cfg["N"])
        first = loss if first is None else first
        net.adamw(2e-3)
    say("loss", first, "->", loss)
    assert loss < 0.3 * first
    net.close()


def test_save_load_roundtrip(ctx, tmp_path):
    cfg = CFGS[0]
    net, th = make_net(ctx, cfg)
    net.set_norm([1.0, 2.0, 3.0, 4.0, 5.0], [0.5, 0.25, 2.0, 8.0, 4.0], 0.125, 3.0, 1e-4)
    p = str(tmp_path / "net.bin")
    net.save(p)
    other, _ = make_net(ctx, cfg, seed=99)
    other.load(p)
    assert np.array_equal(other.get_params(), net.get_params())
    assert other.get_norm() == net.get_norm()
    # a different architecture is rejected
    from paper_1902_02999_amd import mlb
    bad = mlb.Net(ctx, 64, 64, base_ch=64, levels=2, in_ch=32, max_batch=1)
    with pytest.raises(mlb.MlbError):
        bad.load(p)
    bad.close()
    other.close()
    net.close()


def test_bad_configs_rejected(ctx):
    from paper_1902_02999_amd import mlb
    for kw in (dict(height=64, width=64, base_ch=16), dict(height=64, width=96, levels=2),
               dict(height=63, width=64, levels=2), dict(height=64, width=64, in_ch=8),
               dict(height=64, width=64, levels=1), dict(height=64, width=64, base_ch=2048, levels=2)):
        args = dict(height=64, width=64, base_ch=32, levels=2, in_ch=32)
        args.update(kw)
        with pytest.raises(mlb.MlbError):
            mlb.Net(ctx, args.pop("height"), args.pop("width"), **args)


def test_features_targets_infer(ctx):
    """Features of a grid, targets from its state, and the warm-start write
    (mean surface perturbation removed, zero discharge on walls), with and
    without per-basin stress scaling."""
    import torch
    import oracle
    spec = wl.learned_set(1, 4242, n=64)[0]
    H = spec.H
    tx, ty = oracle.wind_stress(*spec.wind_speed)
    cb = oracle.bed_coeff(spec.chezy)
    mag = np.hypot(tx, ty)
    mean = [2.0, 1e-4, -2e-4, 3e-4, 0.003]
    std = [0.1, 3e-4, 5e-4, 2e-4, 0.002]
    for tau_ref in (0.0, 2.5e-4):
        from paper_1902_02999_amd import mlb
        g = mlb.grid_from_spec(ctx, spec)
        net, _ = make_net(ctx, dict(H=64, W=64, in_ch=32, base=32, levels=2), max_batch=1)
        net.set_norm(mean, std, 0.01, 0.05, tau_ref)
        f = mag / tau_ref if tau_ref > 0 else 1.0
        x = torch.empty((64, 64, NF), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        net.features(g, x)
        ctx.sync()
        xf = x.cpu().numpy().astype(np.float64)
        assert np.abs(xf[..., 0] - (H - mean[0]) / std[0]).max() <= 1e-5 * np.abs(H / std[0]).max()
        exp = [(tx / mag, ty / mag) if tau_ref > 0 else ((tx - mean[1]) / std[1], (ty - mean[2]) / std[2])]
        exp = list(exp[0]) + [(mag - mean[3]) / std[3], (cb - mean[4]) / std[4]]
        for k, v in zip((1, 2, 3, 4), exp):
            assert abs(xf[0, 0, k] - v) <= 1e-6 * (abs(v) + 1), (tau_ref, k, xf[0, 0, k], v)
            assert np.all(xf[..., k] == xf[0, 0, k])
        lin = np.linspace(-1.0, 1.0, 64)
        assert np.abs(xf[..., 5] - lin[None, :]).max() <= 1e-6
        assert np.abs(xf[..., 6] - lin[:, None]).max() <= 1e-6
        assert np.all(xf[..., 7] == 1.0)

        # targets of a seeded state
        h0, qx0, qy0 = wl.seeded_state(spec, 3)
        g.set_state(h0, qx0, qy0)
        t = torch.empty((64, 64, 3), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        net.targets(g, t)
        ctx.sync()
        tf = t.cpu().numpy().astype(np.float64)
        se, sq = 0.01 * f, 0.05 * f
        assert np.abs(tf[..., 0] - (h0 - H) / se).max() <= 1e-4 * np.abs((h0 - H) / se).max() + 1e-3
        assert np.abs(tf[..., 1] - qx0 / sq).max() <= 1e-5 * np.abs(qx0 / sq).max() + 1e-6
        assert np.abs(tf[..., 2] - qy0 / sq).max() <= 1e-5 * np.abs(qy0 / sq).max() + 1e-6

        # inference: y = net(features); eta = s_eta f y0 - mean, q = s_q f y12, walls q = 0
        y = torch.empty((1, 64, 64, 3), dtype=torch.float32, device="cuda")
        net.forward(x.reshape(1, 64, 64, NF), 1, y)
        ctx.sync()
        yf = binomial3(y.cpu().numpy()[0].astype(np.float64))
        net.infer(g)
        h, qx, qy = g.get_state()
        eta_exp = se * yf[..., 0]
        eta_exp -= eta_exp.mean()
        assert np.abs((h - H) - eta_exp).max() <= 1e-5 * (np.abs(eta_exp).max() + 1e-3 * se)
        # volume kept: sum of eta is zero to FP32 rounding of the stored fields
        assert abs((h - H).sum()) <= 64 * 64 * 1e-6 * (np.abs(eta_exp).max() + 2.0)
        inner = (slice(1, -1), slice(1, -1))
        assert np.abs(qx[inner] - sq * yf[..., 1][inner]).max() <= 1e-6 * (np.abs(yf[..., 1]).max() * sq + 1e-6)
        for a in (qx, qy):
            assert np.all(a[0, :] == 0) and np.all(a[-1, :] == 0) and np.all(a[:, 0] == 0) and np.all(a[:, -1] == 0)
        # the written state steps finitely
        g.step(10)
        assert not g.diag()["nonfinite"]
        net.close()
        g.close()


def binomial3(y):
    """3x3 (1 2 1) x (1 2 1) / 16 smoothing with clamped edges, per channel."""
    p = np.pad(y, ((1, 1), (1, 1), (0, 0)), mode="edge")
    r = p[:, :-2] + 2.0 * p[:, 1:-1] + p[:, 2:]
    return (r[:-2] + 2.0 * r[1:-1] + r[2:]) / 16.0


def test_no_wind_guess_is_still_water(ctx):
    """With stress scaling, a basin without wind gets the exact still-water guess."""
    import torch
    from paper_1902_02999_amd import mlb
    spec = wl.learned_set(1, 4243, n=64)[0]
    spec.wind_speed = (0.0, 0.0)
    g = mlb.grid_from_spec(ctx, spec)
    net, _ = make_net(ctx, dict(H=64, W=64, in_ch=32, base=32, levels=2), max_batch=1)
    net.set_norm([2.0, 0, 0, 3e-4, 0.003], [0.1, 1, 1, 2e-4, 0.002], 0.01, 0.05, 2.5e-4)
    g.set_state(*wl.seeded_state(spec, 4))
    net.infer(g)
    h, qx, qy = g.get_state()
    assert np.all(qx == 0) and np.all(qy == 0)
    assert np.abs(h - spec.H).max() == 0.0
    t = torch.empty((64, 64, 3), dtype=torch.float32, device="cuda")
    net.targets(g, t)
    ctx.sync()
    assert torch.all(t == 0)
    net.close()
    g.close()
