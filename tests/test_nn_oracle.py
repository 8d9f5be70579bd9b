"""Pins of the FP64 warm-start network oracle: the hand-written backward
against central finite differences, layer-level identities, AdamW against
its closed form on a quadratic."""
import numpy as np
import pytest

from oracle import nn_ref as R

CFG = dict(in_ch=4, out_ch=3, base=4, levels=3)


def small_problem(seed=0, H=8, W=8, N=2):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((N, H, W, CFG["in_ch"]))
    t = rng.standard_normal((N, H, W, CFG["out_ch"]))
    mask = (rng.uniform(size=(N, H, W)) > 0.2).astype(float)
    theta = R.init_params(seed=seed, **CFG) + 0.05 * rng.standard_normal(R.param_count(**CFG))
    return theta, x, t, mask


def test_param_layout():
    names = [n for n, *_ in R.layer_shapes(**CFG)]
    assert names == ["enc0_a", "enc0_b", "enc1_a", "enc1_b", "enc2_a", "enc2_b",
                     "dec1_up", "dec1_a", "dec1_b", "dec0_up", "dec0_a", "dec0_b", "head"]
    # the 4-level, 32..256-channel net of the warm start has about 2.1 M parameters
    assert 2.0e6 < R.param_count(in_ch=32, out_ch=3, base=32, levels=4) < 2.3e6


def test_gradient_matches_finite_differences():
    theta, x, t, mask = small_problem()
    L, g = R.loss_grad_flat(theta, x, t, mask, **CFG)
    rng = np.random.default_rng(1)
    idx = rng.choice(theta.size, 60, replace=False)
    # include the head and both ends of the vector
    idx = np.concatenate([idx, [0, theta.size - 1, theta.size - 5]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (R.loss_grad_flat(tp, x, t, mask, **CFG)[0] - R.loss_grad_flat(tm, x, t, mask, **CFG)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 5, 6, 3))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    y = R.conv3x3(x, w, b)
    for (n, i, j, o) in [(0, 0, 0, 0), (0, 4, 5, 1), (0, 2, 3, 1), (0, 0, 5, 0)]:
        s = b[o]
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ii, jj = i + dy, j + dx
                if 0 <= ii < 5 and 0 <= jj < 6:
                    s += (x[n, ii, jj, :] * w[o, dy + 1, dx + 1, :]).sum()
        assert abs(y[n, i, j, o] - s) < 1e-12


def test_pool_up_adjoint():
    """<pool(x), y> = <x, pool^T(y)> and <up(x), y> = <x, up^T(y)>."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 6, 8, 3))
    y = rng.standard_normal((2, 3, 4, 3))
    assert abs((R.pool2(x) * y).sum() - (x * R.pool2_backward(y)).sum()) < 1e-12
    z = rng.standard_normal((2, 6, 8, 3))
    assert abs((R.up2(y) * z).sum() - (y * R.up2_backward(z)).sum()) < 1e-12


def test_adamw_closed_form():
    """First AdamW step moves every parameter by lr (sign of the gradient) plus
    the decoupled decay; on f = |theta|^2 / 2 repeated steps shrink theta."""
    th = np.array([1.0, -2.0, 0.5])
    g = th.copy()
    m = np.zeros(3)
    v = np.zeros(3)
    t1, m, v = R.adamw_step(th, g, m, v, 1, lr=0.1, wd=0.01)
    assert np.allclose(t1, th - 0.1 * (np.sign(th) * (1 - 1e-8 / (np.abs(th) + 1e-8)) + 0.01 * th), atol=1e-12)
    t = th.copy()
    m = np.zeros(3); v = np.zeros(3)
    for k in range(1, 200):
        t, m, v = R.adamw_step(t, t.copy(), m, v, k, lr=0.05)
    assert np.abs(t).max() < 0.05
