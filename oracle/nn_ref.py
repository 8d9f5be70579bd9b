"""FP64 numpy oracle of the warm-start network (TEST INFRASTRUCTURE ONLY).

Only the tests and the smoke check use it; the product path never does.  It
shares no code with the GPU kernels.

Network (encoder-decoder on NHWC fields, one conv = 3x3 "same" zero padding,
stride 1, bias, ReLU unless stated):
  levels l = 0..L-1 with ch[l] = base * 2^l channels;
  encoder level l: conv(c_in -> ch[l]), conv(ch[l] -> ch[l]) = skip_l;
                   2x2 average pool between levels;
  decoder level l = L-2..0: nearest x2 upsample, conv(ch[l+1] -> ch[l]),
                   concat [that, skip_l], conv(2 ch[l] -> ch[l]), conv(ch[l] -> ch[l]);
  head: 1x1 conv ch[0] -> out_ch, no activation.
Loss: masked mean squared error over all output channels.
Parameters in forward order: each conv's weight [Cout][3][3][Cin] then bias [Cout];
the head's weight [Cout][Cin] then bias.

The backward pass is written out by hand (no autodiff); it is pinned by
central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------- layers
def conv3x3(x, w, b):
    """x [N,H,W,Ci], w [Co,3,3,Ci], b [Co] -> [N,H,W,Co]."""
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (N, H, W, w.shape[0])).astype(np.float64).copy()
    for dy in range(3):
        for dx in range(3):
            y += xp[:, dy:dy + H, dx:dx + W, :] @ w[:, dy, dx, :].T
    return y


def conv3x3_backward(x, w, dz):
    """Gradients of conv3x3 given dL/dy = dz: (dx, dw, db)."""
    N, H, W, Ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros_like(w)
    dxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            win = xp[:, dy:dy + H, dx:dx + W, :]
            dw[:, dy, dx, :] = np.einsum("nhwo,nhwi->oi", dz, win)
            dxp[:, dy:dy + H, dx:dx + W, :] += dz @ w[:, dy, dx, :]
    db = dz.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1, :], dw, db


def relu(z):
    return np.maximum(z, 0.0)


def pool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# ----------------------------------------------------------------------------- network
def layer_shapes(in_ch, out_ch, base, levels):
    """[(name, Cout, Cin, k)] in forward order (k = 3 for convs, 1 for the head)."""
    ch = [base * 2 ** l for l in range(levels)]
    s = []
    c = in_ch
    for l in range(levels):
        s.append(("enc%d_a" % l, ch[l], c, 3))
        s.append(("enc%d_b" % l, ch[l], ch[l], 3))
        c = ch[l]
    for l in range(levels - 2, -1, -1):
        s.append(("dec%d_up" % l, ch[l], ch[l + 1], 3))
        s.append(("dec%d_a" % l, ch[l], 2 * ch[l], 3))
        s.append(("dec%d_b" % l, ch[l], ch[l], 3))
    s.append(("head", out_ch, ch[0], 1))
    return s


def param_count(in_ch, out_ch, base, levels):
    return sum(co * ci * k * k + co for _, co, ci, k in layer_shapes(in_ch, out_ch, base, levels))


def unpack(theta, in_ch, out_ch, base, levels):
    """Flat parameter vector -> {name: (w, b)}."""
    out, o = {}, 0
    for name, co, ci, k in layer_shapes(in_ch, out_ch, base, levels):
        nw = co * ci * k * k
        w = theta[o:o + nw].reshape((co, 3, 3, ci) if k == 3 else (co, ci))
        o += nw
        out[name] = (w, theta[o:o + co])
        o += co
    assert o == theta.size
    return out


def pack(grads, in_ch, out_ch, base, levels):
    parts = []
    for name, *_ in layer_shapes(in_ch, out_ch, base, levels):
        gw, gb = grads[name]
        parts += [gw.ravel(), gb.ravel()]
    return np.concatenate(parts)


def forward(theta, x, in_ch, out_ch, base, levels, keep=False):
    P = unpack(np.asarray(theta, np.float64), in_ch, out_ch, base, levels)
    cache = {}
    h = np.asarray(x, np.float64)
    skips = []
    for l in range(levels):
        if l > 0:
            h = pool2(h)
        for tag in ("a", "b"):
            name = "enc%d_%s" % (l, tag)
            cache[name] = h
            h = relu(conv3x3(h, *P[name]))
            cache[name + ":y"] = h
        skips.append(h)
    for l in range(levels - 2, -1, -1):
        u = up2(h)
        name = "dec%d_up" % l
        cache[name] = u
        h = relu(conv3x3(u, *P[name]))
        cache[name + ":y"] = h
        h = np.concatenate([h, skips[l]], axis=-1)
        for tag in ("a", "b"):
            name = "dec%d_%s" % (l, tag)
            cache[name] = h
            h = relu(conv3x3(h, *P[name]))
            cache[name + ":y"] = h
    cache["head"] = h
    w, b = P["head"]
    y = h @ w.T + b
    return (y, cache, P) if keep else y


def loss_and_grad(theta, x, t, mask, in_ch, out_ch, base, levels):
    """Masked MSE L = sum(mask (y - t)^2) / (count(mask) out_ch), its gradient
    dict {name: (dw, db)} and the output y."""
    y, cache, P = forward(theta, x, in_ch, out_ch, base, levels, keep=True)
    m = np.asarray(mask, np.float64)[..., None]
    cnt = m.sum() * out_ch
    r = (y - t) * m
    L = float((r * r).sum() / cnt)
    dy = 2.0 * r / cnt
    return L, _backward_full(cache, P, dy, levels), y


def _backward_full(cache, P, dy, levels):
    """Backward in exact reverse order of the forward pass."""
    G = {}
    h = cache["head"]
    w, b = P["head"]
    G["head"] = (np.einsum("nhwo,nhwi->oi", dy, h), dy.sum(axis=(0, 1, 2)))
    dh = dy @ w
    dskip = [np.zeros(0)] * levels
    # decoder levels were applied for l = L-2 down to 0; reverse: l = 0 up to L-2
    for l in range(0, levels - 1):
        for tag in ("b", "a"):
            name = "dec%d_%s" % (l, tag)
            dz = dh * (cache[name + ":y"] > 0)
            dh, gw, gb = conv3x3_backward(cache[name], P[name][0], dz)
            G[name] = (gw, gb)
        c = P["dec%d_up" % l][0].shape[0]
        dup, dskip[l] = dh[..., :c], dh[..., c:]
        name = "dec%d_up" % l
        dz = dup * (cache[name + ":y"] > 0)
        du, gw, gb = conv3x3_backward(cache[name], P[name][0], dz)
        G[name] = (gw, gb)
        dh = up2_backward(du)  # gradient w.r.t. the input of decoder l = output of level l+1
    # encoder in reverse: level L-1 output gets dh; each level's output also gets its skip grad
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            dh = dh + dskip[l]
        for tag in ("b", "a"):
            name = "enc%d_%s" % (l, tag)
            dz = dh * (cache[name + ":y"] > 0)
            dh, gw, gb = conv3x3_backward(cache[name], P[name][0], dz)
            G[name] = (gw, gb)
        if l > 0:
            dh = pool2_backward(dh)
    return G


def loss_grad_flat(theta, x, t, mask, in_ch, out_ch, base, levels):
    L, G, y = loss_and_grad(theta, x, t, mask, in_ch, out_ch, base, levels)
    return L, pack(G, in_ch, out_ch, base, levels)


def adamw_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0):
    """One AdamW update (decoupled weight decay), FP64; step counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    theta = theta - lr * (mh / (np.sqrt(vh) + eps) + wd * theta)
    return theta, m, v


def init_params(in_ch, out_ch, base, levels, seed=0):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, co, ci, k in layer_shapes(in_ch, out_ch, base, levels):
        fan = ci * k * k
        parts.append(rng.standard_normal(co * fan) * np.sqrt(2.0 / fan))
        parts.append(np.zeros(co))
    return np.concatenate(parts)
