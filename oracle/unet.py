"""FP64 reference of the warm-start network (test infrastructure only).

A 4-level U-Net with `base` channels at the top level, 3x3 convolutions
(zero padding, stride 1) with bias and ReLU, 2x2 max pooling, 2x2 stride-2
transposed convolutions for upsampling, skip connections by channel
concatenation (upsampled first, skip second) and a final 1x1 convolution:

  level l (l = 0..2): conv(c_l -> C_l), relu, conv(C_l -> C_l), relu -> skip_l, maxpool
  level 3:            conv(C_2 -> C_3), relu, conv(C_3 -> C_3), relu
  up l (l = 2..0):    convT2x2(C_{l+1} -> C_l), concat(., skip_l),
                      conv(2 C_l -> C_l), relu, conv(C_l -> C_l), relu
  out:                conv1x1(C_0 -> cout)

with C_l = base * 2^l. Tensors are NHWC float64 arrays. Weights of a 3x3
convolution are [Cout][3][3][Cin], of a transposed convolution [2][2][Cin][Cout],
of the 1x1 head [cout][Cin]. `quant` rounds weights and activations to bfloat16 where
the GPU kernels hold them in bfloat16 (accumulation stays exact here).

Backward passes are written out by hand (no autodiff); finite differences pin
them in the tests.
"""
from __future__ import annotations

import numpy as np


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(x, quant):
    return bf16(x) if quant else x


# ---------------------------------------------------------------- layers

def conv3x3(x, w, b):
    """y[n,i,j,o] = b[o] + sum_{dy,dx,c} w[o,dy,dx,c] x[n,i+dy-1,j+dx-1,c]."""
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((n, h, wd, w.shape[0])) + b
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("nhwc,oc->nhwo", xp[:, dy:dy + h, dx:dx + wd], w[:, dy, dx, :])
    return y


def conv3x3_backward(x, w, gy):
    """Gradients of conv3x3 w.r.t. x, w and b for upstream gradient gy."""
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1] = x
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            gw[:, dy, dx, :] = np.einsum("nhwo,nhwc->oc", gy, xp[:, dy:dy + h, dx:dx + wd])
            gxp[:, dy:dy + h, dx:dx + wd] += np.einsum("nhwo,oc->nhwc", gy, w[:, dy, dx, :])
    gb = gy.sum(axis=(0, 1, 2))
    return gxp[:, 1:-1, 1:-1], gw, gb


def maxpool2(x):
    """2x2 max pooling; returns (y, argmax index 0..3 within each window,
    first maximum in row-major window order)."""
    n, h, wd, c = x.shape
    win = x.reshape(n, h // 2, 2, wd // 2, 2, c).transpose(0, 1, 3, 5, 2, 4).reshape(n, h // 2, wd // 2, c, 4)
    idx = np.argmax(win, axis=-1)
    return np.take_along_axis(win, idx[..., None], -1)[..., 0], idx


def maxpool2_backward(gy, idx, shape):
    n, h, wd, c = shape
    g = np.zeros((n, h // 2, wd // 2, c, 4))
    np.put_along_axis(g, idx[..., None], gy[..., None], -1)
    return g.reshape(n, h // 2, wd // 2, c, 2, 2).transpose(0, 1, 4, 2, 5, 3).reshape(shape)


def convT2(x, w, b):
    """y[n, 2i+a, 2j+e, o] = b[o] + sum_c w[a,e,c,o] x[n,i,j,c]."""
    n, h, wd, c = x.shape
    y = np.zeros((n, 2 * h, 2 * wd, w.shape[3]))
    for a in range(2):
        for e in range(2):
            y[:, a::2, e::2] = np.einsum("nhwc,co->nhwo", x, w[a, e]) + b
    return y


def convT2_backward(x, w, gy):
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for a in range(2):
        for e in range(2):
            g = gy[:, a::2, e::2]
            gx += np.einsum("nhwo,co->nhwc", g, w[a, e])
            gw[a, e] = np.einsum("nhwc,nhwo->co", x, g)
    return gx, gw, gy.sum(axis=(0, 1, 2))


# ---------------------------------------------------------------- network

def param_shapes(base=32, levels=4, cin=1, cout=1):
    """Ordered (name, shape) of every parameter tensor."""
    ch = [base * 2 ** l for l in range(levels)]
    shapes = []
    c = cin
    for l in range(levels):
        shapes += [(f"d{l}a.w", (ch[l], 3, 3, c)), (f"d{l}a.b", (ch[l],)),
                   (f"d{l}b.w", (ch[l], 3, 3, ch[l])), (f"d{l}b.b", (ch[l],))]
        c = ch[l]
    for l in range(levels - 2, -1, -1):
        shapes += [(f"u{l}t.w", (2, 2, ch[l + 1], ch[l])), (f"u{l}t.b", (ch[l],)),
                   (f"u{l}a.w", (ch[l], 3, 3, 2 * ch[l])), (f"u{l}a.b", (ch[l],)),
                   (f"u{l}b.w", (ch[l], 3, 3, ch[l])), (f"u{l}b.b", (ch[l],))]
    shapes += [("out.w", (cout, ch[0])), ("out.b", (cout,))]
    return shapes


def init_params(rng, base=32, levels=4, cout=1):
    """He-normal weights, zero biases."""
    p = {}
    for name, shp in param_shapes(base, levels, cout=cout):
        if name.endswith(".b"):
            p[name] = np.zeros(shp)
        else:
            transposed = name.split(".")[0].startswith("u") and name.split(".")[0].endswith("t")
            if transposed:
                fan_in = shp[2]
            elif len(shp) == 4:
                fan_in = int(np.prod(shp[1:]))
            else:
                fan_in = shp[1]
            p[name] = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
    return p


def forward(p, x, levels=4, quant=False):
    """Network output [N][H][W][cout] and the cache needed by backward.
    x: [N][H][W][1]."""
    P = {k: (_q(v, quant) if k.endswith(".w") else v) for k, v in p.items()}
    cache = {"x": x}
    h = x
    skips = []
    for l in range(levels):
        a = _q(np.maximum(conv3x3(h, P[f"d{l}a.w"], P[f"d{l}a.b"]), 0), quant)
        cache[f"d{l}a.in"], cache[f"d{l}a.out"] = h, a
        s = _q(np.maximum(conv3x3(a, P[f"d{l}b.w"], P[f"d{l}b.b"]), 0), quant)
        cache[f"d{l}b.in"], cache[f"d{l}b.out"] = a, s
        if l < levels - 1:
            skips.append(s)
            h, idx = maxpool2(s)
            cache[f"pool{l}"] = (idx, s.shape)
        else:
            h = s
    for l in range(levels - 2, -1, -1):
        t = _q(convT2(h, P[f"u{l}t.w"], P[f"u{l}t.b"]), quant)
        cache[f"u{l}t.in"] = h
        cat = np.concatenate([t, skips[l]], axis=-1)
        a = _q(np.maximum(conv3x3(cat, P[f"u{l}a.w"], P[f"u{l}a.b"]), 0), quant)
        cache[f"u{l}a.in"], cache[f"u{l}a.out"] = cat, a
        h = _q(np.maximum(conv3x3(a, P[f"u{l}b.w"], P[f"u{l}b.b"]), 0), quant)
        cache[f"u{l}b.in"], cache[f"u{l}b.out"] = a, h
    y = np.einsum("nhwc,kc->nhwk", h, P["out.w"]) + P["out.b"]
    cache["out.in"] = h
    cache["P"] = P
    return y, cache


def mse(y, t):
    """Mean squared error over all elements and its gradient."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(cache, gy, levels=4, quant=False):
    """Gradients of every parameter for upstream gradient gy = dL/dy.

    With `quant`, gradients passed between layers are rounded to bfloat16 after
    each layer (the GPU keeps them in bfloat16 as matrix-core operands);
    parameter gradients stay exact."""
    P = cache["P"]
    g = {}
    h = cache["out.in"]
    g["out.w"] = np.einsum("nhwc,nhwk->kc", h, gy)
    g["out.b"] = gy.sum(axis=(0, 1, 2))
    gh = _q(np.einsum("nhwk,kc->nhwc", gy, P["out.w"]), quant)
    gskip = {}
    # decoder, from the output (level 0) up to level levels-2
    for l in range(0, levels - 1):
        gh = gh * (cache[f"u{l}b.out"] > 0)
        gh, g[f"u{l}b.w"], g[f"u{l}b.b"] = conv3x3_backward(cache[f"u{l}b.in"], P[f"u{l}b.w"], gh)
        gh = _q(gh, quant) * (cache[f"u{l}a.out"] > 0)
        gcat, g[f"u{l}a.w"], g[f"u{l}a.b"] = conv3x3_backward(cache[f"u{l}a.in"], P[f"u{l}a.w"], gh)
        gcat = _q(gcat, quant)
        c = P[f"u{l}t.w"].shape[3]
        gt, gskip[l] = gcat[..., :c], gcat[..., c:]
        gh, g[f"u{l}t.w"], g[f"u{l}t.b"] = convT2_backward(cache[f"u{l}t.in"], P[f"u{l}t.w"], gt)
        gh = _q(gh, quant)
    # encoder, from the bottom level up
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            idx, shp = cache[f"pool{l}"]
            gh = _q(maxpool2_backward(gh, idx, shp) + gskip[l], quant)
        gh = gh * (cache[f"d{l}b.out"] > 0)
        gh, g[f"d{l}b.w"], g[f"d{l}b.b"] = conv3x3_backward(cache[f"d{l}b.in"], P[f"d{l}b.w"], gh)
        gh = _q(gh, quant) * (cache[f"d{l}a.out"] > 0)
        gh, g[f"d{l}a.w"], g[f"d{l}a.b"] = conv3x3_backward(cache[f"d{l}a.in"], P[f"d{l}a.w"], gh)
        gh = _q(gh, quant)
    return g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of every parameter, in place; t >= 1."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
