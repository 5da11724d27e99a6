"""FP64 oracle of the learned starting guess: a 3-level 3D encoder-decoder.

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline leg may use this module.

The network is not in the paper; it supplies the start H0 of the fixed-point
iteration of Sect. 2.1 (any H0 is allowed there; the paper starts from zero).
Parity unpinned against the paper: its values are pinned by finite
differences of the loss, by closed forms of single layers, and by the
GPU-vs-oracle comparison on identical inputs.

Architecture (channels 16 / 32 / 64, 3x3x3 convolutions with zero padding,
ReLU after every convolution except the last 1x1x1 one):

    level 1 (n^3):      e1a: 4 -> 16,  e1b: 16 -> 16          -> skip1
    down (2x average):
    level 2 (n/2)^3:    e2a: 16 -> 32, e2b: 32 -> 32          -> skip2
    down:
    level 3 (n/4)^3:    b3a: 32 -> 64, b3b: 64 -> 64
    up (nearest 2x), concat [skip2, up] (32 + 64 = 96):
    level 2:            d2a: 96 -> 32, d2b: 32 -> 32
    up, concat [skip1, up] (16 + 32 = 48):
    level 1:            d1a: 48 -> 16, d1b: 16 -> 16
    out (1x1x1):        16 -> 3

Arrays are channels-first [C, D, H, W] here; 3x3x3 weights are [27, Cin, Cout]
with tap t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1), the 1x1x1 head is
[1, 16, 3].  With bf16=True the input and every activation stored between
layers is rounded to BF16 (round to nearest even), as the GPU stores them;
the output stays unrounded, and weights are taken as given.
"""
from __future__ import annotations

import numpy as np

LAYERS = [  # name, cin, cout, ksize
    ("e1a", 4, 16, 3), ("e1b", 16, 16, 3),
    ("e2a", 16, 32, 3), ("e2b", 32, 32, 3),
    ("b3a", 32, 64, 3), ("b3b", 64, 64, 3),
    ("d2a", 96, 32, 3), ("d2b", 32, 32, 3),
    ("d1a", 48, 16, 3), ("d1b", 16, 16, 3),
    ("out", 16, 3, 1),
]

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed=0, scale=1.0):
    """He-style random initialisation (FP64), biases zero."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, cin, cout, k in LAYERS:
        taps = k ** 3
        std = scale * np.sqrt(2.0 / (taps * cin))
        p[name + ".w"] = rng.standard_normal((taps, cin, cout)) * std
        p[name + ".b"] = np.zeros(cout)
    return p


def conv3d(x, w, b, periodic=False):
    """3D convolution (cross-correlation): out[o, v] = b[o] + sum over taps t
    and input channels c of x[c, v + tap_t] w[t, c, o], with x zero outside
    the array, or periodic when periodic=True."""
    C, D, H, W = x.shape
    taps = w.shape[0]
    if taps == 1:
        return np.einsum("cdhw,co->odhw", x, w[0]) + b[:, None, None, None]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="wrap" if periodic else "constant")
    out = np.zeros((w.shape[2], D, H, W))
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
        out += np.einsum("cdhw,co->odhw", xs, w[t], optimize=True)
    return out + b[:, None, None, None]


def conv3d_backward(x, w, gout, periodic=False):
    """Gradients of conv3d with respect to x, w and b."""
    C, D, H, W = x.shape
    taps = w.shape[0]
    gb = gout.sum(axis=(1, 2, 3))
    if taps == 1:
        gw = np.einsum("cdhw,odhw->co", x, gout)[None]
        gx = np.einsum("odhw,co->cdhw", gout, w[0])
        return gx, gw, gb
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="wrap" if periodic else "constant")
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for t, (dz, dy, dx) in enumerate(TAPS):
        sl = (slice(None), slice(1 + dz, 1 + dz + D), slice(1 + dy, 1 + dy + H), slice(1 + dx, 1 + dx + W))
        gw[t] = np.einsum("cdhw,odhw->co", xp[sl], gout, optimize=True)
        gxp[sl] += np.einsum("odhw,co->cdhw", gout, w[t], optimize=True)
    if periodic:
        # the halo cells are copies of the opposite faces: fold their gradient back
        # (halo index 0 holds the last cell, index -1 the first)
        for ax in (1, 2, 3):
            first, last, h0, h1 = ([slice(None)] * 4 for _ in range(4))
            first[ax], last[ax], h0[ax], h1[ax] = 1, -2, 0, -1
            gxp[tuple(last)] += gxp[tuple(h0)]
            gxp[tuple(first)] += gxp[tuple(h1)]
    return gxp[:, 1:-1, 1:-1, 1:-1], gw, gb


def pool2(x):
    """2x2x2 average pooling."""
    C, D, H, W = x.shape
    return x.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(2, 4, 6))


def pool2_backward(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    """Nearest-neighbour 2x upsampling."""
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_backward(g):
    C, D, H, W = g.shape
    return g.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(2, 4, 6))


def forward(p, x, bf16=False, periodic=False):
    """Network output for input x [4, n, n, n] and the cache for backward
    (periodic: convolutions wrap around the array, as on the FFT box)."""
    r = bf16_round if bf16 else (lambda a: a)
    cache = {"periodic": periodic}

    def cr(name, a, relu=True):
        z = conv3d(a, p[name + ".w"], p[name + ".b"], periodic)
        cache[name] = (a, z)
        return r(np.maximum(z, 0.0)) if relu else z

    x = r(x)
    s1 = cr("e1b", cr("e1a", x))
    s2 = cr("e2b", cr("e2a", r(pool2(s1))))
    b3 = cr("b3b", cr("b3a", r(pool2(s2))))
    c2 = np.concatenate([s2, up2(b3)], axis=0)
    d2 = cr("d2b", cr("d2a", c2))
    c1 = np.concatenate([s1, up2(d2)], axis=0)
    d1 = cr("d1b", cr("d1a", c1))
    y = cr("out", d1, relu=False)
    return y, cache


def backward(p, cache, gy):
    """Gradients of all parameters given dL/dy (activations as in the cache)."""
    g = {}

    periodic = cache["periodic"]

    def br(name, gout, relu=True):
        a, z = cache[name]
        if relu:
            gout = gout * (z > 0.0)
        ga, gw, gb = conv3d_backward(a, p[name + ".w"], gout, periodic)
        g[name + ".w"], g[name + ".b"] = gw, gb
        return ga

    gd1 = br("out", gy, relu=False)
    gc1 = br("d1a", br("d1b", gd1))
    gs1 = gc1[:16].copy()
    gd2 = up2_backward(gc1[16:])
    gc2 = br("d2a", br("d2b", gd2))
    gs2 = gc2[:32].copy()
    gb3 = up2_backward(gc2[32:])
    gs2 = gs2 + pool2_backward(br("b3a", br("b3b", gb3)))
    gs1 = gs1 + pool2_backward(br("e2a", br("e2b", gs2)))
    br("e1a", br("e1b", gs1))
    return g


def mse(y, t, mask=None):
    """Mean squared error over all elements (and its gradient)."""
    d = y - t
    if mask is not None:
        d = d * mask
    n = d.size
    return float((d * d).sum() / n), 2.0 * d / n


def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of the FP64 parameters in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m." + k, np.zeros_like(p[k]))
        v = state.setdefault("v." + k, np.zeros_like(p[k]))
        m *= b1
        m += (1 - b1) * g[k]
        v *= b2
        v += (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)
