"""FP64 NumPy oracle of the learned Stokes-map denoiser.

TEST INFRASTRUCTURE ONLY (imported by tests; never by the product path).

The denoiser is not part of the paper's method: it is a small convolutional
encoder-decoder that maps a low-packet Stokes map to an estimate of the
high-packet map's Q and U.  This module states plainly what the HIP kernels
compute, in FP64, with explicit backward passes.

Per image with maps (I, Q, U, V) and s = mean of I over the image:
  Ihat  = I / s
  x     = (ln max(Ihat, 1e-6), Q/I, U/I, V/I)   [N, H, W, 4]
          (fractions clipped to [-1, 1], their physical range; 0 where I <= 0)
The network (widths c1, c2, c3):
  enc1  = relu(conv3(relu(conv3(x,  4->c1)), c1->c1))          H x W
  enc2  = relu(conv3(relu(conv3(pool(enc1), c1->c2)), c2->c2)) H/2
  mid   = relu(conv3(relu(conv3(pool(enc2), c2->c3)), c3->c3)) H/4
  dec2  = relu(conv3(relu(conv3([up(mid), enc2], c3+c2->c2)), c2->c2))
  dec1  = relu(conv3(relu(conv3([up(dec2), enc1], c2+c1->c1)), c1->c1))
  delta = conv1(dec1, c1->2)                                    [N, H, W, 2]
Prediction: q' = Q/I + delta_0, u' = U/I + delta_1; denoised Q = q' I,
U = u' I (I and V unchanged).  Loss against target maps (Q_t, U_t):
  L = mean over images of  sum_p [(q' Ihat - Q_t/s)^2 + (u' Ihat - U_t/s)^2]
                           / sum_p Ihat^2
which is the squared relative Q/U error of the image.
conv3 is a 3x3 cross-correlation with zero padding 1 and a bias; pool is a
2x2 mean; up repeats each pixel 2x2; [a, b] concatenates channels.
Weights of conv3 are stored [Cout, 3, 3, Cin], of conv1 [2, c1].
Adam (Kingma & Ba 2015) with bias correction updates FP64 master weights.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (48, 96, 192)
LAYERS = ("e1a", "e1b", "e2a", "e2b", "m3a", "m3b", "d2a", "d2b", "d1a", "d1b")


def layer_shapes(widths=WIDTHS, cin=4):
    c1, c2, c3 = widths
    io = {"e1a": (cin, c1), "e1b": (c1, c1), "e2a": (c1, c2), "e2b": (c2, c2),
          "m3a": (c2, c3), "m3b": (c3, c3), "d2a": (c3 + c2, c2), "d2b": (c2, c2),
          "d1a": (c2 + c1, c1), "d1b": (c1, c1)}
    shapes = {}
    for k in LAYERS:
        ci, co = io[k]
        shapes[k + ".w"] = (co, 3, 3, ci)
        shapes[k + ".b"] = (co,)
    shapes["head.w"] = (2, c1)
    shapes["head.b"] = (2,)
    return shapes


def n_params(widths=WIDTHS) -> int:
    return int(sum(np.prod(s) for s in layer_shapes(widths).values()))


def unflatten(flat, widths=WIDTHS):
    """Parameters from one flat array in the order of layer_shapes()."""
    out, o = {}, 0
    for k, s in layer_shapes(widths).items():
        n = int(np.prod(s))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(s)
        o += n
    assert o == len(flat)
    return out


def flatten(params, widths=WIDTHS):
    return np.concatenate([np.asarray(params[k], np.float64).ravel() for k in layer_shapes(widths)])


# --------------------------------------------------------------------------
# layers (NHWC)
# --------------------------------------------------------------------------
def conv3(x, w, b):
    """3x3 cross-correlation, zero padding 1: y[n,h,w,o] = b[o] +
    sum_{dy,dx,c} x[n,h+dy-1,w+dx-1,c] w[o,dy,dx,c]."""
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1] = x
    cols = np.stack([xp[:, dy:dy + h, dx:dx + wd] for dy in range(3) for dx in range(3)], axis=3)
    # cols: [n, h, w, 9, c]  ->  matmul with w: [o, 9, c]
    return cols.reshape(n, h, wd, 9 * c) @ w.reshape(w.shape[0], 9 * c).T + b


def conv3_backward(x, w, gy):
    """Gradients of conv3 w.r.t. its input, weights and bias."""
    n, h, wd, c = x.shape
    o = w.shape[0]
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1] = x
    cols = np.stack([xp[:, dy:dy + h, dx:dx + wd] for dy in range(3) for dx in range(3)], axis=3)
    gw = (gy.reshape(-1, o).T @ cols.reshape(-1, 9 * c)).reshape(w.shape)
    gb = gy.reshape(-1, o).sum(0)
    gcols = (gy.reshape(-1, o) @ w.reshape(o, 9 * c)).reshape(n, h, wd, 9, c)
    gxp = np.zeros_like(xp)
    for k, (dy, dx) in enumerate((dy, dx) for dy in range(3) for dx in range(3)):
        gxp[:, dy:dy + h, dx:dx + wd] += gcols[:, :, :, k]
    return gxp[:, 1:-1, 1:-1], gw, gb


def pool(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool_backward(gy):
    return np.repeat(np.repeat(gy, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(gy):
    n, h, w, c = gy.shape
    return gy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def relu(z):
    return np.maximum(z, 0.0)


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------
def forward(p, x):
    """Network output delta [N,H,W,2] and the cache for backward."""
    c = {"x": x}

    def block(name, inp):
        za = conv3(inp, p[name + "a.w"], p[name + "a.b"])
        ya = relu(za)
        zb = conv3(ya, p[name + "b.w"], p[name + "b.b"])
        yb = relu(zb)
        c[name] = (inp, ya, yb)
        return yb

    e1 = block("e1", x)
    e2 = block("e2", pool(e1))
    m3 = block("m3", pool(e2))
    d2 = block("d2", np.concatenate([up(m3), e2], axis=3))
    d1 = block("d1", np.concatenate([up(d2), e1], axis=3))
    return d1 @ p["head.w"].T + p["head.b"], c


def features(maps):
    """[N, 4, H, W] Stokes maps -> (x [N,H,W,4], Ihat [N,H,W], s [N])."""
    I, Q, U, V = (maps[:, k] for k in range(4))
    s = I.mean(axis=(1, 2))
    sd = np.where(s > 0, s, 1.0)
    Ihat = np.where(s[:, None, None] > 0, I / sd[:, None, None], 0.0)
    pos = I > 0
    Id = np.where(pos, I, 1.0)
    with np.errstate(over="ignore"):
        fr = [np.where(pos, np.clip(c / Id, -1.0, 1.0), 0.0) for c in (Q, U, V)]
    x = np.stack([np.log(np.maximum(Ihat, 1e-6))] + fr, axis=-1)
    return x, Ihat, s


def loss(delta, x, Ihat, target):
    """target [N,H,W,2] = (Q_t, U_t) / s.  Returns L."""
    e = (x[..., 1:3] + delta) * Ihat[..., None] - target
    w = (Ihat ** 2).sum(axis=(1, 2))
    return float(np.mean((e ** 2).sum(axis=(1, 2, 3)) / w))


def loss_grad(delta, x, Ihat, target):
    """dL / d delta."""
    e = (x[..., 1:3] + delta) * Ihat[..., None] - target
    w = (Ihat ** 2).sum(axis=(1, 2))
    return 2.0 * e * Ihat[..., None] / (w[:, None, None, None] * delta.shape[0])


def backward(p, cache, gdelta):
    """Gradient of a loss with dL/d delta = gdelta w.r.t. every parameter."""
    g = {}
    d1 = cache["d1"][2]
    g["head.w"] = gdelta.reshape(-1, 2).T @ d1.reshape(-1, d1.shape[-1])
    g["head.b"] = gdelta.reshape(-1, 2).sum(0)
    gd1 = gdelta @ p["head.w"]

    def block_back(name, gy):
        inp, ya, yb = cache[name]
        gzb = gy * (yb > 0)
        gya, g[name + "b.w"], g[name + "b.b"] = conv3_backward(ya, p[name + "b.w"], gzb)
        gza = gya * (ya > 0)
        ginp, g[name + "a.w"], g[name + "a.b"] = conv3_backward(inp, p[name + "a.w"], gza)
        return ginp

    c1 = cache["e1"][2].shape[-1]
    c2 = cache["e2"][2].shape[-1]
    gcat1 = block_back("d1", gd1)
    gup2, ge1 = gcat1[..., :c2], gcat1[..., c2:]
    gcat2 = block_back("d2", up_backward(gup2))
    c3 = gcat2.shape[-1] - c2
    gup3, ge2 = gcat2[..., :c3], gcat2[..., c3:]
    gm3_in = block_back("m3", up_backward(gup3))
    ge2 = ge2 + pool_backward(gm3_in)
    ge2_in = block_back("e2", ge2)
    ge1 = ge1 + pool_backward(ge2_in)
    block_back("e1", ge1)
    assert gcat1.shape[-1] == c2 + c1
    return g


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); updates p, m, v in place."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


