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
With two independent runs A and B of an image ([N, 8, H, W]: A's I, Q, U, V,
then B's), (I, Q, U, V) above are the runs' mean and four more features
follow: |S_A - S_B| / (2 I) for S = I, Q, U, V (clipped to 1; 0 where
I <= 0), so x is [N, H, W, 8] and the first convolution has 8 inputs.
The network: a U-Net of L levels with widths c1..cL (two 3x3 convolutions
+ relu per block; for L = 3):
  enc1  = relu(conv3(relu(conv3(x,  4->c1)), c1->c1))          H x W
  enc2  = relu(conv3(relu(conv3(pool(enc1), c1->c2)), c2->c2)) H/2
  mid   = relu(conv3(relu(conv3(pool(enc2), c2->c3)), c3->c3)) H/4
  dec2  = relu(conv3(relu(conv3([up(mid), enc2], c3+c2->c2)), c2->c2))
  dec1  = relu(conv3(relu(conv3([up(dec2), enc1], c2+c1->c1)), c1->c1))
  delta = conv1(dec1, c1->2)                                    [N, H, W, 2]
and in general encoder blocks e1..e(L-1) (each followed by pool), the block
mL at H / 2^(L-1), decoder blocks d(L-1)..d1 on [up(below), skip].
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


def layer_names(widths=WIDTHS):
    L = len(widths)
    enc = [f"e{l}" for l in range(1, L)]
    dec = [f"d{l}" for l in range(L - 1, 0, -1)]
    return [b + s for b in enc + [f"m{L}"] + dec for s in ("a", "b")]


def layer_shapes(widths=WIDTHS, cin=4):
    c = list(widths)
    L = len(c)
    io = {"e1a": (cin, c[0]), "e1b": (c[0], c[0])}
    for l in range(2, L):
        io[f"e{l}a"], io[f"e{l}b"] = (c[l - 2], c[l - 1]), (c[l - 1], c[l - 1])
    io[f"m{L}a"], io[f"m{L}b"] = (c[L - 2], c[L - 1]), (c[L - 1], c[L - 1])
    for l in range(L - 1, 0, -1):
        io[f"d{l}a"], io[f"d{l}b"] = (c[l] + c[l - 1], c[l - 1]), (c[l - 1], c[l - 1])
    shapes = {}
    for k in layer_names(widths):
        ci, co = io[k]
        shapes[k + ".w"] = (co, 3, 3, ci)
        shapes[k + ".b"] = (co,)
    shapes["head.w"] = (2, c[0])
    shapes["head.b"] = (2,)
    return shapes


def n_params(widths=WIDTHS, cin=4) -> int:
    return int(sum(np.prod(s) for s in layer_shapes(widths, cin).values()))


def unflatten(flat, widths=WIDTHS, cin=4):
    """Parameters from one flat array in the order of layer_shapes()."""
    out, o = {}, 0
    for k, s in layer_shapes(widths, cin).items():
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
    L = 1 + sum(1 for k in p if k[0] == "e" and k.endswith("a.w"))
    c = {"x": x, "L": L}

    def block(name, inp):
        za = conv3(inp, p[name + "a.w"], p[name + "a.b"])
        ya = relu(za)
        zb = conv3(ya, p[name + "b.w"], p[name + "b.b"])
        yb = relu(zb)
        c[name] = (inp, ya, yb)
        return yb

    skips, h = [], x
    for l in range(1, L):
        h = block(f"e{l}", h)
        skips.append(h)
        h = pool(h)
    h = block(f"m{L}", h)
    for l in range(L - 1, 0, -1):
        h = block(f"d{l}", np.concatenate([up(h), skips[l - 1]], axis=3))
    return h @ p["head.w"].T + p["head.b"], c


def features(maps):
    """[N, 4, H, W] Stokes maps -> (x [N,H,W,4], Ihat [N,H,W], s [N]);
    [N, 8, H, W] two-run maps -> (x [N,H,W,8], Ihat, s) of their mean."""
    if maps.shape[1] == 8:
        mean = 0.5 * (maps[:, :4] + maps[:, 4:])
        x, Ihat, s = features(mean)
        I = mean[:, 0]
        pos = I > 0
        Id = np.where(pos, I, 1.0)
        with np.errstate(over="ignore"):
            noise = [np.where(pos, np.minimum(0.5 * np.abs(maps[:, k] - maps[:, 4 + k]) / Id, 1.0), 0.0)
                     for k in range(4)]
        return np.concatenate([x, np.stack(noise, axis=-1)], axis=-1), Ihat, s
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
    L = cache["L"]
    d1 = cache["d1"][2]
    g["head.w"] = gdelta.reshape(-1, 2).T @ d1.reshape(-1, d1.shape[-1])
    g["head.b"] = gdelta.reshape(-1, 2).sum(0)
    gh = gdelta @ p["head.w"]

    def block_back(name, gy):
        inp, ya, yb = cache[name]
        gzb = gy * (yb > 0)
        gya, g[name + "b.w"], g[name + "b.b"] = conv3_backward(ya, p[name + "b.w"], gzb)
        gza = gya * (ya > 0)
        ginp, g[name + "a.w"], g[name + "a.b"] = conv3_backward(inp, p[name + "a.w"], gza)
        return ginp

    gskip = {}
    for l in range(1, L):                       # decoder, top level first
        gcat = block_back(f"d{l}", gh)
        cb = cache[f"d{l}"][0].shape[-1] - cache[f"e{l}"][2].shape[-1]   # channels of up(below)
        gskip[l] = gcat[..., cb:]
        gh = up_backward(gcat[..., :cb])        # gradient of the block below's output
    gin = block_back(f"m{L}", gh)               # gradient of pool(e(L-1))
    for l in range(L - 1, 0, -1):
        gin = block_back(f"e{l}", gskip[l] + pool_backward(gin))
    return g


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); updates p, m, v in place."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


