"""Checks shared by the denoiser's GPU parity tests and smoke(): the FP64
oracle evaluated on the operands the kernels see, a replay of it with the
kernels' BF16 roundings, and the norm and element-wise bars derived from
that replay.

The oracle is evaluated on exactly the operands the kernels see: the
parameters and the normalised input rounded to BF16 (nearest even), the
fractions Q/I, U/I, the intensity ratio I/s and the targets in FP32.  What
remains is the rounding of every stored intermediate (activations and their
gradients) to BF16 and the order of FP32 accumulation.

The tolerance is derived from the arithmetic by replaying the oracle's own
layer functions with a BF16 rounding wherever the kernels store BF16
(`bf16_replay`): the replay's distance from the exact oracle is the size of
the rounding noise, and the GPU -- another realisation of the same noise --
must lie
 * per tensor, within twice that distance plus 2e-3 of the exact oracle
   (relative Frobenius norm).  Forward: about 3.6e-3 (sqrt(10) x the RMS
   relative error 2^-9/sqrt(3) of one rounding); weight gradients of the
   deepest layers reach 2-3e-2, because the backward pass compounds the
   roundings of both passes and ends in short sums over few coarse pixels;
 * per element (the forward correction of every network; gradients of a
   network in its linear regime, see check_gradients), within K_ULP BF16
   units in the last place of the replay's
   value plus K_SIGMA times the element's RMS rounding noise plus K_FLOOR of
   the tensor's RMS (elementwise_ratio: the noise estimated from replay
   minus exact, for gradients in proportion to the root sum of squares of
   the products summed into each element).
   The difference of two independent realisations of a noise of RMS sigma
   has RMS sqrt(2) sigma, whose largest value over ~1e5 elements is about
   4.5 sqrt(2) sigma ~ 6.4 sigma if it is Gaussian; the ulp term covers elements whose own magnitude (and so
   rounding) is far above the tensor's typical one.  A wrong index, sign or
   mask in a few tiles or at image borders gives errors of order the
   element itself, hundreds of sigma.
"""
import numpy as np

from oracle import denoiser as D
from paper_2512_01283_amd import workloads as W

K_ULP = 8.0
K_SIGMA = 10.0
K_FLOOR = 1e-3

TOL_FWD = 1.5e-2


def bf16(a):
    """Round to BF16, nearest even, returned as FP64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def dihedral(m, code):
    """Transform [4, H, W] maps by code = r + 4 f (mirror the width axis if f,
    then r quarter turns) with the spin-2 Stokes sign rules."""
    r, f = code & 3, code >> 2
    out = m[:, :, ::-1] if f else m
    out = np.rot90(out, r, axes=(1, 2)).copy()
    out[1] *= (-1) ** r
    out[2] *= (-1) ** (r + f)
    out[3] *= (-1) ** f
    return out


def dihedral_inverse(m, code):
    """The inverse of dihedral(m, code)."""
    r, f = code & 3, code >> 2
    out = m.copy()
    out[1] *= (-1) ** r
    out[2] *= (-1) ** (r + f)
    out[3] *= (-1) ** f
    out = np.rot90(out, -r, axes=(1, 2))
    return (out[:, :, ::-1] if f else out).copy()


def _operands(params32, low, high, widths):
    """Parameters and inputs as the kernels see them: 3x3 weights BF16
    (biases and head FP32), features FP32 -> BF16 for the network, the
    fractions Q/I, U/I, Ihat and the targets FP32."""
    p = D.unflatten(params32.astype(np.float64), widths, cin=low.shape[1])
    for k in p:
        if k.endswith(".w") and not k.startswith("head"):
            p[k] = bf16(p[k])
    xf, Ihat, s = D.features(low)
    xf = np.float32(xf).astype(np.float64)
    Ihat = np.float32(Ihat).astype(np.float64)
    t = None
    if high is not None:
        t = np.float32(np.moveaxis(high[:, 1:3], 1, -1) / s[:, None, None, None]).astype(np.float64)
    return p, xf, bf16(xf), Ihat, t


def oracle_pass(params32, low, high=None, widths=W.DN_WIDTHS):
    """Exact FP64 oracle forward (and backward if high is given) on the
    kernels' operands.  Returns dict(delta, loss, grads)."""
    p, xf, x, Ihat, t = _operands(params32, low, high, widths)
    delta, cache = D.forward(p, x)
    res = dict(delta=delta)
    if high is not None:
        res["loss"] = D.loss(delta, xf, Ihat, t)
        res["grads"] = D.backward(p, cache, D.loss_grad(delta, xf, Ihat, t))
    return res


def bf16_replay(params32, low, high=None, widths=W.DN_WIDTHS):
    """The oracle's layer functions in FP64 with a BF16 rounding at every
    point where the kernels store BF16: each convolution's output (after
    bias and relu), pooled maps, the head's input gradient, each input
    gradient, the adjoints of upsampling and pooling (masks applied before
    rounding).  Returns dict(delta, loss, grads, terms): terms[k] is, for
    each element of the gradient k, the root of the sum of the squares of
    the products summed into it."""
    R = bf16
    p, xf, x, Ihat, t = _operands(params32, low, high, widths)
    L = len(widths)
    c = {}

    def block(name, inp):
        ya = R(D.relu(D.conv3(inp, p[name + "a.w"], p[name + "a.b"])))
        yb = R(D.relu(D.conv3(ya, p[name + "b.w"], p[name + "b.b"])))
        c[name] = (inp, ya, yb)
        return yb

    skips, h = [], x
    for l in range(1, L):
        h = block(f"e{l}", h)
        skips.append(h)
        h = R(D.pool(h))
    h = block(f"m{L}", h)
    for l in range(L - 1, 0, -1):
        h = block(f"d{l}", np.concatenate([D.up(h), skips[l - 1]], axis=3))
    delta = h @ p["head.w"].T + p["head.b"]
    if t is None:
        return dict(delta=delta)
    g, terms = {}, {}
    go = D.loss_grad(delta, xf, Ihat, t)
    g["head.w"] = go.reshape(-1, 2).T @ h.reshape(-1, h.shape[-1])
    g["head.b"] = go.reshape(-1, 2).sum(0)
    terms["head.w"] = np.sqrt((go ** 2).reshape(-1, 2).T @ (h ** 2).reshape(-1, h.shape[-1]))
    terms["head.b"] = np.sqrt((go ** 2).reshape(-1, 2).sum(0))

    def root_sum_squares(name, inp, gz):
        # the same sums over pixels taken of the squared products
        _, sw, sb = D.conv3_backward(inp ** 2, p[name + ".w"], gz ** 2)
        terms[name + ".w"], terms[name + ".b"] = np.sqrt(sw), np.sqrt(sb)

    def block_back(name, gzb):
        inp, ya, yb = c[name]
        gya, g[name + "b.w"], g[name + "b.b"] = D.conv3_backward(ya, p[name + "b.w"], gzb)
        root_sum_squares(name + "b", ya, gzb)
        gza = R(gya * (ya > 0))
        ginp, g[name + "a.w"], g[name + "a.b"] = D.conv3_backward(inp, p[name + "a.w"], gza)
        root_sum_squares(name + "a", inp, gza)
        return R(ginp)

    gy = R((go @ p["head.w"]) * (h > 0))
    gskip = {}
    for l in range(1, L):
        gcat = block_back(f"d{l}", gy)
        cb = widths[l]
        gskip[l] = gcat[..., cb:]
        below = c[f"d{l + 1}"][2] if l + 1 < L else c[f"m{L}"][2]
        gy = R(D.up_backward(gcat[..., :cb]) * (below > 0))
    gin = block_back(f"m{L}", gy)
    for l in range(L - 1, 0, -1):
        gin = block_back(f"e{l}", R((gskip[l] + D.pool_backward(gin)) * (c[f"e{l}"][2] > 0)))
    return dict(delta=delta, loss=D.loss(delta, xf, Ihat, t), grads=g, terms=terms)


def fractions(maps):
    """(Q/I, U/I) as the kernels form them (clamped to [-1, 1], FP32)."""
    return np.float32(D.features(maps)[0][..., 1:3]).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def bf16_ulp(x):
    """Unit in the last place of BF16 (8 significant bits) at |x|; 0 at 0."""
    a = np.abs(np.asarray(x, np.float64))
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, np.exp2(e - 7), 0.0)


def elementwise_ratio(got, rep, exact, label="", terms=None):
    """Largest |got - rep| over its element-wise allowance (<= 1 passes):
        K_ULP ulp(rep) + K_SIGMA sigma + K_FLOOR RMS(rep).
    sigma is the element's RMS rounding noise.  For activations it is the
    tensor's RMS of rep - exact.  A gradient element is a sum of products
    over pixels, and its rounding noise scales with the root of the sum of
    the squared products, `terms` (so a sum that cancels to a small value
    can still carry a large noise): sigma = eps * terms with eps the ratio of
    the RMS of rep - exact to the RMS of terms over the tensor.  The floor
    covers relu decisions taken on pre-activations within rounding noise of
    zero, which flip between two realisations: the value then passed on is
    itself of the noise size, ~1e-3 of a typical activation.  The worst
    elements are printed."""
    got, rep, exact = (np.asarray(a, np.float64) for a in (got, rep, exact))
    res = rep - exact
    if terms is None:
        sigma = np.sqrt(np.mean(res ** 2))
    else:
        terms = np.asarray(terms, np.float64)
        t2 = float(np.mean(terms ** 2))
        sigma = terms * (np.sqrt(np.mean(res ** 2) / t2) if t2 > 0 else 0.0)
    allow = K_ULP * bf16_ulp(rep) + K_SIGMA * sigma + K_FLOOR * np.sqrt(np.mean(rep ** 2)) + 1e-300
    ratio = np.abs(got - rep) / allow
    worst = float(ratio.max())
    if worst > 0.7:
        sig = np.broadcast_to(sigma, ratio.shape)
        for i in np.argsort(ratio, axis=None)[::-1][:3]:
            ix = np.unravel_index(i, ratio.shape)
            print(f"  {label}{[int(j) for j in ix]}: ratio {ratio[ix]:.2f} got {got[ix]:.4e} replay "
                  f"{rep[ix]:.4e} exact {exact[ix]:.4e} sigma {sig[ix]:.3e} (tensor RMS of rep "
                  f"{np.sqrt(np.mean(rep ** 2)):.3e}, of rep - exact {np.sqrt(np.mean(res ** 2)):.3e})")
    return worst


def check_forward(delta_gpu, ref, rep, label):
    """The network's correction from the GPU against the exact oracle (norm
    bar) and against the BF16 replay (element-wise bar)."""
    e, e_rep = rel(delta_gpu, ref), rel(rep, ref)
    r = elementwise_ratio(delta_gpu, rep, ref)
    print(f"{label}: relative error of the correction {e:.2e} (BF16 replay {e_rep:.2e}); "
          f"worst element {r:.2f} of its allowance")
    assert e < TOL_FWD and e < 2.0 * e_rep + 2e-3, (e, e_rep)
    assert r <= 1.0, r
    return e


def check_gradients(g, low, high, params, label, widths=W.DN_WIDTHS, elementwise=False, cin=4):
    """GPU gradients against the exact oracle, per tensor, within twice the
    distance of the BF16 replay from the exact oracle plus 2e-3 (the GPU and
    the replay are two realisations of the same rounding noise), and with
    elementwise=True also element by element against the replay.  The
    element-wise bar needs a network none of whose relu decisions can flip
    between realisations (linear_regime_params): a pre-activation within
    rounding noise of zero takes either branch, and in the backward pass the
    flipped mask passes or stops a whole gradient value, a change of the
    order of the element itself (measured: the exact oracle and its BF16
    replay of a random network differ by up to 66 allowances on coarse-level
    weight gradients, whole channels sitting near zero)."""
    ref = oracle_pass(params, low, high, widths)
    rep = bf16_replay(params, low, high, widths)
    worst, worst_el = 0.0, 0.0
    for k, gr in ref["grads"].items():
        bound = 2.0 * rel(rep["grads"][k], gr) + 2e-3
        e = rel(g[k], gr)
        worst = max(worst, e / bound)
        assert e < bound, (k, e, bound)
        if elementwise:
            r = elementwise_ratio(g[k], rep["grads"][k], gr, k, terms=rep["terms"][k])
            worst_el = max(worst_el, r)
            assert r <= 1.0, (k, r)
    print(f"{label}: worst gradient error {worst:.2f} of its bound" +
          (f"; worst element {worst_el:.2f} of its allowance" if elementwise else ""))
    return ref


def linear_regime_params(seed, widths=W.DN_WIDTHS, cin=4):
    """Parameters under which every relu of the network passes, so that no
    decision of the forward or backward pass can differ between two
    realisations of the rounding: 3x3 weights uniform in [0, 2 / (9 cin)]
    (each output a weighted mean of its inputs), the first convolution's
    biases 16 + U[0, 0.1] (the features lie in [-13.9, ~3]: ln 1e-6 is the
    floor of the intensity feature, fractions in [-1, 1]), the others
    0.1 + U[0, 0.1], so every pre-activation is positive; head N(0, 0.05).
    Indices, borders, tile shapes and the order of the sums are exercised as
    with any parameters."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (ci, co) in enumerate(W.denoiser_layer_io(widths, cin)):
        parts.append(rng.uniform(0.0, 2.0 / (9 * ci), co * 9 * ci))
        parts.append((16.0 if k == 0 else 0.1) + rng.uniform(0.0, 0.1, co))
    parts.append(rng.standard_normal(2 * widths[0]) * 0.05)
    parts.append(rng.standard_normal(2) * 0.05)
    return np.concatenate(parts).astype(np.float32)
