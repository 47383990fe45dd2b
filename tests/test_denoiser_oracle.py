"""Pins of the FP64 denoiser oracle: convolution against scipy, adjoint
identities of the resampling layers, central finite differences of the whole
network's loss, and Adam's closed-form first step."""
import numpy as np
from scipy.signal import correlate

from oracle import denoiser as D

RNG = np.random.default_rng(7)


def test_conv3_matches_scipy_correlate():
    x = RNG.standard_normal((2, 7, 9, 3))
    w = RNG.standard_normal((4, 3, 3, 3))
    b = RNG.standard_normal(4)
    y = D.conv3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate(x[n, :, :, c], w[o, :, :, c], mode="same")
                             for c in range(3))
            assert np.allclose(y[n, :, :, o], ref, atol=1e-12)


def test_resampling_adjoints():
    x = RNG.standard_normal((2, 8, 6, 3))
    y = RNG.standard_normal((2, 4, 3, 3))
    assert abs((D.pool(x) * y).sum() - (x * D.pool_backward(y)).sum()) < 1e-12
    z = RNG.standard_normal((2, 16, 12, 3))
    x2 = RNG.standard_normal((2, 8, 6, 3))
    assert abs((D.up(x2) * z).sum() - (x2 * D.up_backward(z)).sum()) < 1e-12


def test_conv3_backward_adjoint():
    x = RNG.standard_normal((1, 6, 5, 2))
    w = RNG.standard_normal((3, 3, 3, 2))
    gy = RNG.standard_normal((1, 6, 5, 3))
    gx, gw, gb = D.conv3_backward(x, w, gy)
    # <conv(x), gy> is bilinear in (x, w): its derivatives are gx and gw
    zero = np.zeros(3)
    assert abs((D.conv3(x, w, zero) * gy).sum() - (x * gx).sum()) < 1e-10
    assert abs((D.conv3(x, w, zero) * gy).sum() - (w * gw).sum()) < 1e-10
    assert np.allclose(gb, gy.reshape(-1, 3).sum(0))


def test_network_gradient_finite_differences():
    widths = (3, 4, 5)
    shapes = D.layer_shapes(widths)
    p = {k: RNG.standard_normal(s) * 0.4 for k, s in shapes.items()}
    x = RNG.standard_normal((2, 8, 8, 4))
    t = RNG.standard_normal((2, 8, 8, 2))
    out, cache = D.forward(p, x)
    g = D.backward(p, cache, out, t)
    h = 1e-6
    for k in shapes:
        flat = p[k].ravel()
        for idx in RNG.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = D.loss(D.forward(p, x)[0], t)
            flat[idx] = old - h
            lm = D.loss(D.forward(p, x)[0], t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].ravel()[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, fd, an)


def test_adam_first_step_closed_form():
    p = {"a": np.array([1.0, -2.0, 0.5])}
    g = {"a": np.array([0.3, -0.01, 2.0])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    D.adam(p, g, m, v, 1, lr=0.1)
    # after one step m_hat = g and v_hat = g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(p["a"], [1.0 - 0.1, -2.0 + 0.1, 0.5 - 0.1], atol=1e-7)


def test_parameter_count_and_flattening():
    n = D.n_params()
    assert 1.0e6 < n < 1.1e6
    flat = RNG.standard_normal(n)
    assert np.array_equal(D.flatten(D.unflatten(flat)), flat)
