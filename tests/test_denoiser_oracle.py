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


def _maps(rng, n, h, w):
    I = 0.5 + rng.uniform(size=(n, h, w))
    m = np.empty((n, 4, h, w))
    m[:, 0] = I
    m[:, 1:] = 0.3 * I[:, None] * rng.uniform(-1, 1, size=(n, 3, h, w))
    return m


def test_network_gradient_finite_differences():
    widths = (3, 4, 5)
    shapes = D.layer_shapes(widths)
    p = {k: RNG.standard_normal(s) * 0.4 for k, s in shapes.items()}
    maps = _maps(RNG, 2, 8, 8)
    x, Ihat, s = D.features(maps)
    t = RNG.standard_normal((2, 8, 8, 2)) * 0.1

    def L():
        return D.loss(D.forward(p, x)[0], x, Ihat, t)

    delta, cache = D.forward(p, x)
    g = D.backward(p, cache, D.loss_grad(delta, x, Ihat, t))
    h = 1e-6
    for k in shapes:
        flat = p[k].ravel()
        for idx in RNG.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = L()
            flat[idx] = old - h
            lm = L()
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].ravel()[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, fd, an)


def test_loss_gradient_in_delta_finite_differences():
    maps = _maps(RNG, 3, 4, 6)
    x, Ihat, _ = D.features(maps)
    t = RNG.standard_normal((3, 4, 6, 2)) * 0.2
    d = RNG.standard_normal((3, 4, 6, 2)) * 0.1
    g = D.loss_grad(d, x, Ihat, t)
    h = 1e-6
    for idx in [(0, 1, 2, 0), (2, 3, 5, 1), (1, 0, 0, 1)]:
        dp, dm = d.copy(), d.copy()
        dp[idx] += h
        dm[idx] -= h
        fd = (D.loss(dp, x, Ihat, t) - D.loss(dm, x, Ihat, t)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(fd))


def test_features_and_loss_at_zero_correction_is_relative_error():
    """x holds ln(I/s) and the polarisation fractions; with delta = 0 the loss
    is the mean over images of sum[(Q - Q_t)^2 + (U - U_t)^2] / sum I^2."""
    maps = _maps(RNG, 2, 6, 6)
    maps[0, :, 0, 0] = 0.0  # a dark pixel: features 0 (log floor for I)
    x, Ihat, s = D.features(maps)
    assert np.allclose(s, maps[:, 0].mean(axis=(1, 2)))
    assert x[0, 0, 0, 0] == np.log(1e-6) and np.all(x[0, 0, 0, 1:] == 0)
    assert np.allclose(x[1, ..., 1], maps[1, 1] / maps[1, 0])
    bad = maps.copy()
    bad[0, 0, 2, 2], bad[0, 1, 2, 2] = 1e-310, 0.3  # |Q| > I: fraction clipped to 1
    assert D.features(bad)[0][0, 2, 2, 1] == 1.0
    assert np.allclose(np.exp(x[1, ..., 0]), maps[1, 0] / s[1])
    tgt = maps.copy()
    tgt[:, 1:3] += 0.05 * RNG.standard_normal(tgt[:, 1:3].shape)
    t = np.moveaxis(tgt[:, 1:3], 1, -1) / s[:, None, None, None]
    L = D.loss(np.zeros(x.shape[:-1] + (2,)), x, Ihat, t)
    E2 = [(((maps[b, 1:3] - tgt[b, 1:3]) ** 2).sum() / (maps[b, 0] ** 2).sum()) for b in range(2)]
    assert abs(L - np.mean(E2)) <= 1e-12 * L


def test_two_run_features_worked_pixel_and_invariances():
    """Two runs A, B of an image: the first four features are those of the
    mean map, the last four |S_A - S_B| / (2 I_mean).  Worked pixel:
    A = (2, 0.4, -0.2, 0), B = (1, 0.1, 0.1, 0.05) -> mean (1.5, 0.25, -0.05,
    0.025): fractions (1/6, -1/30, 1/60), noise features (1/3, 0.1, 0.1, 1/60)."""
    maps = np.ones((1, 8, 2, 2))
    maps[0, 4:] = maps[0, :4]
    maps[0, :, 0, 0] = [2.0, 0.4, -0.2, 0.0, 1.0, 0.1, 0.1, 0.05]
    maps[0, 1:4, 1, 1] = maps[0, 5:8, 1, 1] = 0.0
    x, Ihat, s = D.features(maps)
    assert x.shape == (1, 2, 2, 8)
    assert np.allclose(x[0, 0, 0, 1:], [1 / 6, -1 / 30, 1 / 60, 1 / 3, 0.1, 0.1, 1 / 60], rtol=1e-14, atol=0)
    assert np.isclose(s[0], (1.5 + 3.0) / 4) and np.isclose(Ihat[0, 0, 0], 1.5 / s[0])
    # pixels where the runs agree carry no noise feature
    assert np.all(x[0, 1, 1, 4:] == 0) and np.all(x[0, 0, 1, 4:] == 0)
    # identical runs: the single-map features and zero noise features
    m4 = _maps(RNG, 2, 6, 6)
    x2, Ih2, s2 = D.features(np.concatenate([m4, m4], axis=1))
    x1, Ih1, s1 = D.features(m4)
    assert np.array_equal(x2[..., :4], x1) and np.all(x2[..., 4:] == 0)
    assert np.array_equal(Ih2, Ih1) and np.array_equal(s2, s1)
    # swapping the runs changes nothing
    a, b = _maps(RNG, 2, 6, 6), _maps(RNG, 2, 6, 6)
    assert np.array_equal(D.features(np.concatenate([a, b], 1))[0], D.features(np.concatenate([b, a], 1))[0])


def test_two_run_network_has_eight_inputs():
    n8, n4 = D.n_params(cin=8), D.n_params()
    assert n8 - n4 == 4 * 9 * D.WIDTHS[0]
    assert D.layer_shapes(cin=8)["e1a.w"] == (D.WIDTHS[0], 3, 3, 8)
    flat = RNG.standard_normal(n8)
    assert np.array_equal(D.flatten(D.unflatten(flat, cin=8)), flat)


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


def test_bf16_rounding_model_stays_near_the_exact_oracle():
    """The BF16 replay used to bound the GPU's error differs from the exact
    oracle by a few 1e-3 in the forward correction and by at most ~1e-1 in
    any weight gradient (deepest layers largest)."""
    import test_gpu_denoiser as T
    from paper_2512_01283_amd import workloads as W
    params = W.denoiser_params(12, bias_std=0.05, head_std=0.05)
    low = W.synthetic_stokes_maps(6, 2, 16, 16, noise=0.3)
    high = W.synthetic_stokes_maps(6, 2, 16, 16, noise=0.0)
    ref = T.oracle_pass(params, low, high)
    rep = T.bf16_replay(params, low, high)
    assert T.rel(rep["delta"], ref["delta"]) < 8e-3
    errs = [T.rel(rep["grads"][k], g) for k, g in ref["grads"].items()]
    assert max(errs) < 1e-1 and min(errs) < 2e-3


def test_four_level_network_gradient_finite_differences():
    widths = (2, 3, 4, 5)
    shapes = D.layer_shapes(widths)
    assert list(shapes)[:4] == ["e1a.w", "e1a.b", "e1b.w", "e1b.b"]
    p = {k: RNG.standard_normal(s) * 0.4 for k, s in shapes.items()}
    maps = _maps(RNG, 1, 16, 8)
    x, Ihat, _ = D.features(maps)
    t = RNG.standard_normal((1, 16, 8, 2)) * 0.1
    delta, cache = D.forward(p, x)
    g = D.backward(p, cache, D.loss_grad(delta, x, Ihat, t))
    h = 1e-6
    for k in ("e1a.w", "e3b.w", "m4a.w", "d3a.w", "d1b.b", "head.w"):
        flat = p[k].ravel()
        idx = 1
        old = flat[idx]
        flat[idx] = old + h
        lp = D.loss(D.forward(p, x)[0], x, Ihat, t)
        flat[idx] = old - h
        lm = D.loss(D.forward(p, x)[0], x, Ihat, t)
        flat[idx] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k].ravel()[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, k


def test_parameter_layout_of_three_levels_unchanged():
    names = D.layer_names((48, 96, 192))
    assert names == ["e1a", "e1b", "e2a", "e2b", "m3a", "m3b", "d2a", "d2b", "d1a", "d1b"]
