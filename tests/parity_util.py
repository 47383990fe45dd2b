"""Helpers shared by the GPU parity tests: running a workload through the HIP
library and through the oracle on the same seeded inputs, and comparing."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(cfg, counts=None, device_arrays=True, **opts):
    from paper_2512_01283_amd import polrad as P
    ctx = P.Context(0).load(cfg, device_arrays=device_arrays)
    ctx.run(counts, **opts)
    return ctx


def compare_traces(g, o, tol, min_match=1.0, label="", tau_coef=0.0, frac_within=1.0, hard_cap=None):
    """Per-packet parity: identical event sequences (hash, end kind, counts,
    last cell); on matched packets the final direction agrees to `tol`
    absolutely and the Stokes vector to tol + tau_coef * tau_path relative to
    the packet's I (tau_path: optical depth of the continuous extinction the
    packet went through -- in FP32 the segment lengths carry an absolute
    rounding of order 1e-7 cell, so the weight's relative error grows by about
    that times the optical depth per cell crossed).  Returns the matched
    fraction.  With frac_within < 1, only that fraction of matched packets
    must meet the allowance and every packet must stay below hard_cap
    (relative to I): the FP32 mode for dichroic grains, whose error is set by
    the conditioning of each packet's path."""
    assert len(g) == len(o)
    assert np.array_equal(g["packet"], o["packet"]), "traced packet ids differ"
    same = ((g["hash"] == o["hash"]) & (g["end_kind"] == o["end_kind"]) &
            (g["events"] == o["events"]) & (g["steps"] == o["steps"]) &
            (g["last_cell"] == o["last_cell"]))
    frac = same.mean()
    say(f"[{label}] event-sequence match {same.sum()}/{len(g)}")
    assert frac >= min_match, f"only {frac:.4f} of packets follow the oracle's event sequence"
    gs, os_ = g["stokes"][same], o["stokes"][same]
    scale = np.maximum(np.abs(os_[:, :1]), 1e-300)
    allow = tol + tau_coef * o["tau_path"][same][:, None]
    ds = np.abs(gs - os_) / scale / allow
    dn = np.abs(g["n"][same] - o["n"][same])
    raw = np.abs(gs - os_) / scale
    if raw.size:
        k = int(np.argmax(raw.max(1)))
        say(f"[{label}] max |dS|/I = {raw.max():.3e} (tau_path {o['tau_path'][same][k]:.3g}), "
            f"max over allowance = {ds.max():.3e}, max |dn| = {dn.max():.3e}")
        tp = o["tau_path"][same]
        if "tau_path" in g.dtype.names:
            assert np.allclose(g["tau_path"][same], tp, rtol=10 * max(tol, 1e-6), atol=1e-6)
    if frac_within >= 1.0:
        assert (ds <= 1.0).all(), f"Stokes mismatch beyond allowance ({ds.max():.3e})"
    elif ds.size:
        within = float((ds.max(1) <= 1.0).mean())
        say(f"[{label}] {within:.4f} of packets within the allowance, worst |dS|/I {raw.max():.3e}")
        assert within >= frac_within, f"only {within:.4f} of packets within the allowance"
        assert raw.max() <= hard_cap, f"Stokes mismatch {raw.max():.3e} beyond {hard_cap}"
    assert (dn <= tol).all(), f"direction mismatch {dn.max():.3e} > {tol}"
    return frac


def oracle_batches(cfg, nb=8, lam=0, nthreads=0):
    """Oracle step 1 + 2 split into nb packet batches of one wavelength (same
    packet streams and weights as the whole run): returns (image of the whole
    run, per-batch images of the scattered light).  Step 2 is linear in the
    scattering source, so the whole run's scattered light is the sum of the
    batches'; the dust's direct thermal emission (source kind 2) is
    deterministic and added once."""
    from oracle import oracle as O
    N = int(cfg["packets"][lam])
    edges = np.linspace(0, N, nb + 1).astype(np.int64)
    direct = O.image(cfg, None, lam=lam) if int(cfg["source"].get("kind", 0)) == 2 else 0.0
    imgs = []
    for b in range(nb):
        S, _, _ = O.transport(cfg, lam=lam, p_begin=int(edges[b]), p_end=int(edges[b + 1]),
                              n_total=N, nthreads=nthreads)
        imgs.append(O.image(cfg, S, lam=lam) - direct)
    imgs = np.array(imgs)
    return imgs.sum(0) + direct, imgs


def compare_images_stat(img_g, img_o, batches, k_sigma=3.0, rel_floor=1e-9, label="",
                        max_outlier_frac=0.003):
    """Per-pixel agreement within k_sigma Monte Carlo standard errors, the
    standard error of the sum estimated from the spread of the batch images.
    A small fraction of outliers is allowed (3 sigma is exceeded by 0.3 % of
    pixels for Gaussian noise)."""
    nb = batches.shape[0]
    sig = batches.std(0, ddof=1) * np.sqrt(nb)
    floor = rel_floor * np.abs(img_o[:, 0:1]).max(axis=(-1, -2), keepdims=True)
    d = np.abs(img_g - img_o)
    bad = d > k_sigma * sig + floor
    frac = bad.mean()
    say(f"[{label}] pixels beyond {k_sigma} sigma: {bad.sum()} of {bad.size} ({frac:.2e}); "
        f"max |d|/I_max = {(d / np.abs(img_o[:, 0:1]).max()).max():.3e}")
    assert frac <= max_outlier_frac
    return frac
