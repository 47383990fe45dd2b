"""Training and evaluation driver of the Stokes-map denoiser.

Pairs come from the transport itself: each member of the randomised disk
family (workloads.denoiser_disk) is run twice with independent random
streams, once with few packets (the input) and once with many (the target);
one run images all eight views.  The target's own Monte Carlo noise is
independent of the input's and has zero mean, so the mean-squared-error
minimiser is the same as for a noiseless target (Lehtinen et al. 2018,
"Noise2Noise"); the target only needs enough packets for a useful gradient
signal, not the full reference count.

Evaluation follows the packets-to-fixed-error protocol:
  E(N) = sqrt( sum_w [(Q_N - Q_ref)^2 + (U_N - U_ref)^2] / sum_w I_ref^2 )
over pixels with I_ref > 1e-3 max I_ref, per image, averaged over the test
images; eps = E_plain(1e7); N_plain(eps) from a fit E = a N^-1/2 over plain
runs; N_den(eps) by log-log interpolation of the denoised error over the
input packet counts; the reference's own error is estimated from two
independent halves and must be at most eps / 3.

    python -m paper_2512_01283_amd.dn_train --out dn_out/dn   # full run
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import denoiser as DN
from . import polrad as P
from . import workloads as W


def _disks(seeds, n, npix, lookahead=2):
    """Yield (seed, workload) with the next workloads built on a worker
    thread while the GPU runs the current one (numpy releases the GIL)."""
    from collections import deque
    from concurrent.futures import ThreadPoolExecutor
    seeds = list(seeds)
    with ThreadPoolExecutor(1) as ex:
        q = deque()
        for s in seeds[:lookahead]:
            q.append((s, ex.submit(W.denoiser_disk, s, 1, n=n, npix=npix)))
        k = lookahead
        while q:
            s, f = q.popleft()
            if k < len(seeds):
                q.append((seeds[k], ex.submit(W.denoiser_disk, seeds[k], 1, n=n, npix=npix)))
                k += 1
            yield s, f.result()


def run_images(ctx, packets, seed):
    """Images [views, 4, H, W] (CUDA float64) of one run with its own stream seed.
    A run in which a packet reached a non-finite state still images the
    others; it is reported and kept."""
    try:
        ctx.run([int(packets)], seed=int(seed))
    except P.KpError as e:
        if e.status != P.KP_ERR_NUMERIC:
            raise
        print(f"  warning: run seed {seed}: {e}", flush=True)
    return ctx.images_device()[0].clone()


def run_input(ctx, packets, seed, runs=1):
    """Denoiser input of `packets` packets: one run [views, 4, H, W], or with
    runs = 2 two independent runs of packets / 2 each, [views, 8, H, W]."""
    import torch
    if runs == 1:
        return run_images(ctx, packets, seed)
    half = packets / 2
    return torch.cat([run_images(ctx, half, seed), run_images(ctx, half, seed + 500009)], dim=1)


def make_pairs(seeds, n_lo, n_hi, n=256, npix=None, log=print, runs=1):
    """Returns (lo, hi) CUDA tensors [len(seeds) * 8 * len(n_lo), 4 runs, H, W]
    and [..., 4, H, W].  n_lo is one input packet count or a sequence of
    them: each disk then gives one input per count, all paired with the same
    target run."""
    import torch
    counts = [n_lo] if np.isscalar(n_lo) else list(n_lo)
    los, his = [], []
    t0 = time.time()
    for k, (s, cfg) in enumerate(_disks(seeds, n, npix)):
        with P.Context(0) as ctx:
            ctx.load(cfg)
            hi = run_images(ctx, n_hi, 2 * s + 2)
            for j, c in enumerate(counts):
                los.append(run_input(ctx, c, 2 * s + 1 + 1000003 * j, runs))
                his.append(hi)
        if log and (k + 1) % 8 == 0:
            log(f"  pairs: {k + 1}/{len(seeds)} disks, {time.time() - t0:.1f} s", flush=True)
    torch.cuda.synchronize()
    return torch.cat(los), torch.cat(his)


def image_error(maps, ref):
    """Per-image E (see module docstring); maps, ref CUDA [B, 4, H, W]."""
    import torch
    I = ref[:, 0]
    mask = I > 1e-3 * I.amax(dim=(1, 2), keepdim=True)
    num = ((maps[:, 1] - ref[:, 1]) ** 2 + (maps[:, 2] - ref[:, 2]) ** 2) * mask
    den = (I ** 2) * mask
    return torch.sqrt(num.sum(dim=(1, 2)) / den.sum(dim=(1, 2)))


def train(dn, lo, hi, steps, batch=8, lr=1e-3, lr_min=1e-5, seed=0, aug=True, log=print,
          log_every=200):
    """Adam on random minibatches with random dihedral augmentation and a
    cosine learning-rate decay.  Returns the list of (step, loss)."""
    rng = np.random.default_rng(seed)
    n = lo.shape[0]
    hist = []
    square = lo.shape[2] == lo.shape[3]
    t0 = time.time()
    for it in range(steps):
        idx = rng.choice(n, size=min(batch, n), replace=False)
        import torch
        ii = torch.from_numpy(idx).cuda()
        xb, yb = lo.index_select(0, ii).contiguous(), hi.index_select(0, ii).contiguous()
        codes = None
        if aug:
            codes = rng.integers(0, 8, size=len(idx)).astype(np.int32)
            if not square:
                codes &= ~1
        a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * it / max(steps, 1)))
        loss = dn.train_step(xb, yb, a, aug=codes)
        if not math.isfinite(loss):
            raise FloatingPointError(f"training loss is {loss} at step {it}")
        hist.append((it, loss))
        if log and (it % log_every == 0 or it == steps - 1):
            log(f"  step {it}: loss {loss:.4e} lr {a:.2e} ({time.time() - t0:.1f} s)", flush=True)
    return hist


def _packets_to_eps(counts, errors, eps):
    """(N, bound): the input count at which the error curve reaches eps, by
    log-log interpolation of errors[count] over the counts tried."""
    dc = np.array(counts, dtype=float)
    de = np.array([errors[c] for c in counts])
    if eps >= de[0]:
        return float(dc[0]), "<="  # reached at or below the smallest count tried
    if eps < de.min():
        return float("nan"), "not reached"
    order = np.argsort(dc)
    le, lc = np.log(de[order]), np.log(dc[order])
    for j in range(len(lc) - 1):
        if (le[j] - math.log(eps)) * (le[j + 1] - math.log(eps)) <= 0:
            t = (math.log(eps) - le[j]) / (le[j + 1] - le[j])
            return math.exp(lc[j] + t * (lc[j + 1] - lc[j])), "="
    return float("nan"), "="


def evaluate(dn, seeds, plain_counts=(1e6, 3e6, 1e7, 3e7), den_counts=(1e5, 3e5, 1e6, 3e6),
             ref_half=1.5e8, n=256, npix=None, log=print, tta=False):
    """Packets-to-fixed-error comparison of plain and denoised maps.  A
    two-run denoiser gets each count as two runs of half the packets; its
    "input" error is that of their mean, the plain map of that count."""
    import torch
    Ep = {c: [] for c in plain_counts}
    Ed = {c: [] for c in den_counts}
    Ein = {c: [] for c in den_counts}
    Etta = {c: [] for c in den_counts}
    Eref = []
    for s, cfg in _disks(seeds, n, npix):
        with P.Context(0) as ctx:
            ctx.load(cfg)
            h1 = run_images(ctx, ref_half, 10 * s + 1)
            h2 = run_images(ctx, ref_half, 10 * s + 2)
            ref = 0.5 * (h1 + h2)
            # E of the mean of two halves = E(half1 - half2) / 2
            Eref += (0.5 * image_error(h1, h2)).tolist()
            for k, c in enumerate(plain_counts):
                Ep[c] += image_error(run_images(ctx, c, 10 * s + 3 + k), ref).tolist()
            for k, c in enumerate(den_counts):
                m = run_input(ctx, c, 100 * s + 7 + k, dn.runs)
                Ein[c] += image_error(0.5 * (m[:, :4] + m[:, 4:]) if dn.runs == 2 else m, ref).tolist()
                Ed[c] += image_error(dn.infer(m), ref).tolist()
                if tta:
                    Etta[c] += image_error(dn.infer(m, tta=True), ref).tolist()
        torch.cuda.synchronize()
        if log:
            log(f"  evaluated disk {s}", flush=True)
    per = dict((k, d) for k, d in (("plain", Ep), ("denoised", Ed), ("input", Ein)) +
               ((("denoised_tta", Etta),) if tta else ()))
    res = _ratios(per, plain_counts, den_counts, tta)
    res.update(E_ref=float(np.mean(Eref)), ref_ok=bool(np.mean(Eref) <= res["eps"] / 3), seeds=list(seeds))
    # spread: the same quantities over bootstrap resamples of the test disks
    # (each disk's images resampled together)
    nimg = len(Ep[plain_counts[0]])
    per_disk = max(1, nimg // max(1, len(list(seeds))))
    ndisk = nimg // per_disk
    rng = np.random.default_rng(0)
    boot = {"ratio": [], "ratio_tta": []}
    for _ in range(1000):
        pick = rng.integers(0, ndisk, ndisk)
        idx = (pick[:, None] * per_disk + np.arange(per_disk)[None]).ravel()
        r = _ratios({k: {c: [v[j] for j in idx] for c, v in d.items()} for k, d in per.items()},
                    plain_counts, den_counts, tta)
        boot["ratio"].append(r["ratio"] if r["ratio"] is not None else np.nan)
        if tta:
            boot["ratio_tta"].append(r["ratio_tta"] if r["ratio_tta"] is not None else np.nan)
    for k, v in boot.items():
        if v:
            res[k + "_p16_p84"] = [float(np.nanpercentile(v, 16)), float(np.nanpercentile(v, 84))]
    res["per_image"] = {k: {str(c): [float(x) for x in v] for c, v in d.items()} for k, d in per.items()}
    return res


def _ratios(per, plain_counts, den_counts, tta):
    """Mean errors and the packets-to-error ratios of per-image error lists."""
    mean = {k: {c: float(np.mean(v)) for c, v in d.items()} for k, d in per.items()}
    eps = mean["plain"][1e7]
    # E = a N^-1/2 fitted in log space
    xs = np.log(np.array(plain_counts))
    ys = np.log(np.array([mean["plain"][c] for c in plain_counts]))
    loga = float(np.mean(ys + 0.5 * xs))
    n_plain = math.exp(2 * (loga - math.log(eps)))
    slope = float(np.polyfit(xs, ys, 1)[0])
    n_den, bound = _packets_to_eps(den_counts, mean["denoised"], eps)
    res = dict(eps=eps, plain_slope=slope, N_plain=n_plain, N_den=n_den, N_den_bound=bound,
               ratio=(n_plain / n_den) if n_den == n_den else None, E=mean)
    if tta:
        n_tta, bound_tta = _packets_to_eps(den_counts, mean["denoised_tta"], eps)
        res.update(N_den_tta=n_tta, N_den_tta_bound=bound_tta,
                   ratio_tta=(n_plain / n_tta) if n_tta == n_tta else None)
    return res


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default="dn_out/dn")
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--npix", type=int, default=256)
    ap.add_argument("--train-seeds", default="1000:1064")
    ap.add_argument("--test-seeds", default="3000:3008")
    ap.add_argument("--n-lo", default="1e6", help="input packet count(s), comma-separated")
    ap.add_argument("--n-hi", type=float, default=3e7)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--ref-half", type=float, default=1.5e8)
    ap.add_argument("--widths", default="48,96,192", help="channel widths, one per U-Net level")
    ap.add_argument("--runs", type=int, default=1, choices=(1, 2),
                    help="2: inputs are two independent runs of half the packets each")
    ap.add_argument("--init", default=None, help="start from saved parameters (.npy)")
    ap.add_argument("--skip-eval", action="store_true")
    ap.add_argument("--tta", action="store_true",
                    help="also evaluate the mean over the 8 dihedral transforms of each input")
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)

    def seeds(s):
        lo, hi = (int(v) for v in s.split(":"))
        return list(range(lo, hi))

    log = print
    t0 = time.time()
    log(f"generating training pairs on {torch.cuda.get_device_name(0)}", flush=True)
    n_lo = [float(v) for v in str(a.n_lo).split(",")]
    if a.steps > 0:
        lo, hi = make_pairs(seeds(a.train_seeds), n_lo, a.n_hi, n=a.grid, npix=a.npix, log=log, runs=a.runs)
    t_gen = time.time() - t0
    widths = tuple(int(v) for v in a.widths.split(","))
    dn = DN.Denoiser(0, widths=widths, runs=a.runs)
    init = np.load(a.init) if a.init else W.denoiser_params(0, widths=widths, cin=4 * a.runs)
    dn.set_params(init)
    t1 = time.time()
    hist = [(0, float("nan"))]
    if a.steps > 0:  # 0: evaluate the --init parameters only
        hist = train(dn, lo, hi, a.steps, batch=a.batch, lr=a.lr, log=log)
        del lo, hi
    torch.cuda.synchronize()
    t_train = time.time() - t1
    np.save(os.path.join(a.out, "params.npy"), dn.params())
    res = dict(widths=list(widths), runs=a.runs, params=dn.n, train_seeds=a.train_seeds, n_lo=n_lo, n_hi=a.n_hi,
               steps=a.steps, batch=a.batch,
               lr=a.lr, t_generate_s=t_gen, t_train_s=t_train,
               loss_first=hist[0][1], loss_last=float(np.mean([l for _, l in hist[-50:]])))
    if not a.skip_eval:
        log("evaluating", flush=True)
        res["eval"] = evaluate(dn, seeds(a.test_seeds), ref_half=a.ref_half, n=a.grid, npix=a.npix, log=log,
                               tta=a.tta)
    with open(os.path.join(a.out, "result.json"), "w") as f:
        json.dump(res, f, indent=1)
    log(json.dumps(res), flush=True)
    dn.close()


if __name__ == "__main__":
    main()
