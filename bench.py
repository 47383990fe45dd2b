"""Benchmark: Stokes packets/s of two-step polarized Monte Carlo imaging on the
256^3 flared protoplanetary disk (1e8 packets per step, 8 inclinations,
256x256 I/Q/U/V maps), on one MI355X.

One step = one whole pass of the path over the workload: the persistent
transport kernel (emission, cell marching, analytic dichroic extinction,
coherency tally, scattering, roulette) for all packets, the imaging
ray-march for all views, and the learned denoiser's inference on the eight
maps (widths 64/128/256, averaged over the 8 dihedral transforms).  Inputs (density grid) are resident in HBM before the timed region;
images stay on the device.  The denoiser's training step (BF16 MFMA forward
and backward, Adam) is timed separately, after the timed steps, on batches of
those maps, and reported with its own MFMA roofline under "detail".

Prints one JSON line (see the "metric" fields below) with a "roofline"
object for the dominant kernel (transport) and a "cpu_baseline" object (the
FP64 oracle timed on a bounded sample of the same workload on the host).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BF16_PEAK_TFLOPS = 2500.0
# the denoiser configuration whose packets-to-error gain is quoted: widths
# 64/128/256, averaged over the 8 dihedral transforms of each map
DN_WIDTHS = (64, 128, 256)
METRIC = "Stokes packets/s at 256^3 disk; packets to fixed Q/U error, plain vs denoised"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell step of the transport kernel on Rayleigh spheres:
# the density gather (4 B) and 8 B per FP64 tally atomic, one atomic per
# coherency component of the cell (6 of the 9: spheres never create circular
# polarisation, so the 3 imaginary components are identically zero and are
# not tallied)
BYTES_PER_STEP_SPHERE = 4 + 6 * 8


def counter_record():
    """The committed rocprofv3 counter record of one transport launch
    (profiles/k_transport_disk256_1e8.counters.json), or None when the
    transport kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_transport_disk256_1e8.counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2512_01283_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read()
                   for f in ("kp_kernels.hip", "kp_device.hpp", "kp_internal.hpp"))
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec


def counter_traffic():
    """HBM bytes per transport launch from the committed FETCH_SIZE /
    WRITE_SIZE runs (scaled by a 1 GiB copy's readings), in GB, or None."""
    rec = counter_record()
    return None if rec is None else rec["traffic_bytes"] / 1e9


ATOMIC_CAL_LINES = 1 << 24


def atomic_calibration(lines: int = ATOMIC_CAL_LINES, reps: int = 3, order: int = 0) -> float:
    """64-byte-line FP64 atomics the device sustains, in lines/s: the tally
    flush's own access pattern (lane L adds component L % 6 of block L / 6,
    one wave covering 10 blocks) over the blocks of a [256^3][8] FP64 array
    in uniformly random (order 0) or consecutive (order 1) order, in
    libkpcalib.so (csrc/kp_calib.hip); best of `reps` launches, HIP events."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_2512_01283_amd", "libkpcalib.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run python -m paper_2512_01283_amd.build")
    lib = C.CDLL(path)
    lib.kpcal_atomic_lines_order.argtypes = [C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)]
    lib.kpcal_atomic_lines_order.restype = C.c_int
    out = C.c_double()
    st = lib.kpcal_atomic_lines_order(0, lines, 6, reps, order, C.byref(out))
    if st != 0:
        raise RuntimeError(f"kpcal_atomic_lines_order failed ({st})")
    return float(out.value)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=100_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=400000,
                    help="packets of the oracle's timed sample (all threads)")
    ap.add_argument("--cpu-sample-1t", type=int, default=20000,
                    help="packets of the oracle's one-thread sample")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a device-to-device copy of this size (counter calibration)")
    ap.add_argument("--atomic-calibration", action="store_true",
                    help="only run the random 64-byte-line atomic calibration")
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--no-denoiser", action="store_true")
    ap.add_argument("--train-steps", type=int, default=10,
                    help="timed denoiser training steps (batch of the 8 maps)")
    return ap.parse_args()


def copy_calibration(mib: int) -> None:
    """A plain device-to-device copy of known size, so that rocprofv3's
    FETCH_SIZE / WRITE_SIZE can be converted to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "launches": 3}))


def cpu_baseline(cfg, sample: int, sample_1t: int):
    """The oracle as it stands, on the host cores: step 1 for the first
    `sample` packets of the same run (same weights and streams) on all
    threads, step 2 once for all views; scaled to the whole job's packet
    count.  Then step 1 alone on one thread for the first `sample_1t`
    packets (packets/s per core)."""
    from oracle import oracle as O
    nth = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    N = int(cfg["packets"][0])
    t0 = time.perf_counter()
    S, _, st = O.transport(cfg, p_end=sample, n_total=N, nthreads=nth)
    t1 = time.perf_counter()
    O.image(cfg, S)
    t2 = time.perf_counter()
    del S
    step1, step2 = t1 - t0, t2 - t1
    job_s = step1 * (N / sample) + step2
    t3 = time.perf_counter()
    S1, _, _ = O.transport(cfg, p_end=sample_1t, n_total=N, nthreads=1)
    step1_1t = time.perf_counter() - t3
    del S1
    return {"value": N / job_s, "unit": "packets/s", "cores": nth, "kind": "oracle",
            "step1_packets_per_s": sample / step1,
            "step1_packets_per_s_per_core": sample / step1 / nth,
            "single_thread_step1_packets_per_s": sample_1t / step1_1t,
            "host_logical_cpus": os.cpu_count(),
            "sample": f"first {sample} packets of the {N}-packet run (step 1 on {nth} OpenMP threads, "
                      f"{step1:.1f} s, scaled by {N // sample}) + step 2 for all {len(cfg['views'])} "
                      f"views ({step2:.1f} s), FP64; then step 1 of the first {sample_1t} packets "
                      f"on 1 thread ({step1_1t:.1f} s)"}


def copy_bandwidth(mib: int = 1024, reps: int = 5) -> float:
    """Measured device-to-device copy rate (read + write bytes / s, GB/s) of
    a `mib` MiB buffer: best of `reps`, HIP events on the current stream."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2.0 * n * 4 / (best * 1e-3) / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the path shards by "
              "packet ranges across GPUs but this build runs on one device", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return
    if args.atomic_calibration:
        print(json.dumps({"atomic_calibration_lines": ATOMIC_CAL_LINES,
                          "consecutive_lines_per_s": atomic_calibration(order=1),
                          "uniform_random_lines_per_s": atomic_calibration(order=0)}))
        return

    import numpy as np
    import torch

    from paper_2512_01283_amd import polrad as P
    from paper_2512_01283_amd import workloads as W

    cfg = W.flared_disk(packets=args.packets)
    ctx = P.Context(0).load(cfg)
    stream = torch.cuda.current_stream()
    # launch schedule: the autotuner's cached choice for this workload and
    # device (paper_2512_01283_amd/tuning.json), overridden by the flags
    from paper_2512_01283_amd import autotune as A
    opts = A.tuned_opts(cfg, torch.cuda.get_device_name(0))
    if args.block_size:
        opts["block_size"] = args.block_size
    if args.blocks_per_cu:
        opts["blocks_per_cu"] = args.blocks_per_cu
    dn = None
    if not args.no_denoiser:
        from paper_2512_01283_amd import denoiser as DN
        dn = DN.Denoiser(0, widths=DN_WIDTHS, params=W.denoiser_params(0, widths=DN_WIDTHS))
    nv, npix = len(cfg["views"]), cfg["views"][0]["npx"]
    maps = torch.empty((nv, 4, npix, npix), dtype=torch.float64, device="cuda")
    den = torch.empty_like(maps)

    def one_step():
        ctx.run(stream=stream, **opts)
        if dn is not None:
            ctx.images_device(out=maps.view(1, nv, 4, npix, npix), stream=stream)
            dn.infer(maps, den, stream=stream, tta=True)

    for w in range(args.warmup):
        one_step()
        print(f"warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms_t, ms_i, ms_d, steps, flushes = [], [], [], [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step()
        st = ctx.stats()
        ms_t.append(st["ms_transport"])
        ms_i.append(st["ms_image"])
        steps.append(st["cell_steps"])
        flushes.append(st["tally_flushes"])
        if dn is not None:
            ms_d.append(dn.timing())
        print(f"step {k + 1}/{args.steps}: transport {st['ms_transport']:.1f} ms, imaging "
              f"{st['ms_image']:.1f} ms" + (f", denoiser {ms_d[-1]['ms_total']:.2f} ms" if ms_d else ""),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    ms_per_step = 1000.0 * elapsed / args.steps
    packets = args.packets
    value = packets * args.steps / elapsed
    img = ctx.images()
    assert np.isfinite(img).all()
    avg_t = float(np.mean(ms_t))
    bytes_launch = float(np.mean(steps)) * BYTES_PER_STEP_SPHERE
    achieved = bytes_launch / (avg_t * 1e-3) / 1e9
    traffic = counter_traffic()
    copy_gbs = copy_bandwidth()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "flared disk 256^3, 1e8 packets, 8 inclinations, 256x256 IQUV maps",
                   "grid": 256, "packets": packets, "views": 8, "npix": 256,
                   "midplane_tau": 1.0e4, "albedo": 0.5, "grains": "Rayleigh spheres",
                   "transport": "fp32, fp64 coherency tally", "seed": cfg["opts"]["seed"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "detail": {"kernel": "k_transport32<false,true,false,false,false>",
                   "schedule": opts,
                   "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, "
                                   "profiles/k_transport_disk256_1e8.md)",
                   "algorithmic_gb_per_launch": bytes_launch / 1e9,
                   "transport_ms": avg_t, "imaging_ms": float(np.mean(ms_i)),
                   "cell_steps_per_launch": float(np.mean(steps)),
                   "cell_steps_per_s": float(np.mean(steps)) / (avg_t * 1e-3),
                   "algorithmic_bytes_per_cell_step": BYTES_PER_STEP_SPHERE,
                   "traffic_over_algorithmic": None if traffic is None else traffic * 1e9 / bytes_launch,
                   "measured_copy_gbs": copy_gbs,
                   "frac_of_measured_copy": achieved / copy_gbs,
                   "scatterings": st["scatterings"], "rr_kills": st["rr_kills"]},
    }
    if dn is not None:
        inf = {k: float(np.mean([t[k] for t in ms_d])) for k in ms_d[0]}
        d = {"widths": list(dn.widths), "params": dn.n, "batch": nv, "npix": npix,
             "infer": "mean over the 8 dihedral transforms (8 forward passes)",
             "infer_ms": inf["ms_total"], "infer_conv_ms": inf["ms_conv"],
             "infer_conv_tflops": inf["conv_flop"] / (inf["ms_conv"] * 1e-3) / 1e12}
        d["infer_conv_mfma_frac"] = d["infer_conv_tflops"] / BF16_PEAK_TFLOPS
        # one forward pass, for reference (outside the step)
        one = []
        for _ in range(4):
            dn.infer(maps, den)
            one.append(dn.timing()["ms_total"])
        d["infer_one_pass_ms"] = float(np.mean(one[1:]))
        if args.train_steps > 0:
            # training on the step's maps (input and target the same here: the
            # cost of a step does not depend on the data)
            dn.train_step(maps, den, 1e-4)
            tr = []
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.train_steps):
                dn.train_step(maps, den, 1e-4)
                tr.append(dn.timing())
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t1) / args.train_steps
            tt = {k: float(np.mean([t[k] for t in tr])) for k in tr[0]}
            d.update({"train_step_ms_wall": 1e3 * wall, "train_step_ms_device": tt["ms_total"],
                      "train_conv_ms": tt["ms_conv"], "train_wgrad_ms": tt["ms_wgrad"],
                      "train_other_ms": tt["ms_other"],
                      "train_conv_tflops": tt["conv_flop"] / (tt["ms_conv"] * 1e-3) / 1e12,
                      "train_wgrad_tflops": tt["wgrad_flop"] / (tt["ms_wgrad"] * 1e-3) / 1e12,
                      "train_images_per_s": nv / wall})
            d["train_conv_mfma_frac"] = d["train_conv_tflops"] / BF16_PEAK_TFLOPS
            d["train_wgrad_mfma_frac"] = d["train_wgrad_tflops"] / BF16_PEAK_TFLOPS
        out["detail"]["denoiser"] = d
        dn.close()
    # the transport's binding resource: tally-line atomics, against what a
    # plain scatter-add of the same shape sustains on this device with the
    # most locality (consecutive lines: the bound) and with none (uniformly
    # random lines)
    cal_seq = atomic_calibration(order=1)
    cal = atomic_calibration(order=0)
    lines = float(np.mean(flushes))
    achieved = lines / (avg_t * 1e-3)
    out["detail"]["atomic_roofline"] = {
        "bound": "64-byte-line FP64 atomics (tally flush)",
        "achieved_lines_per_s": achieved, "calibrated_lines_per_s": cal_seq,
        "frac": achieved / cal_seq, "lines_per_launch": lines,
        "uniform_random_lines_per_s": cal, "frac_of_uniform_random": achieved / cal,
        "lines_unit": "tally cell blocks flushed per transport launch (kp_stats.tally_flushes), "
                      "one 64-byte block of six FP64 each",
        "calibration": "2^24 64-byte blocks of a [256^3][8] FP64 array, six FP64 atomics each in the "
                       "flush's lane pattern, consecutive (the bound) and uniformly random, best of 3 each "
                       "(bench.py --atomic-calibration, csrc/kp_calib.hip)"}
    if not args.no_cpu_baseline:
        print("timing the oracle on a bounded sample ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample, args.cpu_sample_1t)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
