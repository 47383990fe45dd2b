"""Autotuner for the persistent transport launch.

Searches the launch and scheduling parameters of ``kp_transport`` --
threads per block, resident blocks per compute unit, and the two knobs of
the wavefront-batched scattering events -- by coordinate descent, timing
each candidate with the transport kernel's own HIP-event time on a reduced
packet count of the real workload (same grid, grains, views and
wavelengths).  None of these parameters changes any packet's path or any
result; they only change the schedule.

Results are cached in ``tuning.json`` beside this file, keyed by the
workload's structure and the device name, so that a production run or the
benchmark picks the tuned schedule without searching again:

    python -m paper_2512_01283_amd.autotune disk      # tune the 256^3 disk
    python -m paper_2512_01283_amd.autotune disk batched --measure
        # tune both, then time each whole workload with the default and the
        # tuned schedule (one warm-up run each) and print one JSON line
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")

SPACE = {
    "block_size": [64, 128, 256],
    "blocks_per_cu": [1, 2, 4, 8],
    "scatter_batch": [1, 4, 8, 16, 32],
    "scatter_wait": [4, 16, 64],
}
DEFAULT = {"block_size": 256, "blocks_per_cu": 0, "scatter_batch": 8, "scatter_wait": 16}


def workload_key(cfg, device_name: str) -> str:
    g = cfg["grid"]
    sphere = all(complex(d["a_perp"]) == complex(d["a_par"]) for d in cfg["dust"])
    return (f"{cfg.get('name', 'workload')}|{g['nx']}x{g['ny']}x{g['nz']}|lam{len(cfg['dust'])}|"
            f"views{len(cfg['views'])}|{'sphere' if sphere else 'aligned'}|"
            f"{cfg.get('precision', 'f32')}|{device_name}")


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def tuned_opts(cfg, device_name: str) -> dict:
    """The cached schedule for this workload on this device, or {}."""
    ent = load_cache().get(workload_key(cfg, device_name))
    return dict(ent["opts"]) if ent else {}


def _time(ctx, counts, opts, repeats):
    best = float("inf")
    for _ in range(repeats):
        ctx.transport(counts, **opts)
        best = min(best, ctx.stats()["ms_transport"])
    return best


def tune(cfg, scale: float = 0.1, repeats: int = 1, sweeps: int = 2, space=None, log=print):
    """Coordinate descent over `space` on `scale` x the workload's packets.
    Returns (best opts, best ms, trials)."""
    import torch

    from . import polrad as P

    space = space or SPACE
    counts = [max(1, int(round(n * scale))) for n in cfg["packets"]]
    ctx = P.Context(0).load(cfg)
    cur = dict(DEFAULT)
    trials = {}

    def cost(o):
        k = tuple(sorted(o.items()))
        if k not in trials:
            trials[k] = _time(ctx, counts, o, repeats)
            log(f"  {o} -> {trials[k]:.1f} ms")
        return trials[k]

    best = cost(cur)
    for _ in range(sweeps):
        improved = False
        for name, values in space.items():
            for v in values:
                cand = dict(cur, **{name: v})
                t = cost(cand)
                if t < best * 0.995:
                    best, cur, improved = t, cand, True
        if not improved:
            break
    ctx.close()
    torch.cuda.synchronize()
    return cur, best, [(dict(k), v) for k, v in trials.items()]


def save(cfg, device_name: str, opts: dict, ms: float, scale: float) -> None:
    cache = load_cache()
    cache[workload_key(cfg, device_name)] = {
        "opts": opts, "ms_transport_at_scale": ms, "packet_scale": scale,
        "date": time.strftime("%Y-%m-%d %H:%M:%S"),
    }
    with open(CACHE + ".tmp", "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(CACHE + ".tmp", CACHE)


def measure(cfg, opts, label):
    """Whole-workload kp_run with the given schedule: one warm-up run, then
    one timed run (HIP-event kernel times, wall clock around kp_run)."""
    import torch

    from . import polrad as P
    ctx = P.Context(0).load(cfg)
    ctx.run(**opts)
    t0 = time.perf_counter()
    ctx.run(**opts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.stats()
    ctx.close()
    return {"schedule": label, "opts": opts, "ms_transport": st["ms_transport"], "ms_image": st["ms_image"],
            "wall_s": wall, "packets": int(st["packets"]), "packets_per_s": st["packets"] / wall,
            "cell_steps": int(st["cell_steps"]), "scatterings": int(st["scatterings"])}


def main(argv):
    import torch

    from . import workloads as W
    names = [a for a in argv[1:] if not a.startswith("--")] or ["disk"]
    dev = torch.cuda.get_device_name(0)
    out = {"device": dev}
    for which in names:
        if which == "disk":
            cfg, scale = W.flared_disk(), 0.1
        elif which == "batched":
            cfg, scale = W.batched_disk(), 0.05
        elif which == "slab":
            cfg, scale = W.slab_clump(), 0.5
        else:
            raise SystemExit(f"unknown workload {which!r} (disk, batched, slab)")
        print(f"tuning {cfg['name']} on {dev} at {scale} x packets", flush=True)
        opts, ms, trials = tune(cfg, scale=scale, log=lambda m: print(m, flush=True))
        save(cfg, dev, opts, ms, scale)
        rec = {"opts": opts, "ms_at_scale": ms, "packet_scale": scale,
               "trials": [{"opts": o, "ms": t} for o, t in trials]}
        if "--measure" in argv:
            rec["whole"] = [measure(cfg, {}, "default"), measure(cfg, opts, "tuned")]
            for r in rec["whole"]:
                print(json.dumps(r), flush=True)
        out[cfg["name"]] = rec
    print(json.dumps(out))


if __name__ == "__main__":
    main(sys.argv)
