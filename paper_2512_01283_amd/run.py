"""Run one of the seeded synthetic workloads through the library (step 1 and
step 2) and print one JSON line per run with its counters and kernel times.

    python -m paper_2512_01283_amd.run WORKLOAD [--runs K] [--packets N]
                                      [--precision auto|fp64|fp32] [--peel-off]

WORKLOAD is one of the names in WORKLOADS below (sizes as in workloads.py;
--packets overrides the packet count of a single-wavelength workload).
The grid is generated on the host, uploaded once, and the runs reuse it;
images stay on the device.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import workloads as W

WORKLOADS = {
    "uniform_sphere": W.uniform_sphere,
    "slab_clump": W.slab_clump,
    "flared_disk": W.flared_disk,
    "batched_disk": W.batched_disk,
    "dust_cylinder": W.dust_cylinder,
    "dust_cylinder_aligned": lambda **kw: W.dust_cylinder(aligned=True, **kw),
    "thermal_cube": W.thermal_cube,
    "table_disk": W.table_disk,
    "mesh_sphere": lambda **kw: W.mesh_sphere(rx=8, block=16, max_level=2, **kw),
    "uniform_sphere128": lambda **kw: W.uniform_sphere(n=128, **kw),
    "periodic_slab": W.periodic_slab,
}
PRECISION = {"auto": 0, "fp64": 1, "fp32": 2}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--runs", type=int, default=2)
    ap.add_argument("--packets", type=int, default=0)
    ap.add_argument("--precision", choices=sorted(PRECISION), default="auto")
    ap.add_argument("--peel-off", action="store_true", help="also form peel-off images")
    a = ap.parse_args(argv)
    import torch

    from . import polrad as P
    kw = {"packets": a.packets} if a.packets else {}
    cfg = WORKLOADS[a.workload](**kw)
    ctx = P.Context(0).load(cfg)
    total = sum(int(n) for n in cfg["packets"])
    for r in range(a.runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.run(transport_fp64=PRECISION[a.precision], peel_off=int(a.peel_off))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = ctx.stats()
        print(json.dumps({"workload": a.workload, "run": r, "packets": total, "wall_s": wall,
                          "packets_per_s": total / wall, "precision": a.precision,
                          **{k: st[k] for k in ("ms_transport", "ms_image", "cell_steps", "scatterings",
                                                "tally_flushes", "escaped", "rr_kills", "budget")}}),
              flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
