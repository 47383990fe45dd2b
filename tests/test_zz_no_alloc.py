"""kp_run_static, the entry point that allocates nothing, against kp_run on
the same inputs, through the C ABI: two calls in a row on one context, the
second on a smaller grid with fewer packets (the static scratch keeps the
first call's contents and must be cleared by the second), then the size and
trace limits.  With FP64 transport the two entry points run the same kernels
on the same packet streams, so the counters are identical and the images
differ only by the order of the FP64 tally atomics (1e-12 of the image
maximum, the bar of the FP64 parity tests)."""
import numpy as np
import pytest

from paper_2512_01283_amd import workloads as W

pytestmark = pytest.mark.gpu


def _both(ctx, cfg, label, **kw):
    import torch

    from paper_2512_01283_amd import polrad as P
    print(f"case: {label}", flush=True)
    ctx.load(cfg)
    ctx.run(**kw)
    ref = ctx.images()
    st_ref = ctx.stats()
    out = torch.full(ref.shape, float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    P.kp_run_static(ctx.h, cfg["packets"], ctx.opts(**kw), out)
    got = out.cpu().numpy()
    st = ctx.stats()
    for k in ("cell_steps", "scatterings", "trials", "escaped", "rr_kills", "budget", "packets",
              "tally_flushes"):
        assert st[k] == st_ref[k], (label, k)
    scale = np.abs(ref[:, :, 0]).max()
    d = np.abs(got - ref).max() / scale
    print(f"{label}: max |static - kp_run| / I_max = {d:.3e}", flush=True)
    assert np.isfinite(got).all() and d <= 1e-12
    return got


def test_static_entry_point_matches_kp_run():
    from paper_2512_01283_amd import polrad as P
    ctx = P.Context(0)
    try:
        # 1: aligned oblate grains, 4 views (128-byte tally blocks, 64^3)
        big = W.slab_clump(n=64, packets=20000, npix=48)
        _both(ctx, big, "slab_clump64 aligned fp64 2e4 packets", transport_fp64=1)
        # 2: a smaller grid and fewer packets on the same context
        small = W.uniform_sphere(n=24, packets=5000, albedo=0.5, tau_radius=2.0, npix=32)
        _both(ctx, small, "sphere24 fp64 5e3 packets", transport_fp64=1)
        # 3: a flared disk with Russian roulette (8 views)
        disk = W.flared_disk(n=48, packets=20000, npix=32)
        _both(ctx, disk, "disk48 fp64 2e4 packets", transport_fp64=1)
    finally:
        ctx.close()


def test_static_entry_point_limits():
    import torch

    from paper_2512_01283_amd import polrad as P
    ctx = P.Context(0)
    try:
        cfg = W.uniform_sphere(n=32, packets=1000)
        ctx.load(cfg)
        shape = (1, 1, 4, 64, 64)
        out = torch.zeros(shape, dtype=torch.float64, device="cuda")
        # traces are not recorded by the static entry point
        with pytest.raises(P.KpError) as e:
            P.kp_run_static(ctx.h, [1000], ctx.opts(trace_packets=10), out)
        assert e.value.status == P.KP_ERR_ARG
        # a destination of the wrong size
        with pytest.raises(P.KpError) as e:
            P.kp_run_static(ctx.h, [1000], ctx.opts(), out[..., :32].contiguous())
        assert e.value.status == P.KP_ERR_ARG
        # a tally beyond the 256 MiB of the scratch (170^3 cells x 64 B = 314 MB)
        big = W.uniform_sphere(n=170, packets=1000)
        ctx.load(big)
        with pytest.raises(P.KpError) as e:
            P.kp_run_static(ctx.h, [1000], ctx.opts(), out)
        assert e.value.status == P.KP_ERR_ARG and "static scratch" in str(e.value)
        # the context still runs after the rejected calls
        ctx.load(cfg)
        P.kp_run_static(ctx.h, [1000], ctx.opts(), out)
        assert np.isfinite(out.cpu().numpy()).all() and ctx.stats()["packets"] == 1000
    finally:
        ctx.close()
