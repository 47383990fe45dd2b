"""GPU parity of the dust's thermal emission (source kind 2: the alpha_abs B
term of eq. polarized-rt, Sec. 2.2) with the FP64 oracle, through the C ABI,
on the same seeded inputs and Philox streams: emission cells, positions,
directions and (for aligned grains) dichroic Stokes vectors drawn identically,
packets followed path by path, and step 2 with the thermal source term.

Bars as in test_gpu_parity.py: FP64 transport 1e-12 per packet (1e-10 for
aligned grains) and images to 1e-10 of the maximum when every packet is the
oracle's; FP32 transport on spheres 1e-5 per packet with identical event
sequences, images within 3 Monte Carlo sigma.
"""
import math

import numpy as np
import pytest

from paper_2512_01283_amd import workloads as W
from parity_util import compare_images_stat, compare_traces, gpu_run, oracle_batches, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O():
    from oracle import oracle as o
    o.lib()
    return o


def p_tau(tau, p0):
    return math.exp(-tau) * math.sinh(p0 * tau) / (1.0 - math.exp(-tau) * math.cosh(p0 * tau))


@pytest.mark.parametrize("tau", [1.0, 10.0, 30.0])
def test_emitting_dichroic_slab_both_steps(O, tau):
    """Sec. 3.3 through both steps: emission packets in the aligned,
    purely absorbing slab follow the oracle's paths, and the image is eq.
    ptau in every pixel (and the oracle's image to 1e-12)."""
    p0 = 0.3
    say(f"case: emission slab tau {tau}")
    cfg = W.emission_slab(tau_total=tau, p0=p0, packets=3000)
    ctx = gpu_run(cfg, trace_packets=3000, transport_fp64=1)
    _, tr_o, st_o = O.transport(cfg, traces=True, tally=False)
    compare_traces(ctx.traces(), tr_o, 1e-10, 1.0, f"emission slab {tau}")
    st = ctx.stats()
    assert abs(st["e_emitted"] - st_o["e_emitted"]) <= 1e-12 * st_o["e_emitted"]
    img = ctx.images()[0, 0]
    ref = O.image(cfg, None)[0]
    assert np.allclose(img, ref, rtol=1e-12, atol=1e-15)
    assert np.allclose(-img[1] / img[0], p_tau(tau, p0), rtol=1e-9)
    assert np.allclose(img[0], 1.0 - math.exp(-tau) * math.cosh(p0 * tau), rtol=1e-10)


def test_thermal_cube_fp64_path_by_path(O):
    """Isothermal thick cube (albedo 0.5): every packet follows the oracle's
    path to 1e-12 and the images agree to 1e-10 of their maximum."""
    say("case: thermal cube 32^3 fp64 4e4 packets")
    cfg = W.thermal_cube(n=32, packets=40_000, tau_half=5.0)
    ctx = gpu_run(cfg, trace_packets=2000, transport_fp64=1)
    img_o, _, tr_o, st_o = O.run(cfg, traces=True)
    compare_traces(ctx.traces(), tr_o[:2000], 1e-12, 1.0, "thermal cube fp64")
    st = ctx.stats()
    for k in ("cell_steps", "scatterings", "escaped", "rr_kills", "packets"):
        assert st[k] == st_o.get(k, st[k]), k
    assert abs(st["e_emitted"] - st_o["e_emitted"]) <= 1e-12 * st_o["e_emitted"]
    img = ctx.images()[0]
    d = np.abs(img - img_o).max() / np.abs(img_o[:, 0]).max()
    say(f"thermal cube image max |d|/I_max = {d:.3e}")
    assert d < 1e-10
    bal = st["e_escaped"] + st["e_absorbed"] + st["e_rr_killed"] - st["e_rr_gained"] + st["e_budget"]
    assert abs(bal - st["e_emitted"] - st["e_scat_delta"]) < 1e-10 * st["e_emitted"]


def test_dust_cylinder_fp32(O):
    """The isothermal Gaussian dust cylinder (self-scattering of thermal
    emission) with Rayleigh spheres in the default FP32 mode: traced packets
    follow the oracle's event sequences to 1e-5, images (direct emission +
    scattered light) within 3 Monte Carlo sigma."""
    say("case: dust cylinder 64^3 fp32 4e4 packets")
    cfg = W.dust_cylinder(n=64, packets=40_000, npix=48)
    ctx = gpu_run(cfg, trace_packets=3000)
    _, tr_o, _ = O.transport(cfg, p_end=3000, tally=False, traces=True)
    compare_traces(ctx.traces(), tr_o, 1e-5, 1.0, "cylinder fp32")
    img_o, batches = oracle_batches(cfg)
    compare_images_stat(ctx.images()[0], img_o, batches, label="cylinder fp32")


def test_dust_cylinder_aligned(O):
    """The cylinder with oblate grains aligned across its axis: dichroic
    emission and extinction (automatic precision: FP64 for these grains),
    every traced packet matches the oracle to 1e-10, images within 3 sigma,
    and I >= |P| in every pixel."""
    say("case: dust cylinder 48^3 aligned 3e4 packets")
    cfg = W.dust_cylinder(n=48, packets=30_000, npix=32, aligned=True)
    ctx = gpu_run(cfg, trace_packets=2000)
    _, tr_o, _ = O.transport(cfg, p_end=2000, tally=False, traces=True)
    compare_traces(ctx.traces(), tr_o, 1e-10, 1.0, "cylinder aligned")
    img_o, batches = oracle_batches(cfg)
    img = ctx.images()[0]
    compare_images_stat(img, img_o, batches, label="cylinder aligned")
    P = np.sqrt(img[:, 1] ** 2 + img[:, 2] ** 2 + img[:, 3] ** 2)
    assert (P <= img[:, 0] * (1 + 1e-9) + 1e-300).all()


def test_emission_state_errors_and_static_entry_point():
    """Kind 2 without a source function (or with another wavelength count)
    is refused before any launch; kp_run_static runs thermal emission once
    kp_run has built the luminosity tables and then matches kp_run."""
    import torch

    from paper_2512_01283_amd import polrad as P
    cfg = W.thermal_cube(n=16, packets=5000, tau_half=3.0)
    ctx = P.Context(0)
    try:
        no_em = dict(cfg)
        no_em.pop("emission")
        ctx.load(no_em)
        with pytest.raises(P.KpError) as e:
            ctx.run()
        assert e.value.status == P.KP_ERR_STATE
        P.kp_set_emission(ctx.h, np.ones((2, 16 ** 3), np.float32))
        with pytest.raises(P.KpError) as e:
            ctx.run()
        assert e.value.status == P.KP_ERR_ARG
        bad = np.ones((1, 16 ** 3), np.float32)
        bad[0, 7] = -1.0
        with pytest.raises(P.KpError) as e:
            P.kp_set_emission(ctx.h, bad)
        assert e.value.status == P.KP_ERR_ARG
        zero = dict(cfg, emission=np.zeros((1, 16 ** 3), np.float32))
        ctx.load(zero)
        with pytest.raises(P.KpError) as e:
            ctx.run()
        assert e.value.status == P.KP_ERR_ARG
        ctx.load(cfg)
        out = torch.zeros((1, 1, 4, 32, 32), dtype=torch.float64, device="cuda")
        with pytest.raises(P.KpError) as e:
            P.kp_run_static(ctx.h, cfg["packets"], ctx.opts(transport_fp64=1), out)
        assert e.value.status == P.KP_ERR_STATE
        ctx.run(transport_fp64=1)
        ref = ctx.images()
        P.kp_run_static(ctx.h, cfg["packets"], ctx.opts(transport_fp64=1), out)
        d = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref[:, :, 0]).max()
        assert d <= 1e-12, d
    finally:
        ctx.close()
