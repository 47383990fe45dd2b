"""ctypes wrapper of the FP64 CPU oracle (``liboracle_polrad.so``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.

The C sources beside this file state, routine by routine, which passage of
the paper (Yang & Wang, arXiv:2512.01283) each step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_polrad.so")
SRC = os.path.join(HERE, "polrad_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
               "-Wno-unused-parameter", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Mesh(C.Structure):
    _fields_ = [("rx", C.c_int32), ("ry", C.c_int32), ("rz", C.c_int32), ("block", C.c_int32),
                ("max_level", C.c_int32), ("n_nodes", C.c_int32), ("child", C.POINTER(C.c_int32))]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("dx", C.c_double), ("boundary", C.c_int32), ("mesh", C.POINTER(Mesh))]


class Dust(C.Structure):
    _fields_ = [("kappa_sca", C.c_double), ("kappa_abs", C.c_double),
                ("a_perp_re", C.c_double), ("a_perp_im", C.c_double),
                ("a_par_re", C.c_double), ("a_par_im", C.c_double),
                ("alpha3_scale", C.c_double), ("n_theta", C.c_int32),
                ("Z", C.POINTER(C.c_double))]


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos", C.c_double * 3),
                ("dir", C.c_double * 3), ("lum", C.c_double),
                ("B", C.POINTER(C.c_float))]


class View(C.Structure):
    _fields_ = [("theta", C.c_double), ("phi", C.c_double),
                ("npx", C.c_int32), ("npy", C.c_int32),
                ("half_width", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("rr_wmin", C.c_double),
                ("rr_psurv", C.c_double), ("max_events", C.c_int64),
                ("nthreads", C.c_int32)]


class Trace(C.Structure):
    _fields_ = [("packet", C.c_uint64), ("end_kind", C.c_int32),
                ("events", C.c_int32), ("steps", C.c_int64),
                ("last_cell", C.c_int64), ("n", C.c_double * 3),
                ("stokes", C.c_double * 4), ("hash", C.c_uint64),
                ("tau_path", C.c_double)]


class Stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in
                ("cell_steps", "scatterings", "trials", "rr_kills",
                 "rr_survivals", "escaped", "budget", "numeric")] + \
               [(k, C.c_double) for k in
                ("e_emitted", "e_escaped", "e_absorbed", "e_rr_killed",
                 "e_rr_gained", "e_budget", "e_scat_delta")]


TRACE_DTYPE = np.dtype([("packet", "<u8"), ("end_kind", "<i4"), ("events", "<i4"),
                        ("steps", "<i8"), ("last_cell", "<i8"), ("n", "<f8", 3),
                        ("stokes", "<f8", 4), ("hash", "<u8"), ("tau_path", "<f8")])
assert TRACE_DTYPE.itemsize == C.sizeof(Trace)

END_ESCAPE, END_RR_KILL, END_BUDGET, END_NUMERIC = 2, 4, 5, 6

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        dp, fp = C.POINTER(C.c_double), C.POINTER(C.c_float)
        u64p = C.POINTER(C.c_uint64)
        L.kpo_transport.argtypes = [C.POINTER(Grid), fp, fp, C.POINTER(Dust), C.c_int32,
                                    C.POINTER(Source), C.c_int32, C.POINTER(View),
                                    C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(Opts),
                                    dp, C.c_void_p, C.POINTER(Stats)]
        L.kpo_transport_peel.argtypes = [C.POINTER(Grid), fp, fp, C.POINTER(Dust), C.c_int32,
                                         C.POINTER(Source), C.c_int32, C.POINTER(View),
                                         C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(Opts),
                                         dp, dp, C.POINTER(Stats)]
        L.kpo_trace_packets.argtypes = [C.POINTER(Grid), fp, fp, C.POINTER(Dust), C.c_int32,
                                        C.POINTER(Source), u64p, C.c_uint64, C.c_uint64,
                                        C.POINTER(Opts), C.c_void_p]
        L.kpo_image.argtypes = [C.POINTER(Grid), fp, fp, C.POINTER(Dust), C.c_int32,
                                C.POINTER(View), dp, dp]
        L.kpo_image_thermal.argtypes = [C.POINTER(Grid), fp, fp, C.POINTER(Dust), C.c_int32,
                                        C.POINTER(View), dp, fp, dp]
        L.kpo_emit_state.argtypes = [C.POINTER(Grid), fp, fp, C.POINTER(Dust), fp, C.c_uint64,
                                     C.c_int32, C.c_uint64, C.c_double, C.POINTER(C.c_int64),
                                     dp, dp, dp]
        L.kpo_emission_luminosity.argtypes = [C.POINTER(Grid), fp, C.POINTER(Dust), fp]
        L.kpo_emission_luminosity.restype = C.c_double
        L.kpo_philox.argtypes = [u64p, u64p, u64p]
        L.kpo_uniform.argtypes = [C.c_uint64] * 4
        L.kpo_uniform.restype = C.c_double
        for name in ("kpo_quat_from_b",):
            getattr(L, name).argtypes = [dp, dp]
        for name in ("kpo_to_grain", "kpo_from_grain"):
            getattr(L, name).argtypes = [dp, dp, dp]
        L.kpo_basis.argtypes = [dp, dp, dp]
        L.kpo_eta.argtypes = [dp, dp]
        L.kpo_eta.restype = C.c_double
        L.kpo_rotate_stokes.argtypes = [C.c_double, dp, dp]
        L.kpo_alphas.argtypes = [C.POINTER(Dust), C.c_double, dp]
        L.kpo_mueller_lab.argtypes = [C.POINTER(Dust), dp, dp, dp, dp, dp]
        L.kpo_appA.argtypes = [C.c_double] * 4 + [dp, dp, dp]
        L.kpo_segment.argtypes = [C.c_double] * 4 + [dp, dp, dp]
        L.kpo_scatter_weight.argtypes = [C.POINTER(Dust), dp, dp, dp]
        L.kpo_scatter_weight.restype = C.c_double
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# array helpers
# --------------------------------------------------------------------------
def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _f(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def cell_count(g) -> int:
    """Cells of a grid record: nx ny nz, or block^3 per leaf of its mesh."""
    m = g.get("mesh")
    if m is None:
        return int(g["nx"]) * int(g["ny"]) * int(g["nz"])
    return int(np.sum(np.asarray(m["child"]) == -1)) * int(m["block"]) ** 3


def make_grid(g) -> Grid:
    """g["mesh"] (optional): dict(rx, ry, rz, block, max_level, child) of a
    composite mesh (reading M1); the arrays are kept alive on the result."""
    out = Grid(int(g["nx"]), int(g["ny"]), int(g["nz"]), float(g["x0"]),
               float(g["y0"]), float(g["z0"]), float(g["dx"]), int(g.get("boundary", 0)), None)
    m = g.get("mesh")
    if m is not None:
        child = np.ascontiguousarray(m["child"], dtype=np.int32)
        mesh = Mesh(int(m["rx"]), int(m["ry"]), int(m["rz"]), int(m["block"]), int(m["max_level"]),
                    len(child), child.ctypes.data_as(C.POINTER(C.c_int32)))
        out.mesh = C.pointer(mesh)
        out._keep = (child, mesh)
    return out


def make_dust(d) -> Dust:
    """d["table"] (optional): [n_theta][6] scattering-plane elements S11 S12
    S22 S33 S34 S44 at Theta uniform on [0, pi] (reading T1); the array is
    kept alive on the returned structure."""
    out = Dust(float(d["kappa_sca"]), float(d["kappa_abs"]),
               float(np.real(d["a_perp"])), float(np.imag(d["a_perp"])),
               float(np.real(d["a_par"])), float(np.imag(d["a_par"])),
               float(d.get("alpha3_scale", 0.0)), 0, None)
    if d.get("table") is not None:
        Z = np.ascontiguousarray(d["table"], dtype=np.float64)
        assert Z.ndim == 2 and Z.shape[1] == 6
        out.n_theta = Z.shape[0]
        out.Z = Z.ctypes.data_as(C.POINTER(C.c_double))
        out._keep = Z
    return out


def make_source(s, B=None) -> Source:
    """B: the source function [ncell] (float32, kept alive by the caller) of
    the wavelength, for thermal emission (kind 2)."""
    return Source(int(s.get("kind", 0)), (C.c_double * 3)(*s.get("pos", (0.0, 0.0, 0.0))),
                  (C.c_double * 3)(*s.get("dir", (0.0, 0.0, 1.0))), float(s.get("lum", 1.0)),
                  None if B is None else B.ctypes.data_as(C.POINTER(C.c_float)))


def emission_of(cfg, lam):
    """The source function of wavelength lam as float32 [ncell] when the
    source is the dust's thermal emission (kind 2), else None."""
    if int(cfg["source"].get("kind", 0)) != 2:
        return None
    return np.ascontiguousarray(np.asarray(cfg["emission"])[lam], dtype=np.float32)


def make_views(vs):
    arr = (View * len(vs))()
    for k, v in enumerate(vs):
        arr[k] = View(float(v["theta"]), float(v["phi"]), int(v["npx"]), int(v["npy"]),
                      float(v["half_width"]))
    return arr


def make_opts(o, nthreads=0) -> Opts:
    return Opts(int(o["seed"]), float(o.get("rr_wmin", 1e-3)), float(o.get("rr_psurv", 0.1)),
                int(o.get("max_events", 10000)), int(nthreads))


# --------------------------------------------------------------------------
# whole-run entry points
# --------------------------------------------------------------------------
def transport(cfg, lam=0, p_begin=0, p_end=None, n_total=None, tally=True,
              traces=False, nthreads=0):
    """Step 1 for one wavelength.  Returns (S or None, traces or None, stats)."""
    L = lib()
    g = make_grid(cfg["grid"])
    ncell = cell_count(cfg["grid"])
    rho, rho_p = _f(cfg["rho"])
    bh, bh_p = _f(cfg.get("bhat"))
    dust = make_dust(cfg["dust"][lam])
    B = emission_of(cfg, lam)
    src = make_source(cfg["source"], B)
    views = make_views(cfg["views"])
    nv = len(cfg["views"])
    n_total = int(cfg["packets"][lam]) if n_total is None else int(n_total)
    p_end = n_total if p_end is None else int(p_end)
    S = np.zeros((ncell, nv, 4)) if tally else None
    Sp = S.ctypes.data_as(C.POINTER(C.c_double)) if tally else None
    tr = np.zeros(p_end - p_begin, dtype=TRACE_DTYPE) if traces else None
    st = Stats()
    o = make_opts(cfg["opts"], nthreads)
    rc = L.kpo_transport(C.byref(g), rho_p, bh_p, C.byref(dust), lam, C.byref(src), nv,
                         views, p_begin, p_end, n_total, C.byref(o), Sp,
                         tr.ctypes.data if traces else None, C.byref(st))
    if rc != 0:
        raise ValueError(f"kpo_transport rejected its inputs ({rc})")
    return S, tr, stats_dict(st)


def transport_peel(cfg, lam=0, p_begin=0, p_end=None, n_total=None, tally=False, nthreads=0):
    """Step 1 for one wavelength with peel-off imaging: returns (peel-off
    images [view][4][npy][npx], S or None, stats).  Open boundaries."""
    L = lib()
    g = make_grid(cfg["grid"])
    ncell = cell_count(cfg["grid"])
    rho, rho_p = _f(cfg["rho"])
    bh, bh_p = _f(cfg.get("bhat"))
    dust = make_dust(cfg["dust"][lam])
    B = emission_of(cfg, lam)
    src = make_source(cfg["source"], B)
    views = make_views(cfg["views"])
    nv = len(cfg["views"])
    npx, npy = cfg["views"][0]["npx"], cfg["views"][0]["npy"]
    n_total = int(cfg["packets"][lam]) if n_total is None else int(n_total)
    p_end = n_total if p_end is None else int(p_end)
    S = np.zeros((ncell, nv, 4)) if tally else None
    Sp = S.ctypes.data_as(C.POINTER(C.c_double)) if tally else None
    peel = np.zeros((nv, 4, npy, npx))
    st = Stats()
    o = make_opts(cfg["opts"], nthreads)
    rc = L.kpo_transport_peel(C.byref(g), rho_p, bh_p, C.byref(dust), lam, C.byref(src), nv,
                              views, p_begin, p_end, n_total, C.byref(o), Sp,
                              peel.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st))
    if rc != 0:
        raise ValueError(f"kpo_transport_peel rejected its inputs ({rc})")
    return peel, S, stats_dict(st)


def trace_packets(cfg, ids, lam=0, n_total=None, nthreads=0):
    L = lib()
    g = make_grid(cfg["grid"])
    rho, rho_p = _f(cfg["rho"])
    bh, bh_p = _f(cfg.get("bhat"))
    dust = make_dust(cfg["dust"][lam])
    B = emission_of(cfg, lam)
    src = make_source(cfg["source"], B)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    n_total = int(cfg["packets"][lam]) if n_total is None else int(n_total)
    tr = np.zeros(len(ids), dtype=TRACE_DTYPE)
    o = make_opts(cfg["opts"], nthreads)
    rc = L.kpo_trace_packets(C.byref(g), rho_p, bh_p, C.byref(dust), lam, C.byref(src),
                             ids.ctypes.data_as(C.POINTER(C.c_uint64)), len(ids), n_total,
                             C.byref(o), tr.ctypes.data)
    if rc != 0:
        raise ValueError(f"kpo_trace_packets rejected its inputs ({rc})")
    return tr


def image(cfg, S, lam=0):
    """Step 2 for one wavelength; returns images [view][4][npy][npx].  S may
    be None (no scattering source); with a thermal-emission source (kind 2)
    the dust's emission is added to the source."""
    L = lib()
    g = make_grid(cfg["grid"])
    rho, rho_p = _f(cfg["rho"])
    bh, bh_p = _f(cfg.get("bhat"))
    dust = make_dust(cfg["dust"][lam])
    views = make_views(cfg["views"])
    nv = len(cfg["views"])
    npx, npy = cfg["views"][0]["npx"], cfg["views"][0]["npy"]
    Sp = None
    if S is not None:
        S, Sp = _d(S)
    B, Bp = _f(emission_of(cfg, lam))
    out = np.zeros((nv, 4, npy, npx))
    rc = L.kpo_image_thermal(C.byref(g), rho_p, bh_p, C.byref(dust), nv, views, Sp, Bp,
                             out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise ValueError(f"kpo_image rejected its inputs ({rc})")
    return out


def run(cfg, lam=0, nthreads=0, traces=False):
    """Both steps for one wavelength: (images, S, traces, stats)."""
    S, tr, st = transport(cfg, lam=lam, traces=traces, nthreads=nthreads)
    return image(cfg, S, lam=lam), S, tr, st


def emit_state(cfg, packet, lam=0, w=1.0):
    """Thermal emission draw of one packet: (cell, position in the cell,
    direction, Stokes vector) for a packet weight w."""
    L = lib()
    g = make_grid(cfg["grid"])
    rho, rho_p = _f(cfg["rho"])
    bh, bh_p = _f(cfg.get("bhat"))
    dust = make_dust(cfg["dust"][lam])
    B, Bp = _f(emission_of(cfg, lam))
    cell = C.c_int64()
    pos, n, s = np.zeros(3), np.zeros(3), np.zeros(4)
    dp = C.POINTER(C.c_double)
    rc = L.kpo_emit_state(C.byref(g), rho_p, bh_p, C.byref(dust), Bp, int(cfg["opts"]["seed"]), lam,
                          int(packet), float(w), C.byref(cell), pos.ctypes.data_as(dp),
                          n.ctypes.data_as(dp), s.ctypes.data_as(dp))
    if rc != 0:
        raise ValueError("kpo_emit_state rejected its inputs")
    return int(cell.value), pos, n, s


def emission_luminosity(cfg, lam=0):
    """4 pi sum_c rho_c kappa_abs B_c V over the grid."""
    g = make_grid(cfg["grid"])
    rho, rho_p = _f(cfg["rho"])
    dust = make_dust(cfg["dust"][lam])
    B, Bp = _f(emission_of(cfg, lam))
    return float(lib().kpo_emission_luminosity(C.byref(g), rho_p, C.byref(dust), Bp))


def stats_dict(st: Stats) -> dict:
    return {k: getattr(st, k) for k, _ in Stats._fields_}


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    P = C.POINTER(C.c_uint64)
    lib().kpo_philox(c.ctypes.data_as(P), k.ctypes.data_as(P), o.ctypes.data_as(P))
    return o


def uniform(seed, lam, packet, draw):
    return lib().kpo_uniform(seed, lam, packet, draw)


def _vec_call(fn, *arrays, out_len):
    args, keep = [], []
    for a in arrays:
        a, p = _d(a)
        keep.append(a)
        args.append(p)
    out = np.zeros(out_len)
    fn(*args, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def quat_from_b(b):
    return _vec_call(lib().kpo_quat_from_b, b, out_len=4)


def to_grain(q, v):
    return _vec_call(lib().kpo_to_grain, q, v, out_len=3)


def from_grain(q, v):
    return _vec_call(lib().kpo_from_grain, q, v, out_len=3)


def basis(n):
    n, p = _d(n)
    th, ph = np.zeros(3), np.zeros(3)
    lib().kpo_basis(p, th.ctypes.data_as(C.POINTER(C.c_double)),
                    ph.ctypes.data_as(C.POINTER(C.c_double)))
    return th, ph


def eta(q, n):
    q, qp = _d(q)
    n, np_ = _d(n)
    return lib().kpo_eta(qp, np_)


def rotate_stokes(e, s):
    s, sp = _d(s)
    out = np.zeros(4)
    lib().kpo_rotate_stokes(float(e), sp, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def alphas(dust, cos_t):
    d = make_dust(dust)
    out = np.zeros(3)
    lib().kpo_alphas(C.byref(d), float(cos_t), out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def mueller_lab(dust, q, m, n, s):
    d = make_dust(dust)
    arrs = [_d(x) for x in (q, m, n, s)]
    out = np.zeros(4)
    lib().kpo_mueller_lab(C.byref(d), *[p for _, p in arrs],
                          out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def appA(a1, a2, a3, dtau, src, s_in):
    src, sp = _d(src)
    s_in, ip = _d(s_in)
    out = np.zeros(4)
    lib().kpo_appA(a1, a2, a3, dtau, sp, ip, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def segment(m1, m2, m3, length, s_in):
    s_in, ip = _d(s_in)
    integ, out = np.zeros(4), np.zeros(4)
    lib().kpo_segment(m1, m2, m3, length, ip, integ.ctypes.data_as(C.POINTER(C.c_double)),
                      out.ctypes.data_as(C.POINTER(C.c_double)))
    return integ, out


def scatter_weight(dust, q, n, s):
    d = make_dust(dust)
    arrs = [_d(x) for x in (q, n, s)]
    return lib().kpo_scatter_weight(C.byref(d), *[p for _, p in arrs])


def scatter_sample(dust, q, n, s, seed=0, lam=0, packet=0, first_draw=0):
    """One scattering event from the stream (seed, lam, packet) starting at
    first_draw: returns (m, stokes_out, trials); raises if it fails."""
    L = lib()
    if not getattr(L.kpo_scatter_sample, "_typed", False):
        dp = C.POINTER(C.c_double)
        L.kpo_scatter_sample.argtypes = [C.POINTER(Dust), dp, dp, dp, C.c_uint64, C.c_uint64,
                                         C.c_uint64, C.c_uint64, dp, dp,
                                         C.POINTER(C.c_int64)]
        L.kpo_scatter_sample._typed = True
    d = make_dust(dust)
    arrs = [_d(x) for x in (q, n, s)]
    m, so = np.zeros(3), np.zeros(4)
    tr = C.c_int64(0)
    rc = L.kpo_scatter_sample(C.byref(d), *[p for _, p in arrs], seed, lam, packet, first_draw,
                              m.ctypes.data_as(C.POINTER(C.c_double)),
                              so.ctypes.data_as(C.POINTER(C.c_double)), C.byref(tr))
    if rc != 0:
        raise RuntimeError("scattering event failed (bound violated or no acceptance)")
    return m, so, tr.value
