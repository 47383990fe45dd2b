"""Thin ctypes binding of libpolrad.so (include/polrad.h).

Argument marshalling only: every step of the transport and imaging runs in
the library's HIP kernels.  Device memory and streams come from PyTorch
(``torch.cuda`` tensors and ``torch.cuda.current_stream()``).  The module
raises at import if the compiled library is missing -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpolrad.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "polrad.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2512_01283_amd.build` "
        "(hipcc, gfx950); the transport has no CPU fallback")

# PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).
# Loading torch first makes the dynamic loader bind libpolrad.so to that one
# runtime, so device pointers and streams from torch are valid in the library
# (two HIP runtimes in one process do not share devices).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

KP_OK, KP_ERR_ARG, KP_ERR_OOM, KP_ERR_DEVICE, KP_ERR_STATE, KP_ERR_NUMERIC, KP_ERR_BUDGET = range(7)
STATUS = {0: "KP_OK", 1: "KP_ERR_ARG", 2: "KP_ERR_OOM", 3: "KP_ERR_DEVICE", 4: "KP_ERR_STATE",
          5: "KP_ERR_NUMERIC", 6: "KP_ERR_BUDGET"}


class KpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class kp_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("dx", C.c_double), ("boundary", C.c_int32)]


class kp_dust(C.Structure):
    _fields_ = [("kappa_sca", C.c_double), ("kappa_abs", C.c_double),
                ("a_perp", C.c_double * 2), ("a_par", C.c_double * 2),
                ("alpha3_scale", C.c_double)]


class kp_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos", C.c_double * 3), ("dir", C.c_double * 3),
                ("lum", C.c_double)]


class kp_view(C.Structure):
    _fields_ = [("theta", C.c_double), ("phi", C.c_double), ("npx", C.c_int32),
                ("npy", C.c_int32), ("half_width", C.c_double)]


class kp_mesh(C.Structure):
    _fields_ = [("rx", C.c_int32), ("ry", C.c_int32), ("rz", C.c_int32), ("block", C.c_int32),
                ("max_level", C.c_int32), ("n_nodes", C.c_int32), ("x0", C.c_double), ("y0", C.c_double),
                ("z0", C.c_double), ("dx", C.c_double)]


class kp_opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("transport_fp64", C.c_int32),
                ("tally_mode", C.c_int32), ("rr_wmin", C.c_double),
                ("rr_psurv", C.c_double), ("max_events", C.c_int64),
                ("trace_packets", C.c_uint32), ("trace_stride", C.c_uint32),
                ("block_size", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("strict", C.c_int32), ("scatter_batch", C.c_int32),
                ("scatter_wait", C.c_int32), ("peel_off", C.c_int32)]


class kp_stats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in
                ("cell_steps", "scatterings", "trials", "rr_kills", "rr_survivals",
                 "escaped", "budget", "numeric")] + \
               [(k, C.c_double) for k in
                ("e_emitted", "e_escaped", "e_absorbed", "e_rr_killed", "e_rr_gained",
                 "e_budget", "e_scat_delta", "ms_transport", "ms_image")] + \
               [("packets", C.c_int64), ("tally_flushes", C.c_int64)]


TRACE_DTYPE = np.dtype([("packet", "<u8"), ("end_kind", "<i4"), ("events", "<i4"),
                        ("steps", "<i8"), ("last_cell", "<i8"), ("n", "<f8", 3),
                        ("stokes", "<f8", 4), ("hash", "<u8"), ("tau_path", "<f8")])

_P = C.c_void_p
_dp = C.POINTER(C.c_double)
_SIGS = {
    "kp_create": ([C.c_int, C.POINTER(_P)], C.c_int),
    "kp_destroy": ([_P], None),
    "kp_last_error": ([_P], C.c_char_p),
    "kp_set_grid": ([_P, C.POINTER(kp_grid), _P, _P], C.c_int),
    "kp_set_grid_device": ([_P, C.POINTER(kp_grid), _P, _P], C.c_int),
    "kp_set_mesh": ([_P, C.POINTER(kp_mesh), _P, _P, _P], C.c_int),
    "kp_set_dust": ([_P, C.c_int32, C.POINTER(kp_dust)], C.c_int),
    "kp_set_source": ([_P, C.POINTER(kp_source)], C.c_int),
    "kp_set_emission": ([_P, C.c_int32, _P], C.c_int),
    "kp_set_dust_tables": ([_P, C.c_int32, C.c_int32, _P], C.c_int),
    "kp_set_views": ([_P, C.c_int32, C.POINTER(kp_view)], C.c_int),
    "kp_run": ([_P, C.POINTER(C.c_uint64), C.POINTER(kp_opts), _P], C.c_int),
    "kp_run_static": ([_P, C.POINTER(C.c_uint64), C.POINTER(kp_opts), _P, C.c_size_t, _P], C.c_int),
    "kp_transport": ([_P, C.POINTER(C.c_uint64), C.POINTER(kp_opts), _P], C.c_int),
    "kp_image": ([_P, _P], C.c_int),
    "kp_image_source": ([_P, _P, _P, _P], C.c_int),
    "kp_get_images": ([_P, _P, C.c_size_t], C.c_int),
    "kp_get_images_device": ([_P, _P, C.c_size_t, _P], C.c_int),
    "kp_get_peel_images": ([_P, _P, C.c_size_t], C.c_int),
    "kp_get_tally": ([_P, _P, C.c_size_t], C.c_int),
    "kp_get_view_tally": ([_P, _P, C.c_size_t], C.c_int),
    "kp_get_stats": ([_P, C.POINTER(kp_stats)], C.c_int),
    "kp_get_trace": ([_P, _P, C.c_size_t], C.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def header_symbols() -> list[str]:
    """Entry points declared in include/polrad.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:kp_status|void|const char \*)\s*(kp_\w+)\s*\(", txt, re.M)))


# --------------------------------------------------------------------------
# the C entry points under their own names (status codes become KpError)
# --------------------------------------------------------------------------
def _check(ctx, st):
    if st != KP_OK:
        msg = _lib.kp_last_error(ctx).decode() if ctx else ""
        raise KpError(st, msg)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _ptr(t):
    return None if t is None else C.c_void_p(int(t.data_ptr()))


def kp_create(device: int = 0) -> C.c_void_p:
    h = _P()
    st = _lib.kp_create(int(device), C.byref(h))
    if st != KP_OK:
        raise KpError(st, f"kp_create(device={device}) failed")
    return h


def kp_destroy(ctx) -> None:
    _lib.kp_destroy(ctx)


def kp_last_error(ctx) -> str:
    return _lib.kp_last_error(ctx).decode()


def make_grid(g) -> kp_grid:
    return kp_grid(int(g["nx"]), int(g["ny"]), int(g["nz"]), float(g["x0"]), float(g["y0"]),
                   float(g["z0"]), float(g["dx"]), int(g.get("boundary", 0)))


def kp_set_grid(ctx, grid, rho: np.ndarray, bhat: np.ndarray | None) -> None:
    rho = np.ascontiguousarray(rho, dtype=np.float32)
    bh = None if bhat is None else np.ascontiguousarray(bhat, dtype=np.float32)
    g = make_grid(grid)
    _check(ctx, _lib.kp_set_grid(ctx, C.byref(g), rho.ctypes.data_as(_P),
                                 None if bh is None else bh.ctypes.data_as(_P)))


def kp_set_grid_device(ctx, grid, d_rho, d_bhat=None) -> None:
    """d_rho, d_bhat: contiguous float32 torch.cuda tensors (borrowed)."""
    for t in (d_rho, d_bhat):
        if t is not None:
            assert t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float32"
    g = make_grid(grid)
    _check(ctx, _lib.kp_set_grid_device(ctx, C.byref(g), _ptr(d_rho), _ptr(d_bhat)))


def kp_set_mesh(ctx, grid, rho: np.ndarray, bhat: np.ndarray | None) -> None:
    """grid: a grid record with a "mesh" entry (see workloads.make_mesh_grid)."""
    m = grid["mesh"]
    child = np.ascontiguousarray(m["child"], dtype=np.int32)
    rho = np.ascontiguousarray(rho, dtype=np.float32)
    mm = kp_mesh(int(m["rx"]), int(m["ry"]), int(m["rz"]), int(m["block"]), int(m["max_level"]), len(child),
                 float(grid["x0"]), float(grid["y0"]), float(grid["z0"]), float(grid["dx"]))
    bp = None
    if bhat is not None:
        bhat = np.ascontiguousarray(bhat, dtype=np.float32)
        bp = bhat.ctypes.data_as(_P)
    _check(ctx, _lib.kp_set_mesh(ctx, C.byref(mm), child.ctypes.data_as(_P), rho.ctypes.data_as(_P), bp))


def make_dust(d) -> kp_dust:
    ap, aa = complex(d["a_perp"]), complex(d["a_par"])
    return kp_dust(float(d["kappa_sca"]), float(d["kappa_abs"]), (C.c_double * 2)(ap.real, ap.imag),
                   (C.c_double * 2)(aa.real, aa.imag), float(d.get("alpha3_scale", 0.0)))


def kp_set_dust(ctx, dust_list) -> None:
    arr = (kp_dust * len(dust_list))(*[make_dust(d) for d in dust_list])
    _check(ctx, _lib.kp_set_dust(ctx, len(dust_list), arr))


def kp_set_dust_tables(ctx, Z) -> None:
    """Z: [n_lambda][n_theta][6] scattering-plane tables (float64), or None
    to return to dipole grains."""
    if Z is None:
        _check(ctx, _lib.kp_set_dust_tables(ctx, 0, 0, None))
        return
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    assert Z.ndim == 3 and Z.shape[2] == 6
    _check(ctx, _lib.kp_set_dust_tables(ctx, Z.shape[0], Z.shape[1], Z.ctypes.data_as(_P)))


def kp_set_source(ctx, src) -> None:
    s = kp_source(int(src.get("kind", 0)), (C.c_double * 3)(*src["pos"]),
                  (C.c_double * 3)(*src.get("dir", (0.0, 0.0, 1.0))), float(src["lum"]))
    _check(ctx, _lib.kp_set_source(ctx, C.byref(s)))


def kp_set_emission(ctx, B: np.ndarray) -> None:
    """B: float32 [n_lambda, ncell] source function of the dust's thermal emission."""
    B = np.ascontiguousarray(B, dtype=np.float32)
    if B.ndim == 1:
        B = B[None]
    _check(ctx, _lib.kp_set_emission(ctx, B.shape[0], B.ctypes.data_as(_P)))


def kp_set_views(ctx, views) -> None:
    arr = (kp_view * len(views))(*[kp_view(float(v["theta"]), float(v["phi"]), int(v["npx"]),
                                           int(v["npy"]), float(v["half_width"])) for v in views])
    _check(ctx, _lib.kp_set_views(ctx, len(views), arr))


def make_opts(o=None, **kw) -> kp_opts:
    o = dict(o or {})
    o.update(kw)
    return kp_opts(int(o.get("seed", 0)), int(o.get("transport_fp64", 0)), int(o.get("tally_mode", 0)),
                   float(o.get("rr_wmin", 1e-3)), float(o.get("rr_psurv", 0.1)),
                   int(o.get("max_events", 10000)), int(o.get("trace_packets", 0)),
                   int(o.get("trace_stride", 1)), int(o.get("block_size", 0)),
                   int(o.get("blocks_per_cu", 0)), int(o.get("strict", 0)),
                   int(o.get("scatter_batch", 0)), int(o.get("scatter_wait", 0)),
                   int(o.get("peel_off", 0)))


def _counts(counts):
    a = (C.c_uint64 * len(counts))(*[int(c) for c in counts])
    return a


def kp_run(ctx, counts, opts: kp_opts, stream=None) -> None:
    _check(ctx, _lib.kp_run(ctx, _counts(counts), C.byref(opts), _stream_ptr(stream)))


def kp_run_static(ctx, counts, opts: kp_opts, d_images, stream=None) -> None:
    """d_images: float64 cuda tensor [n_lambda, n_views, 4, npy, npx] (written)."""
    assert d_images.is_cuda and d_images.is_contiguous() and str(d_images.dtype) == "torch.float64"
    _check(ctx, _lib.kp_run_static(ctx, _counts(counts), C.byref(opts), _ptr(d_images), d_images.numel(),
                                   _stream_ptr(stream)))


def kp_transport(ctx, counts, opts: kp_opts, stream=None) -> None:
    _check(ctx, _lib.kp_transport(ctx, _counts(counts), C.byref(opts), _stream_ptr(stream)))


def kp_image(ctx, stream=None) -> None:
    _check(ctx, _lib.kp_image(ctx, _stream_ptr(stream)))


def kp_image_source(ctx, d_S, d_out, stream=None) -> None:
    """d_S: float64 cuda tensor [ncell, n_views, 4]; d_out: [n_views, 4, npy, npx]."""
    for t in (d_S, d_out):
        assert t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float64"
    _check(ctx, _lib.kp_image_source(ctx, _ptr(d_S), _ptr(d_out), _stream_ptr(stream)))


def kp_get_images(ctx, shape) -> np.ndarray:
    out = np.zeros(shape, dtype=np.float64)
    _check(ctx, _lib.kp_get_images(ctx, out.ctypes.data_as(_P), out.size))
    return out


def kp_get_images_device(ctx, d_out, stream=None) -> None:
    _check(ctx, _lib.kp_get_images_device(ctx, _ptr(d_out), d_out.numel(), _stream_ptr(stream)))


def kp_get_peel_images(ctx, shape) -> np.ndarray:
    out = np.zeros(shape, dtype=np.float64)
    _check(ctx, _lib.kp_get_peel_images(ctx, out.ctypes.data_as(_P), out.size))
    return out


def kp_get_tally(ctx, n_lambda, ncell) -> np.ndarray:
    out = np.zeros((n_lambda, ncell, 9), dtype=np.float64)
    _check(ctx, _lib.kp_get_tally(ctx, out.ctypes.data_as(_P), out.size))
    return out


def kp_get_view_tally(ctx, n_lambda, ncell, n_views) -> np.ndarray:
    out = np.zeros((n_lambda, ncell, n_views, 4), dtype=np.float64)
    _check(ctx, _lib.kp_get_view_tally(ctx, out.ctypes.data_as(_P), out.size))
    return out


def kp_get_stats(ctx) -> dict:
    s = kp_stats()
    _check(ctx, _lib.kp_get_stats(ctx, C.byref(s)))
    return {k: getattr(s, k) for k, _ in kp_stats._fields_}


def kp_get_trace(ctx, n) -> np.ndarray:
    out = np.zeros(n, dtype=TRACE_DTYPE)
    _check(ctx, _lib.kp_get_trace(ctx, out.ctypes.data_as(_P), n))
    return out


# --------------------------------------------------------------------------
# convenience: a context object and a one-call workload runner
# --------------------------------------------------------------------------
class Context:
    """Owns a kp_ctx; methods mirror the C entry points."""

    def __init__(self, device: int = 0):
        self.h = kp_create(device)
        self._keep = []

    def close(self):
        if self.h:
            kp_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, cfg, device_arrays: bool = True):
        """Upload a workload dict (see workloads.py): grid, dust, source, views."""
        import torch
        if cfg["grid"].get("mesh") is not None:
            kp_set_mesh(self.h, cfg["grid"], cfg["rho"], cfg.get("bhat"))
        elif device_arrays:
            rho = torch.from_numpy(np.ascontiguousarray(cfg["rho"], np.float32)).cuda()
            bh = None
            if cfg.get("bhat") is not None:
                bh = torch.from_numpy(np.ascontiguousarray(cfg["bhat"], np.float32)).cuda()
            torch.cuda.synchronize()
            self._keep = [rho, bh]
            kp_set_grid_device(self.h, cfg["grid"], rho, bh)
        else:
            kp_set_grid(self.h, cfg["grid"], cfg["rho"], cfg.get("bhat"))
        if cfg.get("emission") is not None:
            kp_set_emission(self.h, cfg["emission"])
        kp_set_dust(self.h, cfg["dust"])
        tabs = [d.get("table") for d in cfg["dust"]]
        if any(t is not None for t in tabs):
            if any(t is None for t in tabs) or len({np.shape(t) for t in tabs}) != 1:
                raise ValueError("tabulated scattering needs one table of the same size per wavelength")
            kp_set_dust_tables(self.h, np.stack(tabs))
        kp_set_source(self.h, cfg["source"])
        kp_set_views(self.h, cfg["views"])
        self.cfg = cfg
        return self

    def opts(self, **kw) -> kp_opts:
        o = dict(self.cfg["opts"])
        o.setdefault("transport_fp64", 1 if self.cfg.get("precision") == "f64" else 0)
        o.update(kw)
        return make_opts(o)

    def run(self, counts=None, stream=None, **kw):
        counts = self.cfg["packets"] if counts is None else counts
        self.last_opts = self.opts(**kw)
        self.last_counts = list(counts)
        kp_run(self.h, counts, self.last_opts, stream)
        return self

    def transport(self, counts=None, stream=None, **kw):
        counts = self.cfg["packets"] if counts is None else counts
        self.last_opts = self.opts(**kw)
        self.last_counts = list(counts)
        kp_transport(self.h, counts, self.last_opts, stream)
        return self

    def image(self, stream=None):
        kp_image(self.h, stream)
        return self

    def images(self) -> np.ndarray:
        v = self.cfg["views"]
        shape = (len(self.last_counts), len(v), 4, v[0]["npy"], v[0]["npx"])
        return kp_get_images(self.h, shape)

    def images_device(self, out=None, stream=None):
        """Images of the last step 2 as a float64 CUDA tensor
        [n_lambda, n_views, 4, npy, npx] (copied on the device)."""
        import torch
        v = self.cfg["views"]
        shape = (len(self.last_counts), len(v), 4, v[0]["npy"], v[0]["npx"])
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device="cuda")
        kp_get_images_device(self.h, out, stream)
        return out

    def peel_images(self) -> np.ndarray:
        """Peel-off images of the last step 1 run with peel_off=1,
        [n_lambda, n_views, 4, npy, npx]."""
        v = self.cfg["views"]
        nl = len(getattr(self, "last_counts", self.cfg["packets"]))
        return kp_get_peel_images(self.h, (nl, len(v), 4, v[0]["npy"], v[0]["npx"]))

    def tally(self) -> np.ndarray:
        return kp_get_tally(self.h, len(self.last_counts), np.asarray(self.cfg["rho"]).size)

    def view_tally(self) -> np.ndarray:
        """Per-view source of the last step 1 with tabulated grains,
        [n_lambda, ncell, n_views, 4]."""
        return kp_get_view_tally(self.h, len(self.last_counts), np.asarray(self.cfg["rho"]).size,
                                 len(self.cfg["views"]))

    def stats(self) -> dict:
        return kp_get_stats(self.h)

    def traces(self) -> np.ndarray:
        n = len(self.last_counts) * int(self.last_opts.trace_packets)
        return kp_get_trace(self.h, n)
