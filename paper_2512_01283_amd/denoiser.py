"""Thin ctypes binding of the denoiser entry points (include/polrad_denoiser.h).

Argument marshalling only: the forward pass, the backward pass, the loss and
Adam run in the library's HIP kernels.  Maps are FP64 ``torch.cuda`` tensors
of shape [batch, 4, height, width]; parameters, gradients and Adam moments
cross the boundary as FP32 NumPy arrays in the flat layout the header
describes.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

from . import polrad as P

_lib = P._lib
HEADER = os.path.join(os.path.dirname(P.HEADER), "polrad_denoiser.h")
WIDTHS = (48, 96, 192)


class kp_dn_timing(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("ms_total", "ms_conv", "ms_wgrad", "ms_other", "conv_flop", "wgrad_flop")]


_Pv = C.c_void_p
_SIGS = {
    "kp_dn_create": ([C.c_int, _Pv, C.c_int32, C.POINTER(_Pv)], C.c_int),
    "kp_dn_create_runs": ([C.c_int, _Pv, C.c_int32, C.c_int32, C.POINTER(_Pv)], C.c_int),
    "kp_dn_destroy": ([_Pv], None),
    "kp_dn_last_error": ([_Pv], C.c_char_p),
    "kp_dn_num_params": ([_Pv, C.POINTER(C.c_size_t)], C.c_int),
    "kp_dn_set_params": ([_Pv, _Pv, C.c_size_t], C.c_int),
    "kp_dn_get_params": ([_Pv, _Pv, C.c_size_t], C.c_int),
    "kp_dn_get_grads": ([_Pv, _Pv, C.c_size_t], C.c_int),
    "kp_dn_get_adam": ([_Pv, _Pv, _Pv, C.c_size_t, C.POINTER(C.c_int32)], C.c_int),
    "kp_dn_set_adam": ([_Pv, _Pv, _Pv, C.c_size_t, C.c_int32], C.c_int),
    "kp_dn_infer": ([_Pv, _Pv, _Pv, C.c_int32, C.c_int32, C.c_int32, _Pv], C.c_int),
    "kp_dn_infer_tta": ([_Pv, _Pv, _Pv, C.c_int32, C.c_int32, C.c_int32, _Pv], C.c_int),
    "kp_dn_backward": ([_Pv, _Pv, _Pv, C.c_int32, C.c_int32, C.c_int32, _Pv,
                        C.POINTER(C.c_double), _Pv], C.c_int),
    "kp_dn_adam_step": ([_Pv, C.c_float, _Pv], C.c_int),
    "kp_dn_train_step": ([_Pv, _Pv, _Pv, C.c_int32, C.c_int32, C.c_int32, _Pv, C.c_float,
                          C.POINTER(C.c_double), _Pv], C.c_int),
    "kp_dn_get_timing": ([_Pv, C.POINTER(kp_dn_timing)], C.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def header_symbols() -> list[str]:
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:kp_status|void|const char \*)\s*(kp_\w+)\s*\(", txt, re.M)))


def _check(h, st):
    if st != P.KP_OK:
        msg = _lib.kp_dn_last_error(h).decode() if h else ""
        raise P.KpError(st, msg)


def _f32(a, n):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def kp_dn_create(device=0, widths=WIDTHS):
    h = _Pv()
    w = np.ascontiguousarray(widths, dtype=np.int32)
    st = _lib.kp_dn_create(int(device), w.ctypes.data, int(w.size), C.byref(h))
    if st != P.KP_OK:
        raise P.KpError(st, f"kp_dn_create(device={device}, widths={tuple(widths)}) failed")
    return h


def kp_dn_create_runs(device=0, widths=WIDTHS, runs=1):
    h = _Pv()
    w = np.ascontiguousarray(widths, dtype=np.int32)
    st = _lib.kp_dn_create_runs(int(device), w.ctypes.data, int(w.size), int(runs), C.byref(h))
    if st != P.KP_OK:
        raise P.KpError(st, f"kp_dn_create_runs(device={device}, widths={tuple(widths)}, runs={runs}) failed")
    return h


def kp_dn_destroy(h):
    _lib.kp_dn_destroy(h)


def kp_dn_last_error(h) -> str:
    return _lib.kp_dn_last_error(h).decode()


def kp_dn_num_params(h) -> int:
    n = C.c_size_t()
    _check(h, _lib.kp_dn_num_params(h, C.byref(n)))
    return int(n.value)


def kp_dn_set_params(h, params):
    a = _f32(params, kp_dn_num_params(h))
    _check(h, _lib.kp_dn_set_params(h, a.ctypes.data, a.size))


def kp_dn_get_params(h) -> np.ndarray:
    a = np.empty(kp_dn_num_params(h), np.float32)
    _check(h, _lib.kp_dn_get_params(h, a.ctypes.data, a.size))
    return a


def kp_dn_get_grads(h) -> np.ndarray:
    a = np.empty(kp_dn_num_params(h), np.float32)
    _check(h, _lib.kp_dn_get_grads(h, a.ctypes.data, a.size))
    return a


def kp_dn_get_adam(h):
    n = kp_dn_num_params(h)
    m, v, t = np.empty(n, np.float32), np.empty(n, np.float32), C.c_int32()
    _check(h, _lib.kp_dn_get_adam(h, m.ctypes.data, v.ctypes.data, n, C.byref(t)))
    return m, v, int(t.value)


def kp_dn_set_adam(h, m, v, step):
    n = kp_dn_num_params(h)
    m, v = _f32(m, n), _f32(v, n)
    _check(h, _lib.kp_dn_set_adam(h, m.ctypes.data, v.ctypes.data, n, int(step)))


def _maps_args(t, channels=4):
    import torch
    if (t.dtype != torch.float64 or not t.is_cuda or t.dim() != 4 or t.shape[1] != channels
            or not t.is_contiguous()):
        raise ValueError(f"maps must be contiguous float64 CUDA tensors [batch, {channels}, height, width]")
    return int(t.shape[0]), int(t.shape[2]), int(t.shape[3])


def _pair_args(low, high, runs):
    b, hh, ww = _maps_args(low, 4 * runs)
    if tuple(high.shape) != (b, 4, hh, ww):
        raise ValueError(f"high must be [batch, 4, height, width] = {(b, 4, hh, ww)}")
    _maps_args(high)
    return b, hh, ww


def _aug_arg(aug, b):
    if aug is None:
        return None, None
    a = np.ascontiguousarray(aug, dtype=np.int32)
    if a.size != b:
        raise ValueError(f"aug needs one code per image ({b}), got {a.size}")
    return a, C.c_void_p(a.ctypes.data)


def kp_dn_infer(h, maps, out, stream=None, runs=1, tta=False):
    b, hh, ww = _maps_args(maps, 4 * runs)
    _maps_args(out)
    if tuple(out.shape) != (b, 4, hh, ww):
        raise ValueError(f"out must be [batch, 4, height, width] = {(b, 4, hh, ww)}")
    f = _lib.kp_dn_infer_tta if tta else _lib.kp_dn_infer
    _check(h, f(h, P._ptr(maps), P._ptr(out), b, hh, ww, P._stream_ptr(stream)))


def kp_dn_backward(h, low, high, aug=None, stream=None, runs=1) -> float:
    b, hh, ww = _pair_args(low, high, runs)
    keep, ap = _aug_arg(aug, b)
    loss = C.c_double()
    _check(h, _lib.kp_dn_backward(h, P._ptr(low), P._ptr(high), b, hh, ww, ap, C.byref(loss),
                                  P._stream_ptr(stream)))
    del keep
    return float(loss.value)


def kp_dn_adam_step(h, lr, stream=None):
    _check(h, _lib.kp_dn_adam_step(h, float(lr), P._stream_ptr(stream)))


def kp_dn_train_step(h, low, high, lr, aug=None, stream=None, runs=1) -> float:
    b, hh, ww = _pair_args(low, high, runs)
    keep, ap = _aug_arg(aug, b)
    loss = C.c_double()
    _check(h, _lib.kp_dn_train_step(h, P._ptr(low), P._ptr(high), b, hh, ww, ap, float(lr),
                                    C.byref(loss), P._stream_ptr(stream)))
    del keep
    return float(loss.value)


def kp_dn_get_timing(h) -> dict:
    t = kp_dn_timing()
    _check(h, _lib.kp_dn_get_timing(h, C.byref(t)))
    return {k: getattr(t, k) for k, _ in kp_dn_timing._fields_}


# --------------------------------------------------------------------------
# convenience object
# --------------------------------------------------------------------------
class Denoiser:
    """Owns one kp_dn handle.  Parameters are FP32 master weights on the
    device; ``params``/``grads`` return host copies in the flat layout."""

    def __init__(self, device=0, widths=WIDTHS, params=None, runs=1):
        self.widths = tuple(int(c) for c in widths)
        self.runs = int(runs)
        self.h = kp_dn_create_runs(device, self.widths, self.runs)
        self.n = kp_dn_num_params(self.h)
        if params is not None:
            self.set_params(params)

    def close(self):
        if self.h:
            kp_dn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        kp_dn_set_params(self.h, p)

    def params(self):
        return kp_dn_get_params(self.h)

    def grads(self):
        return kp_dn_get_grads(self.h)

    def adam_state(self):
        return kp_dn_get_adam(self.h)

    def set_adam_state(self, m, v, step):
        kp_dn_set_adam(self.h, m, v, step)

    def infer(self, maps, out=None, stream=None, tta=False):
        """Denoised maps; tta=True averages over the dihedral transforms."""
        import torch
        if out is None:
            out = torch.empty((maps.shape[0], 4) + tuple(maps.shape[2:]), dtype=maps.dtype, device=maps.device)
        kp_dn_infer(self.h, maps, out, stream, self.runs, tta)
        return out

    def backward(self, low, high, aug=None, stream=None):
        return kp_dn_backward(self.h, low, high, aug, stream, self.runs)

    def adam_step(self, lr, stream=None):
        kp_dn_adam_step(self.h, lr, stream)

    def train_step(self, low, high, lr, aug=None, stream=None):
        return kp_dn_train_step(self.h, low, high, lr, aug, stream, self.runs)

    def timing(self):
        return kp_dn_get_timing(self.h)
