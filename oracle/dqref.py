"""ctypes binding of the C oracle (TEST INFRASTRUCTURE ONLY).

Host numpy arrays in, host numpy arrays out. Builds oracle/libdqref.so with
gcc if it is missing.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

OK, EINVAL, ERANGE, ECAPACITY, ECORRUPT = 0, -1, -2, -3, -6
EB_MODES = {"abs": 0, "rel": 1}
PAD_MODES = {"zero": 0, "block_mean": 1, "edge_mean": 2, "global_mean": 3,
             "block_min": 4, "block_max": 5, "global_min": 6, "global_max": 7, "given": 8}


class Params(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("eb_mode", C.c_int32),
                ("shape", C.c_int64 * 3), ("eb", C.c_double),
                ("block", C.c_int32), ("pad_mode", C.c_int32),
                ("radius", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.POINTER(Params)
        vp = C.c_void_p
        L.dqref_validate.argtypes = [P]
        L.dqref_validate.restype = C.c_int
        L.dqref_pad_count.argtypes = [P]
        L.dqref_pad_count.restype = C.c_int64
        L.dqref_num_blocks.argtypes = [P]
        L.dqref_num_blocks.restype = C.c_int64
        L.dqref_round_mean.argtypes = [C.c_int64, C.c_int64]
        L.dqref_round_mean.restype = C.c_int64
        L.dqref_resolve_eb.argtypes = [P, vp, C.POINTER(C.c_double)]
        L.dqref_resolve_eb.restype = C.c_int
        L.dqref_prequantize.argtypes = [P, vp, C.c_double, vp]
        L.dqref_prequantize.restype = C.c_int
        L.dqref_pad_values.argtypes = [P, vp, vp]
        L.dqref_pad_values.restype = C.c_int
        L.dqref_residuals.argtypes = [P, vp, vp, vp, C.c_int]
        L.dqref_residuals.restype = C.c_int
        L.dqref_reconstruct.argtypes = [P, vp, vp, vp, C.c_int]
        L.dqref_reconstruct.restype = C.c_int
        L.dqref_compress.argtypes = [P, vp, vp, vp, vp, C.c_uint64,
                                     C.POINTER(C.c_uint64), vp,
                                     C.POINTER(C.c_double), C.c_int]
        L.dqref_compress.restype = C.c_int
        L.dqref_decompress.argtypes = [P, C.c_double, vp, vp, vp, C.c_uint64,
                                       vp, vp, C.c_int]
        L.dqref_decompress.restype = C.c_int
        _lib = L
    return _lib


def params(shape, eb, eb_mode="abs", block=16, pad="zero", radius=512):
    shape = tuple(int(s) for s in shape)
    p = Params()
    p.ndim = len(shape)
    p.eb_mode = EB_MODES[eb_mode] if isinstance(eb_mode, str) else int(eb_mode)
    for a in range(3):
        p.shape[a] = shape[a] if a < len(shape) else 0
    p.eb = float(eb)
    p.block = int(block)
    p.pad_mode = PAD_MODES[pad] if isinstance(pad, str) else int(pad)
    p.radius = int(radius)
    return p


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def _f32(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    return x


def validate(p):
    return lib().dqref_validate(C.byref(p))


def pad_count(p):
    return lib().dqref_pad_count(C.byref(p))


def num_blocks(p):
    return lib().dqref_num_blocks(C.byref(p))


def round_mean(S, n):
    return lib().dqref_round_mean(int(S), int(n))


def resolve_eb(p, x):
    x = _f32(x)
    eb = C.c_double(0.0)
    st = lib().dqref_resolve_eb(C.byref(p), _ptr(x), C.byref(eb))
    return st, eb.value


def prequantize(p, x, eb_abs):
    x = _f32(x)
    q = np.zeros(x.shape, dtype=np.int32)
    st = lib().dqref_prequantize(C.byref(p), _ptr(x), float(eb_abs), _ptr(q))
    return st, q


def pad_values(p, q):
    q = np.ascontiguousarray(q, dtype=np.int32)
    pads = np.zeros(max(pad_count(p), 0), dtype=np.int32)
    st = lib().dqref_pad_values(C.byref(p), _ptr(q), _ptr(pads))
    return st, pads


def residuals(p, q, pads, nthreads=1):
    q = np.ascontiguousarray(q, dtype=np.int32)
    pads = np.ascontiguousarray(pads, dtype=np.int32)
    d = np.zeros(q.shape, dtype=np.int32)
    st = lib().dqref_residuals(C.byref(p), _ptr(q), _ptr(pads), _ptr(d), int(nthreads))
    return st, d


def reconstruct(p, delta, pads, nthreads=1):
    delta = np.ascontiguousarray(delta, dtype=np.int32)
    pads = np.ascontiguousarray(pads, dtype=np.int32)
    q = np.zeros(delta.shape, dtype=np.int32)
    st = lib().dqref_reconstruct(C.byref(p), _ptr(delta), _ptr(pads), _ptr(q), int(nthreads))
    return st, q


@dataclass
class Compressed:
    status: int
    codes: np.ndarray
    out_idx: np.ndarray
    out_val: np.ndarray
    n_out: int
    pads: np.ndarray
    eb_abs: float


def compress(p, x, out_cap=None, nthreads=1, pads=None):
    """pads: the per-block values of the "given" padding mode (an input)."""
    x = _f32(x)
    n = x.size
    if out_cap is None:
        out_cap = n
    codes = np.zeros(x.shape, dtype=np.uint16)
    idx = np.zeros(max(int(out_cap), 1), dtype=np.uint32)
    val = np.zeros(max(int(out_cap), 1), dtype=np.int32)
    npad = max(pad_count(p), 0)
    if pads is None:
        pads = np.zeros(npad, dtype=np.int32)
    else:
        pads = np.array(pads, dtype=np.int32).reshape(-1)
        assert pads.size == npad
    n_out = C.c_uint64(0)
    eb = C.c_double(0.0)
    st = lib().dqref_compress(C.byref(p), _ptr(x), _ptr(codes), _ptr(idx), _ptr(val),
                              int(out_cap), C.byref(n_out), _ptr(pads), C.byref(eb),
                              int(nthreads))
    k = min(int(n_out.value), int(out_cap))
    return Compressed(st, codes, idx[:k].copy(), val[:k].copy(), int(n_out.value),
                      pads, eb.value)


def decompress(p, eb_abs, codes, out_idx, out_val, pads, nthreads=1):
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    out_idx = np.ascontiguousarray(out_idx, dtype=np.uint32)
    out_val = np.ascontiguousarray(out_val, dtype=np.int32)
    pads = np.ascontiguousarray(pads, dtype=np.int32)
    xh = np.zeros(codes.shape, dtype=np.float32)
    st = lib().dqref_decompress(C.byref(p), float(eb_abs), _ptr(codes), _ptr(out_idx),
                                _ptr(out_val), int(out_idx.size), _ptr(pads), _ptr(xh),
                                int(nthreads))
    return st, xh
