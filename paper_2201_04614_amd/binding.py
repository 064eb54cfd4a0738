"""ctypes binding of libdq (include/dq.h): argument marshalling only.

Every step of the codec runs in the HIP kernels of libdq.so; torch provides
device memory and the current stream. Importing this module does not touch
the GPU; the library is loaded on first use and a missing build raises.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdq.so")

DQ_OK, DQ_EINVAL, DQ_ERANGE, DQ_ECAPACITY, DQ_ENOTSUP, DQ_EDEVICE, DQ_ECORRUPT = 0, -1, -2, -3, -4, -5, -6
DQ_ENOSCRATCH = -7
DQ_SCRATCH_BYTES = 64 << 20  # the fixed workspace of dq_compress_noalloc (include/dq.h)
EB_MODES = {"abs": 0, "rel": 1}
PAD_MODES = {"zero": 0, "block_mean": 1, "edge_mean": 2, "global_mean": 3,
             "block_min": 4, "block_max": 5, "global_min": 6, "global_max": 7, "given": 8}

# every function include/dq.h declares
EXPORTS = ["dq_validate", "dq_num_blocks", "dq_pad_count", "dq_compress_workspace",
           "dq_decompress_workspace", "dq_compress", "dq_compress_noalloc", "dq_decompress", "dq_decompress_dev",
           "dq_result_sync",
           "dq_event_create", "dq_event_destroy", "dq_event_elapsed_ms", "dq_strerror"]


class DQError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})" if what else f"{strerror(status)} ({status})")


class Params(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("eb_mode", C.c_int32), ("shape", C.c_int64 * 3),
                ("eb", C.c_double), ("block", C.c_int32), ("pad_mode", C.c_int32),
                ("radius", C.c_int32), ("vec", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_uint32), ("n_out", C.c_uint64),
                ("eb_abs", C.c_double)]


class Hooks(C.Structure):
    _fields_ = [("ev_before", C.c_void_p), ("ev_after", C.c_void_p)]


_lib = None


def lib():
    """Load libdq.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2201_04614_amd/csrc/build.py`")
        # torch first: its HIP runtime (soname libamdhip64.so.7, which
        # libtorch_hip requests under another file name) must be the one in
        # the process when libdq.so resolves that soname; loaded the other
        # way round the process holds two HIP runtimes and libdq cannot use
        # torch's streams
        _torch()
        L = C.CDLL(LIB_PATH)
        P, vp, u64, pu64 = C.POINTER(Params), C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64)
        sig = {
            "dq_validate": ([P], C.c_int),
            "dq_num_blocks": ([P, pu64], C.c_int),
            "dq_pad_count": ([P, pu64], C.c_int),
            "dq_compress_workspace": ([P, u64, pu64], C.c_int),
            "dq_decompress_workspace": ([P, pu64], C.c_int),
            "dq_compress": ([P, vp, vp, vp, vp, u64, vp, vp, vp, u64, vp, C.POINTER(Hooks)], C.c_int),
            "dq_compress_noalloc": ([P, vp, vp, vp, vp, u64, vp, vp, vp], C.c_int),
            "dq_decompress": ([P, C.c_double, vp, vp, vp, u64, vp, vp, vp, vp, u64, vp,
                               C.POINTER(Hooks)], C.c_int),
            "dq_decompress_dev": ([P, vp, u64, vp, vp, vp, vp, vp, vp, vp, u64, vp, C.POINTER(Hooks)], C.c_int),
            "dq_result_sync": ([vp, C.POINTER(Result), vp], C.c_int),
            "dq_event_create": ([C.POINTER(C.c_void_p)], C.c_int),
            "dq_event_destroy": ([vp], C.c_int),
            "dq_event_elapsed_ms": ([vp, vp, C.POINTER(C.c_float)], C.c_int),
            "dq_strerror": ([C.c_int], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def strerror(status):
    try:
        return lib().dq_strerror(int(status)).decode()
    except RuntimeError:
        return f"status {status}"


def make_params(shape, eb, eb_mode="abs", block=16, pad="zero", radius=512, vec=0):
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
    p.vec = int(vec)
    return p


def validate(p):
    return lib().dq_validate(C.byref(p))


def num_blocks(p):
    n = C.c_uint64(0)
    st = lib().dq_num_blocks(C.byref(p), C.byref(n))
    if st != DQ_OK:
        raise DQError(st, "dq_num_blocks")
    return n.value


def pad_count(p):
    n = C.c_uint64(0)
    st = lib().dq_pad_count(C.byref(p), C.byref(n))
    if st != DQ_OK:
        raise DQError(st, "dq_pad_count")
    return n.value


def compress_workspace(p, out_cap):
    n = C.c_uint64(0)
    st = lib().dq_compress_workspace(C.byref(p), int(out_cap), C.byref(n))
    if st != DQ_OK:
        raise DQError(st, "dq_compress_workspace")
    return n.value


def decompress_workspace(p):
    n = C.c_uint64(0)
    st = lib().dq_decompress_workspace(C.byref(p), C.byref(n))
    if st != DQ_OK:
        raise DQError(st, "dq_decompress_workspace")
    return n.value


# ---------------------------------------------------------------- torch side

def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _aligned_bytes(n, device, align=256):
    """Device byte buffer of n bytes whose start is `align`-aligned."""
    torch = _torch()
    raw = torch.empty(int(n) + align, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % align
    return raw[off:off + int(n)] if n else raw[:0]


class Hook:
    """A pair of HIP events recorded around the main kernel of a call."""

    def __init__(self):
        self.before = C.c_void_p()
        self.after = C.c_void_p()
        for ev in (self.before, self.after):
            st = lib().dq_event_create(C.byref(ev))
            if st != DQ_OK:
                raise DQError(st, "dq_event_create")
        self.struct = Hooks(self.before, self.after)

    def elapsed_ms(self):
        ms = C.c_float(0.0)
        st = lib().dq_event_elapsed_ms(self.before, self.after, C.byref(ms))
        if st != DQ_OK:
            raise DQError(st, "dq_event_elapsed_ms")
        return ms.value

    def close(self):
        for ev in (self.before, self.after):
            if ev.value:
                lib().dq_event_destroy(ev)
                ev.value = None


@dataclass
class DQStream:
    """Compressed field: codes, block-major outliers, pads, bound and parameters."""
    shape: tuple
    block: int
    pad: str
    radius: int
    eb_abs: float
    n_out: int
    codes: object      # torch.int16 tensor holding uint16 codes, field shape
    out_idx: object    # torch.int32 tensor holding uint32 indices, n_out entries
    out_val: object    # torch.int32, n_out entries
    pads: object       # torch.int32, pad_count entries
    coded: object = None  # Huffman-coded codes (HuffCoded) when codes is None

    def params(self):
        return make_params(self.shape, self.eb_abs, "abs", self.block, self.pad, self.radius)

    def stream_bytes(self):
        """Bytes of the stream: codes (raw or coded), outliers, pads, code table."""
        b = 8 * self.n_out + 4 * self.pads.numel() + 64
        if self.codes is not None:
            return b + 2 * self.codes.numel()
        c = self.coded
        return b + 4 * c.words.numel() + 8 * c.chunk_off.numel() + 2 * c.sub_off.numel() + c.lengths.numel()


@dataclass
class HuffCoded:
    """Canonical Huffman coding of a stream's codes (see huffman.py)."""
    n_symbols: int
    lengths: object    # torch.uint8 [n_symbols]
    chunk_off: object  # torch.int64 [n_chunks + 1]
    sub_off: object    # torch.int16 [n_chunks, 3]
    words: object      # torch.int32 [words]


def result_sync(res_dev, stream=None):
    r = Result()
    st = lib().dq_result_sync(_ptr(res_dev), C.byref(r), _stream_handle(stream))
    if st != DQ_OK:
        raise DQError(st, "dq_result_sync")
    return r


class Codec:
    """Preallocated device buffers for repeated compress/decompress calls of one
    field configuration (no allocation per call)."""

    def __init__(self, shape, eb, eb_mode="abs", block=16, pad="zero", radius=512,
                 out_cap=None, device="cuda", vec=0):
        torch = _torch()
        self.shape = tuple(int(s) for s in shape)
        self.n = int(np.prod(self.shape))
        self.block, self.pad, self.radius = int(block), pad, int(radius)
        self.p = make_params(self.shape, eb, eb_mode, block, pad, radius, vec)
        st = validate(self.p)
        if st != DQ_OK:
            raise DQError(st, "dq_validate")
        self.device = torch.device(device)
        self.out_cap = int(out_cap) if out_cap is not None else max(1024, self.n // 16)
        self.codes = torch.empty(self.shape, dtype=torch.int16, device=self.device)
        self.out_idx = torch.empty(max(self.out_cap, 1), dtype=torch.int32, device=self.device)
        self.out_val = torch.empty(max(self.out_cap, 1), dtype=torch.int32, device=self.device)
        self.pads = torch.empty(max(pad_count(self.p), 1), dtype=torch.int32, device=self.device)
        self.res = torch.zeros(3, dtype=torch.int64, device=self.device)
        self.dres = torch.zeros(3, dtype=torch.int64, device=self.device)
        self.ws_c = _aligned_bytes(compress_workspace(self.p, self.out_cap), self.device)
        self.ws_d = _aligned_bytes(decompress_workspace(make_params(
            self.shape, 1.0, "abs", block, pad, radius)), self.device)
        self.x_hat = torch.empty(self.shape, dtype=torch.float32, device=self.device)

    def compress_async(self, x, stream=None, hooks=None):
        """Enqueue compression of x (contiguous fp32 CUDA tensor of this shape).
        With the "given" padding mode, self.pads holds the per-block values
        (an input) when this is called."""
        assert x.is_cuda and x.dtype == _torch().float32 and x.is_contiguous()
        assert tuple(x.shape) == self.shape
        st = lib().dq_compress(C.byref(self.p), _ptr(x), _ptr(self.codes), _ptr(self.out_idx),
                               _ptr(self.out_val), self.out_cap, _ptr(self.pads), _ptr(self.res),
                               _ptr(self.ws_c), self.ws_c.numel(), _stream_handle(stream),
                               C.byref(hooks.struct) if hooks else None)
        if st != DQ_OK:
            raise DQError(st, "dq_compress")

    def compress_noalloc_async(self, x, stream=None):
        """As compress_async, through dq_compress_noalloc: the library's fixed
        scratch array replaces this codec's workspace."""
        assert x.is_cuda and x.dtype == _torch().float32 and x.is_contiguous()
        assert tuple(x.shape) == self.shape
        st = lib().dq_compress_noalloc(C.byref(self.p), _ptr(x), _ptr(self.codes), _ptr(self.out_idx),
                                       _ptr(self.out_val), self.out_cap, _ptr(self.pads), _ptr(self.res),
                                       _stream_handle(stream))
        if st != DQ_OK:
            raise DQError(st, "dq_compress_noalloc")

    def result(self, stream=None):
        return result_sync(self.res, stream)

    def decompress_async(self, eb_abs, n_out, out=None, codes=None, out_idx=None, out_val=None,
                         pads=None, stream=None, hooks=None):
        """Enqueue decompression of this codec's buffers (or the ones given)."""
        codes = self.codes if codes is None else codes
        out_idx = self.out_idx if out_idx is None else out_idx
        out_val = self.out_val if out_val is None else out_val
        # the kernels read n_out entries of both lists: never more than they hold
        if int(n_out) > min(out_idx.numel(), out_val.numel()) or (out_idx is self.out_idx and int(n_out) > self.out_cap):
            raise DQError(DQ_EINVAL, f"dq_decompress: n_out {int(n_out)} exceeds the outlier buffers")
        pads = self.pads if pads is None else pads
        out = self.x_hat if out is None else out
        st = lib().dq_decompress(C.byref(self.p), float(eb_abs), _ptr(codes), _ptr(out_idx),
                                 _ptr(out_val), int(n_out), _ptr(pads), _ptr(out), _ptr(self.dres),
                                 _ptr(self.ws_d), self.ws_d.numel(), _stream_handle(stream),
                                 C.byref(hooks.struct) if hooks else None)
        if st != DQ_OK:
            raise DQError(st, "dq_decompress")
        return out

    def decompress_dev_async(self, out=None, stream=None, hooks=None):
        """Enqueue decompression of this codec's last compression, taking the
        outlier count and bound from its device result (no host sync)."""
        out = self.x_hat if out is None else out
        st = lib().dq_decompress_dev(C.byref(self.p), _ptr(self.res), self.out_cap, _ptr(self.codes),
                                     _ptr(self.out_idx), _ptr(self.out_val), _ptr(self.pads), _ptr(out),
                                     _ptr(self.dres), _ptr(self.ws_d), self.ws_d.numel(), _stream_handle(stream),
                                     C.byref(hooks.struct) if hooks else None)
        if st != DQ_OK:
            raise DQError(st, "dq_decompress_dev")
        return out

    def decompress_result(self, stream=None):
        return result_sync(self.dres, stream)


def compress(x, eb, eb_mode="abs", block=16, pad="zero", radius=512, out_cap=None, entropy=False):
    """Compress a contiguous fp32 CUDA tensor; returns a DQStream.

    Raises DQError on a host-side error or a device status other than OK. When
    the outlier capacity is exceeded the call is repeated once with the exact
    count. entropy=True also Huffman-codes the codes (the stream then holds
    the coded form instead of the raw codes)."""
    torch = _torch()
    x = x.contiguous()
    codec = Codec(tuple(x.shape), eb, eb_mode, block, pad, radius, out_cap, x.device)
    codec.compress_async(x)
    r = codec.result()
    if r.status == DQ_ECAPACITY and out_cap is None:
        codec = Codec(tuple(x.shape), eb, eb_mode, block, pad, radius, int(r.n_out), x.device)
        codec.compress_async(x)
        r = codec.result()
    if r.status != DQ_OK:
        raise DQError(r.status, "compress")
    n = int(r.n_out)
    npads = pad_count(codec.p)
    s = DQStream(codec.shape, codec.block, codec.pad, codec.radius, float(r.eb_abs), n,
                 codec.codes, codec.out_idx[:n], codec.out_val[:n], codec.pads[:npads])
    if entropy:
        from . import huffman as HF
        flat = codec.codes.reshape(-1)
        cb = HF.codebook(flat, 2 * codec.radius)
        bs = HF.encode(flat, cb)
        st = int(cb.status.item()) or int(bs.status.item())
        if st != DQ_OK:
            raise DQError(st, "huffman encode")
        total = int(bs.chunk_off[-1].item())
        s.coded = HuffCoded(2 * codec.radius, cb.lengths, bs.chunk_off, bs.sub_off, bs.words[:total].clone())
        s.codes = None
    return s


def decompress(s: DQStream, out=None):
    """Decompress a DQStream into an fp32 CUDA tensor of the field's shape."""
    torch = _torch()
    p = s.params()
    codes = s.codes
    if codes is None:  # Huffman-coded stream: decode the codes first
        from . import huffman as HF
        c = s.coded
        n = int(np.prod(s.shape))
        bs = HF.Bitstream(n, c.chunk_off, c.sub_off, c.words, None)
        flat, hst = HF.decode(bs, HF.Codebook(c.n_symbols, None, c.lengths, None, None))
        if int(hst.item()) != DQ_OK:
            raise DQError(int(hst.item()), "huffman decode")
        codes = flat.reshape(s.shape)
    dev = codes.device
    out = torch.empty(s.shape, dtype=torch.float32, device=dev) if out is None else out
    res = torch.zeros(3, dtype=torch.int64, device=dev)
    ws = _aligned_bytes(decompress_workspace(p), dev)
    pads = s.pads if s.pads.numel() else None
    st = lib().dq_decompress(C.byref(p), float(s.eb_abs), _ptr(codes), _ptr(s.out_idx),
                             _ptr(s.out_val), int(s.n_out), _ptr(pads), _ptr(out), _ptr(res),
                             _ptr(ws), ws.numel(), _stream_handle(), None)
    if st != DQ_OK:
        raise DQError(st, "dq_decompress")
    r = result_sync(res)
    if r.status != DQ_OK:
        raise DQError(r.status, "decompress")
    return out
