"""Streams with one block edge per 16^d super-block (binding of
include/dq_mixed.h; argument marshalling only).

    edges = torch.full((n_super,), 8, dtype=torch.uint8, device="cuda")
    s = compress(x, eb_abs, radius, edges, pads)     # pads: int32, stream order
    x_hat = decompress(s)

The edges and pads come from the per-block padding / block-size selector
(selector.mixed_exhaustive / selector.mixed_learned).
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

from . import binding as dq

EXPORTS = ["dq_mixed_num_super", "dq_mixed_pad_offsets", "dq_mixed_workspace", "dq_mixed_compress",
           "dq_mixed_decompress", "dq_super_label", "dq_super_vote", "dq_mixed_gather_pads"]
EDGES = (4, 8, 16)

_ready = False


def lib():
    global _ready
    L = dq.lib()
    if not _ready:
        P, vp, u64 = C.POINTER(dq.Params), C.c_void_p, C.c_uint64
        sig = {
            "dq_mixed_num_super": [P, C.POINTER(u64)],
            "dq_mixed_pad_offsets": [P, vp, vp, vp, vp],
            "dq_mixed_workspace": [P, C.POINTER(u64)],
            "dq_mixed_compress": [P, vp, vp, vp, vp, vp, vp, vp, u64, vp, vp, u64, vp],
            "dq_mixed_decompress": [P, C.c_double, vp, vp, vp, vp, vp, vp, u64, vp, vp, vp, u64, vp],
            "dq_super_label": [P, vp, vp, vp, vp],
            "dq_super_vote": [P, C.c_int32, vp, vp, vp, vp],
            "dq_mixed_gather_pads": [P, vp, vp, vp, vp, vp, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        _ready = True
    return L


def _torch():
    import torch
    return torch


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def _s(stream=None):
    return dq._stream_handle(stream)


def _check(st, what):
    if st != dq.DQ_OK:
        raise dq.DQError(st, what)


def _params(shape, eb=1.0, radius=512):
    return dq.make_params(shape, eb, "abs", 16, "given", radius)


def num_super(shape):
    n = C.c_uint64(0)
    _check(lib().dq_mixed_num_super(C.byref(_params(shape)), C.byref(n)), "dq_mixed_num_super")
    return int(n.value)


def pad_offsets(shape, edges, stream=None):
    """Exclusive prefix of the blocks per super-block (n_super + 1 int32)."""
    torch = _torch()
    off = torch.empty(num_super(shape) + 1, dtype=torch.int32, device=edges.device)
    st = torch.zeros(1, dtype=torch.int32, device=edges.device)
    _check(lib().dq_mixed_pad_offsets(C.byref(_params(shape)), _p(edges), _p(off), _p(st), _s(stream)),
           "dq_mixed_pad_offsets")
    return off, st


def _ws(shape, device):
    n = C.c_uint64(0)
    _check(lib().dq_mixed_workspace(C.byref(_params(shape)), C.byref(n)), "dq_mixed_workspace")
    return dq._aligned_bytes(int(n.value), device)


@dataclass
class MixedStream:
    shape: tuple
    radius: int
    eb_abs: float
    n_out: int
    status: int
    edges: object    # uint8 [n_super]
    pad_off: object  # int32 [n_super + 1]
    pads: object     # int32 [n_pads], stream order
    codes: object    # int16 (uint16 codes), field shape
    out_idx: object  # int32 (uint32 indices) [n_out]
    out_val: object  # int32 [n_out]


def compress(x, eb_abs, radius, edges, pads, pad_off=None, out_cap=None, stream=None):
    """Mixed-edge compression of x (contiguous fp32 CUDA tensor) with the
    absolute bound eb_abs; edges: uint8 per super-block, pads: int32 per
    block in stream order."""
    torch = _torch()
    shape = tuple(x.shape)
    dev = x.device
    if pad_off is None:
        pad_off, _ = pad_offsets(shape, edges, stream)
    cap = int(out_cap) if out_cap is not None else x.numel()
    codes = torch.empty(shape, dtype=torch.int16, device=dev)
    idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    res = torch.zeros(3, dtype=torch.int64, device=dev)
    ws = _ws(shape, dev)
    p = _params(shape, eb_abs, radius)
    _check(lib().dq_mixed_compress(C.byref(p), _p(x), _p(edges), _p(pad_off), _p(pads), _p(codes), _p(idx),
                                   _p(val), cap, _p(res), _p(ws), ws.numel(), _s(stream)), "dq_mixed_compress")
    r = dq.result_sync(res, stream)
    n = int(r.n_out)
    k = min(n, cap)
    return MixedStream(shape, int(radius), float(r.eb_abs), n, int(r.status), edges, pad_off, pads, codes,
                       idx[:k], val[:k])


def decompress(s, stream=None):
    """x_hat of a mixed stream (raises on a device error status)."""
    torch = _torch()
    dev = s.codes.device
    out = torch.empty(s.shape, dtype=torch.float32, device=dev)
    res = torch.zeros(3, dtype=torch.int64, device=dev)
    ws = _ws(s.shape, dev)
    p = _params(s.shape, s.eb_abs, s.radius)
    _check(lib().dq_mixed_decompress(C.byref(p), float(s.eb_abs), _p(s.edges), _p(s.pad_off), _p(s.pads),
                                     _p(s.codes), _p(s.out_idx), _p(s.out_val), int(s.n_out), _p(out), _p(res),
                                     _p(ws), ws.numel(), _s(stream)), "dq_mixed_decompress")
    r = dq.result_sync(res, stream)
    if r.status != dq.DQ_OK:
        raise dq.DQError(r.status, "dq_mixed_decompress (device)")
    return out


def super_label(shape, cost, stream=None):
    """Edges (uint8) and labels (int32) from the 3 x n_super side costs."""
    torch = _torch()
    n = num_super(shape)
    edges = torch.empty(n, dtype=torch.uint8, device=cost.device)
    label = torch.empty(n, dtype=torch.int32, device=cost.device)
    _check(lib().dq_super_label(C.byref(_params(shape)), _p(cost.contiguous()), _p(edges), _p(label), _s(stream)),
           "dq_super_label")
    return edges, label


def super_vote(shape, base, logits, stream=None):
    """Edges (uint8) and labels from the network's block-size logits at edge base."""
    torch = _torch()
    n = num_super(shape)
    edges = torch.empty(n, dtype=torch.uint8, device=logits.device)
    label = torch.empty(n, dtype=torch.int32, device=logits.device)
    _check(lib().dq_super_vote(C.byref(_params(shape)), int(base), _p(logits.contiguous()), _p(edges), _p(label),
                               _s(stream)), "dq_super_vote")
    return edges, label


def gather_pads(shape, edges, pad_off, pads_by_edge, n_pads, stream=None):
    """Stream-order pads from per-edge pads (dict edge -> int32 tensor)."""
    torch = _torch()
    out = torch.empty(max(int(n_pads), 1), dtype=torch.int32, device=edges.device)
    _check(lib().dq_mixed_gather_pads(C.byref(_params(shape)), _p(edges), _p(pad_off), _p(pads_by_edge[4]),
                                      _p(pads_by_edge[8]), _p(pads_by_edge[16]), _p(out), _s(stream)),
           "dq_mixed_gather_pads")
    return out[:int(n_pads)]
