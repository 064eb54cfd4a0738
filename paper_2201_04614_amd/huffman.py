"""Canonical Huffman coding of quantisation codes on the GPU (binding of
include/dq_huffman.h; argument marshalling only).

    cb = codebook(codes, n_symbols)          # histogram, lengths, codewords (device)
    bs = encode(codes, cb)                   # chunk offsets + words
    back = decode(bs, cb)                    # uint16 codes again
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

from . import binding as dq

CHUNK = 1024
MAX_PRESENT = 2048

# every function include/dq_huffman.h declares
EXPORTS = ["dq_huff_workspace", "dq_huff_max_words", "dq_huff_codebook", "dq_huff_encode", "dq_huff_decode"]

_ready = False


def lib():
    global _ready
    L = dq.lib()
    if not _ready:
        vp, u64, u32, pu64 = C.c_void_p, C.c_uint64, C.c_uint32, C.POINTER(C.c_uint64)
        sig = {
            "dq_huff_workspace": ([u64, pu64], C.c_int),
            "dq_huff_max_words": ([u64, pu64], C.c_int),
            "dq_huff_codebook": ([vp, u64, u32, vp, vp, vp, vp, vp, u64, vp], C.c_int),
            "dq_huff_encode": ([vp, u64, u32, vp, vp, vp, vp, vp, u64, vp, vp, u64, vp], C.c_int),
            "dq_huff_decode": ([vp, u64, vp, vp, u64, u32, vp, vp, vp, vp, u64, vp], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _ready = True
    return L


def _p(t):
    return C.c_void_p(t.data_ptr())


def _s(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check(st, what):
    if st != dq.DQ_OK:
        raise dq.DQError(st, what)


def _ws(n, device):
    import torch
    b = C.c_uint64(0)
    _check(lib().dq_huff_workspace(n, C.byref(b)), "dq_huff_workspace")
    return torch.empty(int(b.value) + 256, dtype=torch.uint8, device=device)


def _aligned(t):
    off = (-t.data_ptr()) % 256
    return t[off:], t.numel() - off


@dataclass
class Codebook:
    n_symbols: int
    hist: object       # int32 [n_symbols] (uint32 counts)
    lengths: object    # uint8 [n_symbols]
    codewords: object  # int32 [n_symbols] (uint32 codewords)
    status: object     # int32 [1]


@dataclass
class Bitstream:
    n: int
    chunk_off: object  # int64 [n_chunks + 1] (uint64 word offsets)
    sub_off: object    # int16 [n_chunks, 3] (uint16 bit offsets of codes 256, 512, 768 in each chunk)
    words: object      # int32 [capacity] (uint32 words)
    status: object


def codebook(codes, n_symbols, stream=None):
    import torch
    n = codes.numel()
    dev = codes.device
    cb = Codebook(int(n_symbols), torch.empty(n_symbols, dtype=torch.int32, device=dev),
                  torch.empty(n_symbols, dtype=torch.uint8, device=dev),
                  torch.empty(n_symbols, dtype=torch.int32, device=dev), torch.zeros(1, dtype=torch.int32, device=dev))
    _check(lib().dq_huff_codebook(_p(codes), n, int(n_symbols), _p(cb.hist), _p(cb.lengths), _p(cb.codewords),
                                  _p(cb.status), None, 0, _s(stream)), "dq_huff_codebook")
    return cb


def encode(codes, cb, ws=None, words_cap=None, stream=None):
    import torch
    n = codes.numel()
    dev = codes.device
    if words_cap is None:
        w = C.c_uint64(0)
        _check(lib().dq_huff_max_words(n, C.byref(w)), "dq_huff_max_words")
        words_cap = int(w.value)
    nch = (n + CHUNK - 1) // CHUNK
    bs = Bitstream(n, torch.empty(nch + 1, dtype=torch.int64, device=dev),
                   torch.empty((nch, 3), dtype=torch.int16, device=dev),
                   torch.empty(max(1, words_cap), dtype=torch.int32, device=dev),
                   torch.zeros(1, dtype=torch.int32, device=dev))
    wsb, nb = _aligned(ws if ws is not None else _ws(n, dev))
    _check(lib().dq_huff_encode(_p(codes), n, cb.n_symbols, _p(cb.lengths), _p(cb.codewords), _p(bs.chunk_off),
                                _p(bs.sub_off), _p(bs.words), int(words_cap), _p(bs.status), _p(wsb), nb,
                                _s(stream)), "dq_huff_encode")
    return bs


def decode(bs, cb, out=None, ws=None, n_words=None, stream=None):
    import torch
    dev = bs.words.device
    out = torch.empty(bs.n, dtype=torch.int16, device=dev) if out is None else out
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb, nb = _aligned(ws if ws is not None else _ws(bs.n, dev))
    nw = bs.words.numel() if n_words is None else int(n_words)
    _check(lib().dq_huff_decode(_p(bs.words), nw, _p(bs.chunk_off), _p(bs.sub_off), bs.n, cb.n_symbols,
                                _p(cb.lengths), _p(out), _p(status), _p(wsb), nb, _s(stream)), "dq_huff_decode")
    return out, status
