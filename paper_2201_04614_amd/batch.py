"""A batch of fields compressed and decompressed by one HIP graph launch
(binding of include/dq_batch.h; argument marshalling only).

    b = Batch([(x0, dict(eb=1e-3, eb_mode="rel", block=8)), (x1, dict(eb=1e-4, block=16)), ...])
    b.launch()             # one graph launch: every field compressed and decompressed
    b.results()            # per field: compress and decompress dq_result

Batch replays every field's own kernels from the graph (over parallel
branches); PersistentBatch captures a fixed handful of kernels whatever the
number of fields: persistent encode and decode kernels draining a flattened
(field, tile) queue with an atomic ticket, one per (dimensionality, block,
cells per lane) class.
"""

from __future__ import annotations

import ctypes as C

from . import binding as dq

# every function include/dq_batch.h declares
EXPORTS = ["dq_batch_graph_create", "dq_batch_graph_launch", "dq_batch_graph_destroy",
           "dq_batch_persistent_workspace", "dq_batch_persistent_create", "dq_batch_persistent_run"]


class Field(C.Structure):
    _fields_ = [("p", dq.Params), ("x", C.c_void_p), ("codes", C.c_void_p), ("out_idx", C.c_void_p),
                ("out_val", C.c_void_p), ("out_cap", C.c_uint64), ("pads", C.c_void_p), ("cres", C.c_void_p),
                ("cws", C.c_void_p), ("cws_bytes", C.c_uint64), ("x_hat", C.c_void_p), ("dres", C.c_void_p),
                ("dws", C.c_void_p), ("dws_bytes", C.c_uint64)]


_ready = False


def lib():
    global _ready
    L = dq.lib()
    if not _ready:
        vp = C.c_void_p
        L.dq_batch_graph_create.argtypes = [C.POINTER(Field), C.c_uint64, C.c_int, C.POINTER(C.c_void_p)]
        L.dq_batch_graph_create.restype = C.c_int
        L.dq_batch_graph_launch.argtypes = [vp, vp]
        L.dq_batch_graph_launch.restype = C.c_int
        L.dq_batch_graph_destroy.argtypes = [vp]
        L.dq_batch_graph_destroy.restype = C.c_int
        L.dq_batch_persistent_workspace.argtypes = [C.POINTER(Field), C.c_uint64, C.POINTER(C.c_uint64)]
        L.dq_batch_persistent_workspace.restype = C.c_int
        L.dq_batch_persistent_create.argtypes = [C.POINTER(Field), C.c_uint64, vp, C.c_uint64,
                                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_void_p)]
        L.dq_batch_persistent_run.argtypes = [vp, vp, C.POINTER(dq.Hooks), C.POINTER(dq.Hooks)]
        L.dq_batch_persistent_run.restype = C.c_int
        L.dq_batch_persistent_create.restype = C.c_int
        _ready = True
    return L


def _p(t):
    return C.c_void_p(t.data_ptr())


def _fields(items, decompress=True):
    codecs = []
    arr = (Field * len(items))()
    for k, (x, kw) in enumerate(items):
        kw = dict(kw)
        eb = kw.pop("eb")
        cd = dq.Codec(tuple(x.shape), eb, device=x.device, **kw)
        codecs.append(cd)
        f = arr[k]
        f.p = cd.p
        f.x, f.codes = _p(x), _p(cd.codes)
        f.out_idx, f.out_val, f.out_cap = _p(cd.out_idx), _p(cd.out_val), cd.out_cap
        f.pads, f.cres = _p(cd.pads), _p(cd.res)
        f.cws, f.cws_bytes = _p(cd.ws_c), cd.ws_c.numel()
        f.x_hat = _p(cd.x_hat) if decompress else None
        f.dres, f.dws, f.dws_bytes = _p(cd.dres), _p(cd.ws_d), cd.ws_d.numel()
    return codecs, arr


class Batch:
    """Codecs for a list of (field tensor, codec keyword arguments) and the
    graph that runs all of them. Each x must stay alive and keep its storage."""

    def __init__(self, items, branches=4, decompress=True):
        self.items = items
        self.codecs, self._fields = _fields(items, decompress)
        h = C.c_void_p()
        st = lib().dq_batch_graph_create(self._fields, len(items), int(branches), C.byref(h))
        if st != dq.DQ_OK:
            raise dq.DQError(st, "dq_batch_graph_create")
        self._h = h

    def launch(self, stream=None):
        st = lib().dq_batch_graph_launch(self._h, dq._stream_handle(stream))
        if st != dq.DQ_OK:
            raise dq.DQError(st, "dq_batch_graph_launch")

    def results(self, stream=None):
        return [(cd.result(stream), cd.decompress_result(stream)) for cd in self.codecs]

    def close(self):
        if getattr(self, "_h", None):
            lib().dq_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PersistentBatch(Batch):
    """The same batch through dq_batch_persistent_create: every field needs
    out_cap >= its cell count and a padding other than global_mean.
    run() enqueues the same kernels without the graph; with hooks=True it
    records HIP events around the largest class's encode and decode kernels
    (self.enc_hook, self.dec_hook)."""

    def __init__(self, items, hooks=False):
        self.items = items
        self.enc_hook = dq.Hook() if hooks else None
        self.dec_hook = dq.Hook() if hooks else None
        self.codecs, self._fields = _fields(items, True)
        need = C.c_uint64(0)
        st = lib().dq_batch_persistent_workspace(self._fields, len(items), C.byref(need))
        if st != dq.DQ_OK:
            raise dq.DQError(st, "dq_batch_persistent_workspace")
        self.ws = dq._aligned_bytes(int(need.value), items[0][0].device)
        h = C.c_void_p()
        cls = (C.c_int32 * len(items))()
        vec = (C.c_int32 * len(items))()
        st = lib().dq_batch_persistent_create(self._fields, len(items), _p(self.ws), self.ws.numel(), cls, vec,
                                              C.byref(h))
        if st != dq.DQ_OK:
            raise dq.DQError(st, "dq_batch_persistent_create")
        self._h = h
        self.field_class = list(cls)  # 0: the class with the most cells (timed by the hooks)
        self.field_vec = list(vec)

    def run(self, stream=None):
        hk = self.enc_hook is not None
        st = lib().dq_batch_persistent_run(self._h, dq._stream_handle(stream),
                                           C.byref(self.enc_hook.struct) if hk else None,
                                           C.byref(self.dec_hook.struct) if hk else None)
        if st != dq.DQ_OK:
            raise dq.DQError(st, "dq_batch_persistent_run")

    def close(self):
        super().close()
        for hk in (self.enc_hook, self.dec_hook):
            if hk:
                hk.close()
