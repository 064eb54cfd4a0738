"""Per-block padding / block-size selector on the GPU (binding of dq_select.h).

The exhaustive search, the training of the 24-64-64-8 network and the
learned selection all run in libdq's kernels; this module marshals arguments
and sequences the calls:

* ``block_features``: statistics, candidates, origin flags, exhaustive pad
  labels and the 24 features of every block;
* ``exhaustive_search``: per block the best of the five candidate pads, per
  16^d super-block the best block edge in {4, 8, 16} (one zero-pad
  compression per edge supplies the other cells' outliers);
* ``train``: Adam on the two heads' cross-entropy with the exhaustive labels;
* ``learned_pads``: bf16 inference and the chosen candidates as the values of
  the "given" padding mode, which decodes exactly like any per-block pad.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import binding as dq

N_FEAT, N_CAND, N_OUT, SUPER = 24, 5, 8, 16
BSIZES = (4, 8, 16)
N_PARAMS = 64 * 24 + 64 + 64 * 64 + 64 + 8 * 64 + 8
STAT_BYTES = 80
STAT_DTYPE = np.dtype([("qo", "<i4"), ("mn", "<i4"), ("mx", "<i4"), ("nonorig", "<u4"), ("sum", "<i8"),
                       ("mad", "<i8"), ("fsum", "<i8", (3,)), ("rough", "<i8", (3,))])
assert STAT_DTYPE.itemsize == STAT_BYTES

# every function include/dq_select.h declares
EXPORTS = ["dq_block_stats", "dq_block_select", "dq_super_cost", "dq_num_super", "dq_gather_pads",
           "dq_mlp_workspace", "dq_mlp_grad", "dq_mlp_adam", "dq_mlp_to_bf16", "dq_mlp_infer_bf16"]

_ready = False


def lib():
    global _ready
    L = dq.lib()
    if not _ready:
        P, vp, u64, pu64 = C.POINTER(dq.Params), C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64)
        sig = {
            "dq_block_stats": ([P, C.c_double, vp, vp, vp, vp, vp], C.c_int),
            "dq_block_select": ([P, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "dq_super_cost": ([P, vp, vp, vp, vp, vp], C.c_int),
            "dq_num_super": ([P, pu64], C.c_int),
            "dq_gather_pads": ([vp, vp, u64, vp, vp], C.c_int),
            "dq_mlp_workspace": ([u64, pu64], C.c_int),
            "dq_mlp_grad": ([vp, vp, vp, vp, u64, vp, vp, vp, u64, vp], C.c_int),
            "dq_mlp_adam": ([vp, vp, vp, vp, C.c_int32, C.c_float, vp], C.c_int),
            "dq_mlp_to_bf16": ([vp, vp, vp], C.c_int),
            "dq_mlp_infer_bf16": ([vp, vp, u64, vp, vp, vp, vp], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _ready = True
    return L


def _torch():
    import torch
    return torch


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _s(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check(st, what):
    if st != dq.DQ_OK:
        raise dq.DQError(st, what)


def num_super(shape, block):
    n = C.c_uint64(0)
    _check(lib().dq_num_super(C.byref(dq.make_params(shape, 1.0, "abs", block)), C.byref(n)), "dq_num_super")
    return int(n.value)


@dataclass
class BlockInfo:
    """Per-block selector data of one field and block edge (device tensors)."""
    stats: object    # uint8 [nb * 80] (dq_block_stat records)
    cand: object     # int32 [nb, 5]
    flags: object    # uint8 [nb]
    label: object    # int32 [nb]
    feat: object     # float32 [nb, 24]
    status: object   # int32 [1]

    def stats_host(self):
        return np.frombuffer(self.stats.cpu().numpy().tobytes(), dtype=STAT_DTYPE)


def block_features(x_dev, eb_abs, block, radius, codes=None, stream=None):
    """Statistics, candidates, flags, exhaustive labels and features of every
    block of x_dev (contiguous fp32 CUDA tensor) for the absolute bound eb_abs."""
    torch = _torch()
    shape = tuple(x_dev.shape)
    p = dq.make_params(shape, 1.0, "abs", block, "zero", radius)
    nb = dq.num_blocks(p)
    dev = x_dev.device
    stats = torch.empty(nb * STAT_BYTES, dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    cand = torch.empty((nb, N_CAND), dtype=torch.int32, device=dev)
    flags = torch.empty(nb, dtype=torch.uint8, device=dev)
    label = torch.empty(nb, dtype=torch.int32, device=dev)
    feat = torch.empty((nb, N_FEAT), dtype=torch.float32, device=dev)
    ws = torch.empty(1, dtype=torch.int64, device=dev)
    s = _s(stream)
    _check(lib().dq_block_stats(C.byref(p), float(eb_abs), _p(x_dev), _p(codes), _p(stats), _p(status), s),
           "dq_block_stats")
    _check(lib().dq_block_select(C.byref(p), _p(stats), _p(cand), _p(flags), _p(label), _p(feat), _p(ws), s),
           "dq_block_select")
    return BlockInfo(stats, cand, flags, label, feat, status)


def super_cost(shape, block, info, choice, stream=None):
    torch = _torch()
    p = dq.make_params(shape, 1.0, "abs", block)
    cost = torch.zeros(num_super(shape, block), dtype=torch.int64, device=info.cand.device)
    _check(lib().dq_super_cost(C.byref(p), _p(info.stats), _p(info.flags), _p(choice), _p(cost), _s(stream)),
           "dq_super_cost")
    return cost


def gather_pads(info, choice, stream=None):
    torch = _torch()
    nb = info.cand.shape[0]
    pads = torch.empty(nb, dtype=torch.int32, device=info.cand.device)
    _check(lib().dq_gather_pads(_p(info.cand), _p(choice), nb, _p(pads), _s(stream)), "dq_gather_pads")
    return pads


def resolve_eb(x_dev, eb, eb_mode):
    """Absolute bound (a relative one from the field's value range, as the codec does)."""
    if eb_mode == "abs":
        return float(eb)
    c = dq.Codec(tuple(x_dev.shape), eb, "rel", 8, "zero", 512, out_cap=0, device=x_dev.device)
    c.compress_async(x_dev)
    r = c.result()
    if r.status not in (dq.DQ_OK, dq.DQ_ECAPACITY):
        raise dq.DQError(r.status, "value range")
    return float(r.eb_abs)


@dataclass
class Search:
    """Exhaustive search of one field (device tensors unless noted); the
    per-edge dicts are keyed by the block edge."""
    eb_abs: float
    base: int                 # block edge of info / zero_out / best_out / sample_bsz
    infos: dict               # BlockInfo per edge
    zero_outs: dict           # outliers with zero padding per edge (host)
    best_outs: dict           # outliers with the best candidate of every block, per edge (host)
    super_cost: object        # int64 [3, n_super]: side cost per edge (8 * outliers + 4 * pads)
    super_label: object       # int64 [n_super]: best edge index (ties to the larger edge)
    sample_bszs: dict         # int32 [nb]: super-block label of every block, per edge

    @property
    def info(self):
        return self.infos[self.base]

    @property
    def zero_out(self):
        return self.zero_outs[self.base]

    @property
    def best_out(self):
        return self.best_outs[self.base]

    @property
    def sample_bsz(self):
        return self.sample_bszs[self.base]


def exhaustive_search(x_dev, eb, eb_mode, radius, base=8, stream=None):
    """Best candidate pad per block (every edge) and best block edge per super-block."""
    torch = _torch()
    shape = tuple(x_dev.shape)
    eb_abs = resolve_eb(x_dev, eb, eb_mode)
    costs, infos, zero_outs, best_outs = [], {}, {}, {}
    for B in BSIZES:
        codec = dq.Codec(shape, eb_abs, "abs", B, "zero", radius, out_cap=0, device=x_dev.device)
        codec.compress_async(x_dev, stream=stream)
        r = codec.result(stream)
        if r.status not in (dq.DQ_OK, dq.DQ_ECAPACITY):
            raise dq.DQError(r.status, f"zero-pad compression, block {B}")
        info = block_features(x_dev, eb_abs, B, radius, codes=codec.codes, stream=stream)
        del codec
        costs.append(super_cost(shape, B, info, info.label, stream))
        infos[B] = info
        zero_outs[B] = int(r.n_out)
        st = info.stats_host()
        fl = info.flags.cpu().numpy()
        lab = info.label.cpu().numpy()
        best_outs[B] = int(st["nonorig"].astype(np.int64).sum() + ((fl >> lab) & 1).astype(np.int64).sum())
    cost = torch.stack(costs)
    # ties keep the larger edge: scan from the largest
    lab = (len(BSIZES) - 1) - torch.argmin(torch.flip(cost, dims=[0]), dim=0)
    samples = {B: lab[_super_of_blocks(shape, B, x_dev.device)].to(torch.int32) for B in BSIZES}
    return Search(eb_abs, base, infos, zero_outs, best_outs, cost, lab, samples)


def _super_of_blocks(shape, B, device):
    torch = _torch()
    nsb = [(n + SUPER - 1) // SUPER for n in shape]
    grids = [torch.arange(0, n, B, device=device) // SUPER for n in shape]
    mesh = torch.meshgrid(*grids, indexing="ij")
    k = torch.zeros_like(mesh[0])
    for a in range(len(shape)):
        k = k * nsb[a] + mesh[a]
    return k.reshape(-1)


# ------------------------------------------------------------------ network

def init_params(seed=0, device="cuda"):
    """He-uniform weights, zero biases."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((64, 24), (64, 64), (8, 64)):
        lim = np.sqrt(6.0 / cols)
        parts += [rng.uniform(-lim, lim, size=rows * cols), np.zeros(rows)]
    return torch.from_numpy(np.concatenate(parts).astype(np.float32)).to(device)


def mlp_grad(theta, X, y_pad, y_bsz, ws=None, stream=None):
    torch = _torch()
    n = X.shape[0]
    need = C.c_uint64(0)
    _check(lib().dq_mlp_workspace(n, C.byref(need)), "dq_mlp_workspace")
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=X.device)
    g = torch.empty(N_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib().dq_mlp_grad(_p(theta), _p(X), _p(y_pad), _p(y_bsz), n, _p(g), _p(loss), _p(ws), ws.numel(),
                             _s(stream)), "dq_mlp_grad")
    return g, loss, ws


def mlp_adam(theta, m, v, g, t, lr, stream=None):
    _check(lib().dq_mlp_adam(_p(theta), _p(m), _p(v), _p(g), int(t), float(lr), _s(stream)), "dq_mlp_adam")


def to_bf16(theta, stream=None):
    torch = _torch()
    out = torch.empty(N_PARAMS, dtype=torch.int16, device=theta.device)
    _check(lib().dq_mlp_to_bf16(_p(theta), _p(out), _s(stream)), "dq_mlp_to_bf16")
    return out


def infer(theta_bf16, X, logits=False, stream=None):
    torch = _torch()
    n = X.shape[0]
    pc = torch.empty(n, dtype=torch.int32, device=X.device)
    bc = torch.empty(n, dtype=torch.int32, device=X.device)
    lg = torch.empty((n, N_OUT), dtype=torch.float32, device=X.device) if logits else None
    _check(lib().dq_mlp_infer_bf16(_p(theta_bf16), _p(X), n, _p(lg), _p(pc), _p(bc), _s(stream)),
           "dq_mlp_infer_bf16")
    return pc, bc, lg


def train(X, y_pad, y_bsz, epochs=8, batch=4096, lr=2e-3, seed=0, log=None):
    """Adam on mini-batches of the (device) samples; returns the fp32 parameters."""
    torch = _torch()
    dev = X.device
    theta = init_params(seed, dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    n = X.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(seed)
    ws, t = None, 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(dev)
        tot = 0.0
        for k in range(0, n, batch):
            idx = perm[k:k + batch]
            g, loss, ws = mlp_grad(theta, X[idx].contiguous(), y_pad[idx].contiguous(), y_bsz[idx].contiguous(),
                                   ws)
            t += 1
            mlp_adam(theta, m, v, g, t, lr)
            tot += float(loss.item()) * idx.numel()
        if log:
            log(f"epoch {ep}: loss {tot / n:.4f}")
    return theta


def learned_pads(theta_bf16, info, stream=None):
    """The network's padding choice for every block, as "given" pad values."""
    pc, bc, _ = infer(theta_bf16, info.feat, stream=stream)
    return gather_pads(info, pc, stream), pc, bc


# ------------------------------------------------------------------ mixed-edge streams

def mixed_exhaustive(x_dev, eb, eb_mode, radius, stream=None):
    """Exhaustive choice for a mixed stream: every super-block's edge with the
    lowest side cost (the search's super-block labels, taken by libdq's
    dq_super_label) and every block's best candidate at that edge. Returns
    (edges, pads in stream order, pad_off, search)."""
    from . import mixed as MX
    shape = tuple(x_dev.shape)
    s = exhaustive_search(x_dev, eb, eb_mode, radius, stream=stream)
    edges, _ = MX.super_label(shape, s.super_cost, stream)
    pad_off, _ = MX.pad_offsets(shape, edges, stream)
    by_edge = {B: gather_pads(s.infos[B], s.infos[B].label, stream) for B in BSIZES}
    n_pads = int(pad_off[-1].item())
    return edges, MX.gather_pads(shape, edges, pad_off, by_edge, n_pads, stream), pad_off, s


def mixed_learned(theta_bf16, x_dev, eb_abs, radius, base=8, stream=None):
    """The network's choice for a mixed stream: the block-size head's logits
    at edge `base` voted per super-block (dq_super_vote), the padding head
    per block at every edge. Returns (edges, pads in stream order, pad_off)."""
    from . import mixed as MX
    shape = tuple(x_dev.shape)
    by_edge = {}
    logits_base = None
    for B in BSIZES:
        info = block_features(x_dev, eb_abs, B, radius, stream=stream)
        pc, _, lg = infer(theta_bf16, info.feat, logits=B == base, stream=stream)
        by_edge[B] = gather_pads(info, pc, stream)
        if B == base:
            logits_base = lg
    edges, _ = MX.super_vote(shape, base, logits_base, stream)
    pad_off, _ = MX.pad_offsets(shape, edges, stream)
    n_pads = int(pad_off[-1].item())
    return edges, MX.gather_pads(shape, edges, pad_off, by_edge, n_pads, stream), pad_off
