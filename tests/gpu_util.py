"""Helpers of the GPU parity tests: run the HIP path and the oracle on the
same fp32 input and compare every output element by element."""

import sys

import numpy as np

from paper_2201_04614_amd import binding as dq


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_compress(x, eb, eb_mode, block, pad, radius, out_cap=None, x_dev=None, vec=0, pads=None):
    """Compress on the GPU; returns host copies of everything. pads: the
    per-block values of the "given" padding mode."""
    import torch
    if x_dev is None:
        x_dev = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    codec = dq.Codec(x.shape, eb, eb_mode, block, pad, radius,
                     out_cap=x.size if out_cap is None else out_cap, vec=vec)
    if pads is not None:
        pv = torch.from_numpy(np.ascontiguousarray(pads, dtype=np.int32).reshape(-1))
        codec.pads[:pv.numel()].copy_(pv)
    codec.compress_async(x_dev)
    r = codec.result()
    n = int(r.n_out)
    k = min(n, codec.out_cap)
    out = dict(status=r.status, n_out=n, eb_abs=r.eb_abs,
               codes=codec.codes.cpu().numpy().view(np.uint16),
               out_idx=codec.out_idx[:k].cpu().numpy().view(np.uint32),
               out_val=codec.out_val[:k].cpu().numpy(),
               pads=codec.pads[:dq.pad_count(codec.p)].cpu().numpy(),
               codec=codec)
    return out


def gpu_decompress(codec, eb_abs, codes, out_idx, out_val, pads):
    import torch
    dev = codec.device
    c = torch.from_numpy(np.ascontiguousarray(codes).view(np.int16)).to(dev)
    i = torch.from_numpy(np.ascontiguousarray(out_idx, dtype=np.uint32).view(np.int32)).to(dev)
    v = torch.from_numpy(np.ascontiguousarray(out_val, dtype=np.int32)).to(dev)
    pd = torch.from_numpy(np.ascontiguousarray(pads, dtype=np.int32)).to(dev)
    if i.numel() == 0:
        i = torch.zeros(1, dtype=torch.int32, device=dev)
        v = torch.zeros(1, dtype=torch.int32, device=dev)
    if pd.numel() == 0:
        pd = None
    out = codec.decompress_async(eb_abs, len(out_idx), codes=c, out_idx=i, out_val=v, pads=pd)
    r = codec.decompress_result()
    return r.status, out.cpu().numpy()


def assert_same_compress(g, c, ctx=""):
    assert g["status"] == c.status, (ctx, g["status"], c.status)
    if c.status != 0:
        return
    assert g["n_out"] == c.n_out, (ctx, g["n_out"], c.n_out)
    assert np.float64(g["eb_abs"]).tobytes() == np.float64(c.eb_abs).tobytes(), (ctx, g["eb_abs"], c.eb_abs)
    gc, cc = g["codes"].ravel(), c.codes.ravel()
    if not np.array_equal(gc, cc):
        bad = np.flatnonzero(gc != cc)
        raise AssertionError(f"{ctx}: {bad.size} codes differ, first {bad[:8]} gpu {gc[bad[:8]]} ref {cc[bad[:8]]}")
    assert np.array_equal(g["out_idx"], c.out_idx), ctx
    assert np.array_equal(g["out_val"], c.out_val), ctx
    assert np.array_equal(g["pads"], c.pads), ctx


def parity(ref, x, eb, eb_mode="abs", block=16, pad="zero", radius=512, nthreads=0,
           check_decode=True, x_dev=None, vec=0, pads=None, out_cap=None):
    """Full comparison of compress and decompress; returns the oracle result.
    out_cap: outlier capacity of the GPU call (default: the cell count); below
    the oracle's count the call must fail with ECAPACITY, report the true
    count and still write the oracle's codes."""
    ctx = f"shape={x.shape} eb={eb} {eb_mode} B={block} pad={pad} R={radius} cap={out_cap}"
    p = ref.params(x.shape, eb, eb_mode, block, pad, radius)
    c = ref.compress(p, x, nthreads=nthreads, pads=pads)
    g = gpu_compress(x, eb, eb_mode, block, pad, radius, out_cap=out_cap, x_dev=x_dev, vec=vec, pads=pads)
    if out_cap is not None and c.status == 0 and c.n_out > out_cap:
        assert g["status"] == dq.DQ_ECAPACITY and g["n_out"] == c.n_out, (ctx, g["status"], g["n_out"], c.n_out)
        assert np.array_equal(g["codes"].ravel(), c.codes.ravel()), ctx
        return c
    assert_same_compress(g, c, ctx)
    if c.status == 0 and check_decode:
        st, xr = ref.decompress(p, c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads, nthreads=nthreads)
        assert st == 0
        gst, xg = gpu_decompress(g["codec"], c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads)
        assert gst == 0, ctx
        if not np.array_equal(xg.view(np.uint32), xr.view(np.uint32)):
            bad = np.flatnonzero(xg.ravel().view(np.uint32) != xr.ravel().view(np.uint32))
            raise AssertionError(f"{ctx}: {bad.size} decoded values differ, first {bad[:8]}")
    return c
