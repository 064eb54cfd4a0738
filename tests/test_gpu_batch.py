"""Device-count decompression and the batch graph: parity with the oracle and
with eager calls, over several replays of one graph."""

import numpy as np
import pytest

import gpu_util as G
from paper_2201_04614_amd import batch as BT
from paper_2201_04614_amd import binding as dq
from paper_2201_04614_amd import fields as F

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,B,pad,R", [((70000,), 256, "zero", 3), ((200, 300), 16, "block_mean", 64),
                                           ((40, 50, 60), 8, "edge_mean", 2), ((33, 17, 65), 4, "global_max", 512)])
def test_decompress_dev_matches_oracle(ref, shape, B, pad, R):
    import torch
    x = F.uniform_field(shape, seed=B + R, lo=-100.0, hi=100.0)
    eb = 1e-3
    G.say(f"decompress_dev {shape} B={B} {pad} R={R}")
    p = ref.params(shape, eb, "abs", B, pad, R)
    c = ref.compress(p, x)
    st, xr = ref.decompress(p, c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads)
    assert st == 0
    cd = dq.Codec(shape, eb, "abs", B, pad, R, out_cap=x.size)
    xd = torch.from_numpy(x).cuda()
    cd.compress_async(xd)
    xh = cd.decompress_dev_async()
    rd = cd.decompress_result()
    assert rd.status == dq.DQ_OK and int(rd.n_out) == c.n_out and rd.eb_abs == c.eb_abs
    assert np.array_equal(xh.cpu().numpy().view(np.uint32), xr.view(np.uint32))
    # a second call on the same result buffer starts from a clean status word
    cd.compress_async(xd)
    cd.decompress_dev_async()
    assert cd.decompress_result().status == dq.DQ_OK


def test_decompress_refuses_counts_beyond_the_buffers():
    """The binding checks n_out against the outlier buffers it passes (the
    kernels read n_out entries), so a count from a compression that ran out
    of capacity is refused on the host."""
    cd = dq.Codec((64, 64), 1e-3, "abs", 8, "zero", 512, out_cap=10)
    with pytest.raises(dq.DQError):
        cd.decompress_async(1e-3, 11)


def test_decompress_dev_passes_compress_errors_on(ref):
    import torch
    x = F.uniform_field((64, 64), seed=3, lo=-100.0, hi=100.0)
    cd = dq.Codec(x.shape, 1e-4, "abs", 8, "zero", 4, out_cap=10)
    cd.compress_async(torch.from_numpy(x).cuda())
    cd.x_hat.fill_(7.0)
    cd.decompress_dev_async()
    r, rd = cd.result(), cd.decompress_result()
    assert r.status == dq.DQ_ECAPACITY and rd.status == dq.DQ_ECAPACITY and rd.n_out == r.n_out
    assert bool((cd.x_hat == 7.0).all())
    y = x.copy()
    y[5, 5] = np.nan
    cd2 = dq.Codec(x.shape, 1e-3, "rel", 8, "zero", 512)
    cd2.compress_async(torch.from_numpy(y).cuda())
    cd2.decompress_dev_async()
    assert cd2.result().status == dq.DQ_ERANGE and cd2.decompress_result().status == dq.DQ_ERANGE


def _batch_items():
    rng = np.random.default_rng(21)
    items = []
    specs = [((1 << 20) + 77,), (300000,), (4097,), (1800, 900), (333, 511), (64, 64), (96, 80, 112), (130, 70, 33),
             (8, 8, 8), (200, 120, 64)]
    for k, shape in enumerate(specs):
        if len(shape) == 3 and min(shape) >= 8:
            x = F.power_law_grf(shape, slope=float(rng.uniform(2, 4)), seed=100 + k)
        elif len(shape) == 2:
            x = F.sinusoid_field(shape, seed=100 + k)
        else:
            x = F.uniform_field(shape, seed=100 + k, lo=-5.0, hi=5.0)
        d = len(shape)
        B = int(rng.choice({1: [64, 256, 1024], 2: [8, 16, 32], 3: [4, 8, 16]}[d]))
        pad = ["zero", "block_mean", "edge_mean", "global_mean", "block_min"][k % 5]
        kw = dict(eb=float(10 ** rng.uniform(-4, -2)), eb_mode=["abs", "rel"][k % 2], block=B, pad=pad,
                  radius=int(rng.choice([64, 512])), out_cap=x.size)
        items.append((np.ascontiguousarray(x, dtype=np.float32), kw))
    return items


def _eager(x_dev, kw):
    kw = dict(kw)
    eb = kw.pop("eb")
    cd = dq.Codec(tuple(x_dev.shape), eb, device=x_dev.device, **kw)
    cd.compress_async(x_dev)
    r = cd.result()
    assert r.status == dq.DQ_OK, dq.strerror(r.status)
    cd.decompress_async(r.eb_abs, int(r.n_out))  # the host-count path
    return cd, r


def test_batch_graph_replays_match_eager(ref):
    import torch
    items = _batch_items()
    devs = [(torch.from_numpy(x).cuda(), kw) for x, kw in items]
    G.say(f"batch graph of {len(devs)} fields")
    b = BT.Batch(devs, branches=4)
    for rep in range(3):
        if rep == 2:  # eager work between replays changes one input in place
            devs[3][0].mul_(1.5)
        b.launch()
        torch.cuda.synchronize()
        for k, ((xd, kw), cd) in enumerate(zip(devs, b.codecs)):
            r, rd = cd.result(), cd.decompress_result()
            ecd, er = _eager(xd, kw)
            erd = ecd.decompress_result()
            ctx = f"replay {rep} field {k} {tuple(xd.shape)} {kw}"
            assert r.status == er.status == dq.DQ_OK, ctx
            assert int(r.n_out) == int(er.n_out) and r.eb_abs == er.eb_abs, ctx
            assert rd.status == erd.status == dq.DQ_OK, ctx
            assert torch.equal(cd.codes, ecd.codes), ctx
            n = int(r.n_out)
            assert torch.equal(cd.out_idx[:n], ecd.out_idx[:n]) and torch.equal(cd.out_val[:n], ecd.out_val[:n]), ctx
            assert torch.equal(cd.x_hat.view(torch.int32), ecd.x_hat.view(torch.int32)), ctx
            if k in (2, 5, 8):  # small fields: the oracle too
                x = xd.cpu().numpy()
                p = ref.params(x.shape, kw["eb"], kw["eb_mode"], kw["block"], kw["pad"], kw["radius"])
                c = ref.compress(p, x)
                assert c.n_out == n and np.array_equal(cd.codes.cpu().numpy().view(np.uint16), c.codes), ctx
    b.close()
