"""Mixed-edge streams on the GPU (dq_mixed_*): bit-exact against the oracle
that codes every super-block as a field of its own with the codec oracle;
the edge choice (exhaustive labels, network vote) and the pad gather against
their oracles; the selector's mixed streams decode to the uniform x_hat."""

import numpy as np
import pytest

import gpu_util as G
from oracle import mixed as M
from oracle import selector as S
from paper_2201_04614_amd import binding as dq
from paper_2201_04614_amd import fields as F
from paper_2201_04614_amd import mixed as MX
from paper_2201_04614_amd import selector as SEL

pytestmark = pytest.mark.gpu

SHAPES = [(100,), (5000,), (40, 37), (300, 517), (20, 33, 18), (64, 48, 40), (33, 70, 130)]


def _field(shape, seed):
    x = F.power_law_grf(shape, slope=2.5, seed=seed) * np.float32(60.0) + np.float32(30.0)
    if len(shape) == 1:
        x = F.uniform_field(shape, seed=seed, lo=-50.0, hi=90.0)
    return np.ascontiguousarray(x, dtype=np.float32)


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


@pytest.mark.parametrize("shape", SHAPES, ids=str)
@pytest.mark.parametrize("R", [16, 512])
def test_mixed_stream_bit_exact(ref, shape, R):
    import torch
    x = _field(shape, sum(shape) + R)
    eb = 0.05
    rng = np.random.default_rng(R + len(shape))
    edges = rng.choice([4, 8, 16], M.num_super(shape)).astype(np.uint8)
    n_pads = int(M.pad_offsets(shape, edges)[-1])
    pads = rng.integers(-300, 300, n_pads).astype(np.int32)
    G.say(f"mixed {shape} R={R}")
    st, codes, idx, val = M.compress(x, eb, R, edges, pads)
    assert st == 0
    ed = _dev(edges)
    off, est = MX.pad_offsets(shape, ed)
    assert int(est.item()) == 0
    assert np.array_equal(off.cpu().numpy(), M.pad_offsets(shape, edges))
    s = MX.compress(_dev(x), eb, R, ed, _dev(pads), pad_off=off)
    assert s.status == dq.DQ_OK and s.n_out == idx.size and s.eb_abs == eb
    assert np.array_equal(s.codes.cpu().numpy().view(np.uint16), codes)
    assert np.array_equal(s.out_idx.cpu().numpy().view(np.uint32), idx)
    assert np.array_equal(s.out_val.cpu().numpy(), val)
    st2, xr = M.decompress(shape, eb, R, edges, pads, codes, idx, val)
    assert st2 == 0
    # the GPU decoder fed the oracle's stream
    s2 = MX.MixedStream(shape, R, eb, int(idx.size), 0, ed, off, _dev(pads), _dev(codes.view(np.int16)),
                        _dev(idx.view(np.int32)) if idx.size else torch.zeros(1, dtype=torch.int32, device="cuda"),
                        _dev(val) if val.size else torch.zeros(1, dtype=torch.int32, device="cuda"))
    xh = MX.decompress(s2)
    assert np.array_equal(xh.cpu().numpy().view(np.uint32), xr.view(np.uint32))


def test_mixed_errors(ref):
    import torch
    shape = (40, 70)
    x = _field(shape, 8)
    rng = np.random.default_rng(8)
    edges = rng.choice([4, 8, 16], M.num_super(shape)).astype(np.uint8)
    n_pads = int(M.pad_offsets(shape, edges)[-1])
    pads = np.zeros(n_pads, dtype=np.int32)
    st, codes, idx, val = M.compress(x, 0.05, 8, edges, pads)
    ed = _dev(edges)
    # capacity: exact count, complete codes
    s = MX.compress(_dev(x), 0.05, 8, ed, _dev(pads), out_cap=idx.size - 1)
    assert s.status == dq.DQ_ECAPACITY and s.n_out == idx.size
    assert np.array_equal(s.codes.cpu().numpy().view(np.uint16), codes)
    # a list out of stream order, and an outlier on a non-zero code
    off, _ = MX.pad_offsets(shape, ed)
    j = idx.size // 2
    bad = idx.copy()
    bad[[j, j + 1]] = bad[[j + 1, j]]
    nz = int(np.flatnonzero(codes.ravel())[0])
    for ii, vv in ((bad, val), (np.sort(np.append(idx, nz)).astype(np.uint32), np.append(val, 0).astype(np.int32))):
        assert M.decompress(shape, 0.05, 8, edges, pads, codes, ii, vv)[0] == ref.ECORRUPT
        s2 = MX.MixedStream(shape, 8, 0.05, int(ii.size), 0, ed, off, _dev(pads), _dev(codes.view(np.int16)),
                            _dev(ii.view(np.int32)), _dev(vv))
        with pytest.raises(dq.DQError) as e:
            MX.decompress(s2)
        assert e.value.status == dq.DQ_ECORRUPT
    # an edge other than 4 / 8 / 16
    e2 = edges.copy()
    e2[0] = 5
    _, est = MX.pad_offsets(shape, _dev(e2))
    assert int(est.item()) == dq.DQ_EINVAL


def test_edge_choice_and_gather_match_oracle():
    import torch
    rng = np.random.default_rng(9)
    for shape in [(100,), (40, 37), (20, 33, 18)]:
        ns = M.num_super(shape)
        cost = rng.integers(0, 50, (3, ns)).astype(np.int64) * 4  # many ties
        ed, lab = MX.super_label(shape, _dev(cost))
        want = np.array([min(range(2, -1, -1), key=lambda i: (cost[i, s], -i)) for s in range(ns)])
        assert np.array_equal(lab.cpu().numpy(), want)
        assert np.array_equal(ed.cpu().numpy(), np.array([4, 8, 16])[want])
        nb8 = int(np.prod([(n + 7) // 8 for n in shape]))
        lg = rng.normal(0, 1, (nb8, 8)).astype(np.float32)
        lg[::3, 5:] = 0.25  # ties
        _, vlab = MX.super_vote(shape, 8, _dev(lg))
        assert np.array_equal(vlab.cpu().numpy(), S.super_vote(shape, 8, lg))
        edges = rng.choice([4, 8, 16], ns).astype(np.uint8)
        pb = {E: rng.integers(-1000, 1000, int(np.prod([(n + E - 1) // E for n in shape]))).astype(np.int32)
              for E in (4, 8, 16)}
        off, _ = MX.pad_offsets(shape, _dev(edges))
        n_pads = int(off[-1].item())
        got = MX.gather_pads(shape, _dev(edges), off, {E: _dev(v) for E, v in pb.items()}, n_pads)
        assert np.array_equal(got.cpu().numpy(), M.gather_pads(shape, edges, pb))


def test_exhaustive_mixed_stream(ref):
    """The selector's exhaustive mixed stream: its side bytes are the sum of
    every super-block's cheapest edge cost, it matches the oracle, and it
    decodes to the x_hat of the plain zero-padding stream."""
    import torch
    shape = (48, 40, 56)
    x = _field(shape, 10) * np.float32(3.0)
    eb, R = 0.05, 64
    xd = _dev(x)
    edges, pads, off, srch = SEL.mixed_exhaustive(xd, eb, "abs", R)
    s = MX.compress(xd, eb, R, edges, pads, pad_off=off)
    assert s.status == dq.DQ_OK
    n_pads = int(off[-1].item())
    assert 8 * s.n_out + 4 * n_pads == int(srch.super_cost.min(dim=0).values.sum().item())
    e_h, p_h = edges.cpu().numpy(), pads.cpu().numpy()
    st, codes, idx, val = M.compress(x, eb, R, e_h, p_h)
    assert st == 0 and idx.size == s.n_out
    assert np.array_equal(s.codes.cpu().numpy().view(np.uint16), codes)
    assert np.array_equal(s.out_idx.cpu().numpy().view(np.uint32), idx)
    xh = MX.decompress(s)
    z = G.gpu_compress(x, eb, "abs", 8, "zero", R)
    zx = z["codec"].decompress_dev_async()
    assert torch.equal(xh.view(torch.int32), zx.view(torch.int32))
