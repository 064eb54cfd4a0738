"""GPU canonical Huffman coding against its oracle: histogram, lengths and
codewords bit-exact, the bitstream word for word, decode round trips, and the
error statuses (every case stays inside its buffers)."""

import numpy as np
import pytest

import gpu_util as G
from oracle import huffman as H
from paper_2201_04614_amd import binding as dq
from paper_2201_04614_amd import fields as F
from paper_2201_04614_amd import huffman as HF

pytestmark = pytest.mark.gpu


def _dev(codes):
    import torch
    return torch.from_numpy(np.ascontiguousarray(codes, dtype=np.uint16).view(np.int16)).cuda()


def _check_codebook(codes, K):
    cb = HF.codebook(_dev(codes), K)
    hist = H.histogram(codes, K)
    L = H.code_lengths(hist)
    Cw = H.canonical_codes(L)
    assert int(cb.status.item()) == 0
    assert np.array_equal(cb.hist.cpu().numpy().view(np.uint32), hist)
    assert np.array_equal(cb.lengths.cpu().numpy(), L)
    assert np.array_equal(cb.codewords.cpu().numpy().view(np.uint32), Cw)
    return cb, L, Cw


def _codes_cases():
    rng = np.random.default_rng(3)
    x = F.sinusoid_field((256, 256), seed=1)
    z = G.gpu_compress(x, 1e-4 * F.field_range(x), "abs", 16, "zero", 512)
    yield "sinusoid codes", z["codes"].ravel(), 1024
    g = F.power_law_grf((48, 40, 36), seed=2)
    z = G.gpu_compress(g, 1e-3, "rel", 8, "block_mean", 64)
    yield "grf codes R64", z["codes"].ravel(), 128
    yield "geometric", np.minimum(rng.geometric(0.02, size=200003) - 1, 4095), 4096
    yield "uniform 2000", rng.integers(0, 2000, size=50000), 2000
    yield "single symbol", np.full(3000, 17), 32
    yield "one code", np.array([5]), 8
    yield "large alphabet", rng.integers(0, 300, size=10000) * 200, 65536


@pytest.mark.parametrize("case", range(7))
def test_codebook_and_bitstream_bit_exact(case):
    name, codes, K = list(_codes_cases())[case]
    G.say(f"huffman {name} n={codes.size} K={K}")
    cb, L, Cw = _check_codebook(codes, K)
    cd = _dev(codes)
    bs = HF.encode(cd, cb)
    words, off, sub = H.encode(codes, L, Cw, with_sub=True)
    assert int(bs.status.item()) == 0
    assert np.array_equal(bs.chunk_off.cpu().numpy().view(np.uint64), off)
    assert np.array_equal(bs.sub_off.cpu().numpy().view(np.uint16), sub)
    assert np.array_equal(bs.words[:words.size].cpu().numpy().view(np.uint32), words)
    back, st = HF.decode(bs, cb)
    assert int(st.item()) == 0
    assert np.array_equal(back.cpu().numpy().view(np.uint16), codes.astype(np.uint16))


def test_length_limit_on_the_gpu():
    """Fibonacci frequencies over 35 symbols: the unlimited tree is 34 deep;
    the limited lengths (frequencies halved) match the oracle and decode."""
    fib = [1, 1]
    while len(fib) < 35:
        fib.append(fib[-1] + fib[-2])
    codes = np.repeat(np.arange(35), fib)
    np.random.default_rng(0).shuffle(codes)
    assert H._lengths_once(np.array(fib)).max() == 34
    cb, L, Cw = _check_codebook(codes, 64)
    assert L.max() <= 32
    bs = HF.encode(_dev(codes), cb)
    back, st = HF.decode(bs, cb)
    assert int(st.item()) == 0 and np.array_equal(back.cpu().numpy().view(np.uint16), codes)


def test_round_trip_full_size_codes():
    """The 256^3 workload's codes (block-mean padding, radius 512): decode
    gives them back; the stream is much smaller than 2 bytes per code."""
    import torch
    x = F.power_law_grf((256, 256, 256), seed=2)
    cdc = dq.Codec(x.shape, 1e-3, "rel", 8, "block_mean", 512)
    cdc.compress_async(torch.from_numpy(x).cuda())
    assert cdc.result().status == dq.DQ_OK
    codes = cdc.codes.reshape(-1)
    cb = HF.codebook(codes, 1024)
    bs = HF.encode(codes, cb)
    back, st = HF.decode(bs, cb)
    assert int(cb.status.item()) == 0 and int(bs.status.item()) == 0 and int(st.item()) == 0
    assert torch.equal(back, codes)
    words = int(bs.chunk_off[-1].item())
    assert 4 * words < codes.numel() * 2 // 2  # under a byte per code


def test_error_statuses():
    import torch
    rng = np.random.default_rng(1)
    codes = rng.integers(0, 100, size=5000)
    cb = HF.codebook(_dev(codes), 50)  # codes >= n_symbols
    assert int(cb.status.item()) == dq.DQ_EINVAL
    many = np.arange(3000) % 2500  # 2500 distinct codes > DQ_HUFF_MAX_PRESENT
    cb = HF.codebook(_dev(many), 4096)
    assert int(cb.status.item()) == dq.DQ_ENOTSUP
    good = rng.integers(0, 100, size=5000)
    cb = HF.codebook(_dev(good), 128)
    bs = HF.encode(_dev(good), cb, words_cap=10)  # too small
    assert int(bs.status.item()) == dq.DQ_ECAPACITY
    bs = HF.encode(_dev(good), cb)
    assert int(bs.status.item()) == 0
    # a stream cut short: decoding stays inside the words given and reports corruption
    total = int(bs.chunk_off[-1].item())
    _, st = HF.decode(bs, cb, n_words=total // 2)
    assert int(st.item()) == dq.DQ_ECORRUPT
    # a codebook without the codes' symbols: encode reports them
    other = HF.codebook(_dev(rng.integers(100, 128, size=100)), 128)
    bs2 = HF.encode(_dev(good), other)
    assert int(bs2.status.item()) == dq.DQ_EINVAL
    torch.cuda.synchronize()


@pytest.mark.parametrize("case", ["sinusoid", "grf-rel", "uniform-outliers"])
def test_end_to_end_stream_with_entropy(ref, case):
    """compress(entropy=True) -> decompress: the decoded field equals the
    oracle's decompression bit for bit, and the coded stream is smaller than
    the raw codes would make it."""
    import torch
    if case == "sinusoid":
        x = F.sinusoid_field((512, 512), seed=1)
        args = (1e-4 * F.field_range(x), "abs", 16, "zero", 512)
    elif case == "grf-rel":
        x = F.power_law_grf((64, 64, 64), seed=2)
        args = (1e-3, "rel", 8, "block_mean", 512)
    else:
        x = F.uniform_field((100000,), seed=5, lo=-10.0, hi=10.0)
        args = (1e-3, "abs", 256, "zero", 64)
    G.say(f"end to end with entropy: {case}")
    s = dq.compress(torch.from_numpy(x).cuda(), *args, entropy=True)
    assert s.codes is None and s.coded is not None
    xh = dq.decompress(s).cpu().numpy()
    p = ref.params(x.shape, *args)
    c = ref.compress(p, x)
    st, xr = ref.decompress(p, c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads)
    assert st == 0 and s.n_out == c.n_out
    assert np.array_equal(xh.view(np.uint32), xr.view(np.uint32))
    raw = 2 * x.size + 8 * s.n_out + 4 * s.pads.numel() + 64
    assert s.stream_bytes() < raw
