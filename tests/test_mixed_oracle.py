"""Pins of the mixed-edge stream oracle (oracle/mixed.py) against the codec
oracle run on the whole field and against hand-counted block layouts."""

import itertools

import numpy as np
import pytest

import npref as NP
from oracle import mixed as M
from paper_2201_04614_amd import fields as F

SHAPES = [(100,), (40, 37), (20, 33, 18)]


def _field(shape, seed):
    x = F.power_law_grf(shape, slope=2.5, seed=seed) * np.float32(60.0) + np.float32(30.0)
    if len(shape) == 1:
        x = F.uniform_field(shape, seed=seed, lo=-50.0, hi=90.0)
    return np.ascontiguousarray(x, dtype=np.float32)


def _uniform_pads(ref, x, eb, B, rng):
    nb = ref.num_blocks(ref.params(x.shape, eb, "abs", B, "given", 64))
    return rng.integers(-300, 300, nb).astype(np.int32)


def test_pad_offsets_hand_counted():
    """20 x 40: super-block rows of 16 and 4 cells, columns of 16, 16, 8."""
    edges = [4, 8, 16, 16, 4, 8]
    # (16x16 at 4) 16, (16x16 at 8) 4, (16x8 at 16) 1, (4x16 at 16) 1, (4x16 at 4) 4, (4x8 at 8) 1
    assert list(M.pad_offsets((20, 40), edges)) == [0, 16, 20, 21, 22, 26, 27]
    assert M.num_super((20, 40)) == 6 and M.num_super((100,)) == 7 and M.num_super((20, 33, 18)) == 12


@pytest.mark.parametrize("shape", SHAPES, ids=str)
def test_all_sixteen_is_the_uniform_stream(ref, shape):
    """Every edge 16: the super-blocks are the blocks, so the stream is the
    codec oracle's block-16 given-pads stream, bit for bit."""
    x = _field(shape, 3)
    eb, R = 0.05, 64
    rng = np.random.default_rng(1)
    pads = _uniform_pads(ref, x, eb, 16, rng)
    edges = [16] * M.num_super(shape)
    st, codes, idx, val = M.compress(x, eb, R, edges, pads)
    c = ref.compress(ref.params(shape, eb, "abs", 16, "given", R), x, out_cap=x.size, pads=pads)
    assert st == 0 and c.status == 0
    assert np.array_equal(codes, c.codes) and np.array_equal(idx, c.out_idx) and np.array_equal(val, c.out_val)


@pytest.mark.parametrize("shape", SHAPES, ids=str)
@pytest.mark.parametrize("E", [4, 8])
def test_one_edge_everywhere_matches_the_uniform_codes(ref, shape, E):
    """Every edge E < 16: the blocks are those of the uniform block-E stream
    (16 is a multiple of E), so the codes and the outlier set are the same;
    the list is ordered super-block by super-block instead."""
    x = _field(shape, 4)
    eb, R = 0.05, 32
    rng = np.random.default_rng(2)
    upads = _uniform_pads(ref, x, eb, E, rng)
    edges = [E] * M.num_super(shape)
    pads = M.gather_pads(shape, edges, {E: upads})
    st, codes, idx, val = M.compress(x, eb, R, edges, pads)
    c = ref.compress(ref.params(shape, eb, "abs", E, "given", R), x, out_cap=x.size, pads=upads)
    assert st == 0 and c.status == 0 and c.n_out == idx.size
    assert np.array_equal(codes, c.codes)
    assert sorted(zip(idx.tolist(), val.tolist())) == sorted(zip(c.out_idx.tolist(), c.out_val.tolist()))
    _check_stream_order(shape, edges, idx)


def _stream_key(shape, edges, i):
    """(super-block, block inside it, cell inside the block) of cell i."""
    coord = np.unravel_index(int(i), shape)
    nsb = [(n + 16 - 1) // 16 for n in shape]
    s = 0
    for a in range(len(shape)):
        s = s * nsb[a] + coord[a] // 16
    E = int(edges[s])
    org = [c // 16 * 16 for c in coord]
    ext = [min(16, n - o) for n, o in zip(shape, org)]
    nb = [(e + E - 1) // E for e in ext]
    b = 0
    for a in range(len(shape)):
        b = b * nb[a] + (coord[a] - org[a]) // E
    bext = [min(E, e - (c - o) // E * E) for e, c, o in zip(ext, coord, org)]
    loc = 0
    for a in range(len(shape)):
        loc = loc * bext[a] + (coord[a] - org[a]) % E
    return (s, b, loc)


def _check_stream_order(shape, edges, idx):
    keys = [_stream_key(shape, edges, i) for i in idx]
    assert all(k1 < k2 for k1, k2 in zip(keys, keys[1:]))


@pytest.mark.parametrize("shape", SHAPES, ids=str)
def test_random_edges_round_trip_and_agree_with_uniform_streams(ref, shape):
    """Random edges: inside each super-block the codes equal those of the
    whole-field uniform stream at that super-block's edge (same blocks, same
    pads); the list is in stream order; decoding gives q back, hence the same
    x_hat as any uniform stream."""
    x = _field(shape, 5)
    eb, R = 0.05, 16
    rng = np.random.default_rng(3)
    edges = rng.choice([4, 8, 16], M.num_super(shape))
    upads = {E: _uniform_pads(ref, x, eb, E, rng) for E in (4, 8, 16)}
    pads = M.gather_pads(shape, edges, upads)
    st, codes, idx, val = M.compress(x, eb, R, edges, pads)
    assert st == 0
    for E in (4, 8, 16):
        c = ref.compress(ref.params(shape, eb, "abs", E, "given", R), x, out_cap=x.size, pads=upads[E])
        for sl, e in zip(M.super_slices(shape), edges):
            if e == E:
                assert np.array_equal(codes[sl], c.codes[sl])
                inside = [(i, v) for i, v in zip(c.out_idx.tolist(), c.out_val.tolist())
                          if all(s.start <= k < s.stop for k, s in zip(np.unravel_index(i, shape), sl))]
                mine = [(i, v) for i, v in zip(idx.tolist(), val.tolist())
                        if all(s.start <= k < s.stop for k, s in zip(np.unravel_index(i, shape), sl))]
                assert sorted(inside) == sorted(mine)
    _check_stream_order(shape, edges, idx)
    st2, xh = M.decompress(shape, eb, R, edges, pads, codes, idx, val)
    assert st2 == 0
    z = ref.compress(ref.params(shape, eb, "abs", 8, "zero", R), x, out_cap=x.size)
    st3, xz = ref.decompress(ref.params(shape, eb, "abs", 8, "zero", R), z.eb_abs, z.codes, z.out_idx, z.out_val,
                             z.pads)
    assert st3 == 0 and np.array_equal(xh.view(np.uint32), xz.view(np.uint32))


def test_out_of_order_list_is_corrupt(ref):
    shape = (40, 37)
    x = _field(shape, 6)
    edges = np.random.default_rng(4).choice([4, 8, 16], M.num_super(shape))
    pads = np.zeros(int(M.pad_offsets(shape, edges)[-1]), dtype=np.int32)
    st, codes, idx, val = M.compress(x, 0.05, 8, edges, pads)
    assert st == 0 and idx.size > 2
    j = int(np.flatnonzero(np.diff([_stream_key(shape, edges, i)[0] for i in idx]))[0])  # last of a super-block
    bad = idx.copy()
    bad[[j, j + 1]] = bad[[j + 1, j]]
    assert M.decompress(shape, 0.05, 8, edges, pads, codes, bad, val)[0] == ref.ECORRUPT


def test_gather_pads_hand_worked():
    """1-D, 40 cells, edges 4, 16, 8: blocks 0..3 of the edge-4 grid, block 1
    of the edge-16 grid, block 4 of the edge-8 grid (cells 32..39)."""
    pb = {4: np.arange(100, 110), 8: np.arange(200, 205), 16: np.arange(300, 303)}
    assert list(M.gather_pads((40,), [4, 16, 8], pb)) == [100, 101, 102, 103, 301, 204]
