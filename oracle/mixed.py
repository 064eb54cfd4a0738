"""Oracle of streams with one block edge per 16^d super-block (TEST
INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's CPU
baseline may use it; the product path never does).

The paper tunes the block size by trying configurations on the data
(Section III-E) and reports that the best padding depends on the data
(Sections IV, V-I). A mixed stream lets every 16^d super-block (aligned at
the origin, truncated at the field's end) carry its own block edge in
{4, 8, 16}; its blocks are aligned at the super-block origin. Since a block
never crosses a super-block, every super-block is coded exactly as a field of
its own: this oracle cuts the field into super-blocks and runs the codec
oracle (oracle/dqref.c, DQ_PAD_GIVEN with the super-block's slice of the
pads) on each, in row-major super-block order. Block order, pad order and
outlier order are those of the super-blocks one after another; outlier
indices are C-order indices into the whole field.
"""

from __future__ import annotations

import itertools

import numpy as np

from . import dqref

SUPER = 16
EDGES = (4, 8, 16)


def super_slices(shape):
    """Slices of every super-block, in row-major order of the super-block grid."""
    grids = [range(0, n, SUPER) for n in shape]
    for origin in itertools.product(*grids):
        yield tuple(slice(o, min(o + SUPER, n)) for o, n in zip(origin, shape))


def num_super(shape):
    return int(np.prod([(n + SUPER - 1) // SUPER for n in shape]))


def blocks_of(sub_shape, E):
    return int(np.prod([(n + E - 1) // E for n in sub_shape]))


def pad_offsets(shape, edges):
    """Exclusive prefix of the blocks of every super-block (n_super + 1 entries)."""
    counts = [blocks_of([s.stop - s.start for s in sl], int(E)) for sl, E in zip(super_slices(shape), edges)]
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def _to_global(local_idx, sl, shape):
    coords = np.unravel_index(np.asarray(local_idx, dtype=np.int64), [s.stop - s.start for s in sl])
    return np.ravel_multi_index(tuple(c + s.start for c, s in zip(coords, sl)), shape).astype(np.uint32)


def compress(x, eb_abs, radius, edges, pads):
    """(status, codes, out_idx, out_val) of the mixed stream; pads in stream order."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    off = pad_offsets(x.shape, edges)
    codes = np.zeros(x.shape, dtype=np.uint16)
    idx, val = [], []
    for s, sl in enumerate(super_slices(x.shape)):
        E = int(edges[s])
        sub = np.ascontiguousarray(x[sl])
        p = dqref.params(sub.shape, eb_abs, "abs", E, "given", radius)
        c = dqref.compress(p, sub, out_cap=sub.size, pads=np.asarray(pads[off[s]:off[s + 1]], dtype=np.int32))
        if c.status != dqref.OK:
            return c.status, None, None, None
        codes[sl] = c.codes
        idx.append(_to_global(c.out_idx, sl, x.shape))
        val.append(c.out_val)
    cat = (lambda a, t: np.concatenate(a).astype(t) if a else np.zeros(0, t))
    return dqref.OK, codes, cat(idx, np.uint32), cat(val, np.int32)


def decompress(shape, eb_abs, radius, edges, pads, codes, out_idx, out_val):
    """(status, x_hat): each super-block decoded by the codec oracle from its
    run of the outlier list (runs must follow the super-block order)."""
    shape = tuple(int(n) for n in shape)
    off = pad_offsets(shape, edges)
    out_idx = np.asarray(out_idx, dtype=np.int64)
    N = int(np.prod(shape))
    if out_idx.size and (out_idx.max() >= N):
        return dqref.ECORRUPT, None
    # super-block of every outlier; the list must visit them in order
    coords = np.unravel_index(out_idx, shape) if out_idx.size else [np.zeros(0, np.int64)] * len(shape)
    nsb = [(n + SUPER - 1) // SUPER for n in shape]
    sb = np.zeros(out_idx.size, dtype=np.int64)
    for a in range(len(shape)):
        sb = sb * nsb[a] + coords[a] // SUPER
    if sb.size and np.any(np.diff(sb) < 0):
        return dqref.ECORRUPT, None
    starts = np.searchsorted(sb, np.arange(num_super(shape) + 1), side="left")
    x_hat = np.zeros(shape, dtype=np.float32)
    for s, sl in enumerate(super_slices(shape)):
        E = int(edges[s])
        sub_shape = tuple(t.stop - t.start for t in sl)
        p = dqref.params(sub_shape, eb_abs, "abs", E, "given", radius)
        lo, hi = starts[s], starts[s + 1]
        g = out_idx[lo:hi]
        c = np.unravel_index(g, shape)
        local = np.ravel_multi_index(tuple(ci - t.start for ci, t in zip(c, sl)), sub_shape) if g.size else g
        st, xh = dqref.decompress(p, eb_abs, np.ascontiguousarray(codes[sl]), local.astype(np.uint32),
                                  np.asarray(out_val[lo:hi], dtype=np.int32),
                                  np.asarray(pads[off[s]:off[s + 1]], dtype=np.int32))
        if st != dqref.OK:
            return st, None
        x_hat[sl] = xh
    return dqref.OK, x_hat


def gather_pads(shape, edges, pads_by_edge):
    """Stream-order pads from per-edge pads in row-major block order of the
    whole field: block b of super-block s (edge E) takes pads_by_edge[E] at
    its block index in the field's grid of E-blocks."""
    out = []
    for sl, E in zip(super_slices(shape), edges):
        E = int(E)
        nbf = [(n + E - 1) // E for n in shape]
        ranges = [range(s.start // E, (s.stop + E - 1) // E) for s in sl]
        for bc in itertools.product(*ranges):
            u = 0
            for a in range(len(shape)):
                u = u * nbf[a] + bc[a]
            out.append(int(pads_by_edge[E][u]))
    return np.array(out, dtype=np.int32)
