"""Independent numpy restatement of the blocked Lorenzo transform (test pin).

It reaches the oracle's results by a different route, so that a mistake in
either shows up as a disagreement:

* padding statistics use exact rational means (fractions.Fraction), rounded
  to the nearest integer with halves toward +infinity;
* the Lorenzo residual of a block is np.diff applied along every axis of the
  block after the halo row/plane (the padding) has been prepended - the
  textbook mixed backward difference, instead of the oracle's signed sum
  over the corners of the unit cell;
* the inverse for zero padding is np.cumsum along every axis of the block
  (a summed-area table), instead of the oracle's point-by-point
  reconstruction.

All integer arithmetic wraps modulo 2^32 like the codec's.
"""

from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

ZERO, BLOCK_MEAN, EDGE_MEAN, GLOBAL_MEAN = 0, 1, 2, 3
BLOCK_MIN, BLOCK_MAX, GLOBAL_MIN, GLOBAL_MAX = 4, 5, 6, 7
GIVEN = 8  # per-block values supplied by the caller


def wrap32(a):
    a = np.asarray(a, dtype=np.int64)
    return ((a + 2 ** 31) % 2 ** 32 - 2 ** 31).astype(np.int64)


def nearest_half_up(num, den):
    """Nearest integer to num/den, exact halves rounded toward +infinity."""
    return int(math.floor(Fraction(int(num), int(den)) + Fraction(1, 2)))


def block_slices(shape, B):
    """Slices of every block, blocks in row-major order of the block grid."""
    grids = [range(0, n, B) for n in shape]
    for origin in itertools.product(*grids):
        yield tuple(slice(o, min(o + B, n)) for o, n in zip(origin, shape))


def pad_values(q, B, mode):
    q = np.asarray(q, dtype=np.int64)
    d = q.ndim
    if mode == ZERO:
        return np.zeros(0, dtype=np.int64)
    if mode == GLOBAL_MEAN:
        return np.array([nearest_half_up(int(q.sum()), q.size)], dtype=np.int64)
    if mode in (GLOBAL_MIN, GLOBAL_MAX):
        return np.array([q.min() if mode == GLOBAL_MIN else q.max()], dtype=np.int64)
    out = []
    for sl in block_slices(q.shape, B):
        blk = q[sl]
        if mode == BLOCK_MEAN:
            out.append(nearest_half_up(int(blk.sum()), blk.size))
        elif mode in (BLOCK_MIN, BLOCK_MAX):
            out.append(int(blk.min() if mode == BLOCK_MIN else blk.max()))
        else:
            for a in range(d):
                face = np.take(blk, 0, axis=a)
                out.append(nearest_half_up(int(face.sum()), face.size))
    return np.array(out, dtype=np.int64)


def halo_of(mode, pads, b, d, axes):
    """Padding value of a halo cell lying in front of the block along `axes`."""
    if mode == ZERO:
        return 0
    if mode in (GLOBAL_MEAN, GLOBAL_MIN, GLOBAL_MAX):
        return int(pads[0])
    if mode in (BLOCK_MEAN, BLOCK_MIN, BLOCK_MAX, GIVEN):
        return int(pads[b])
    vals = [int(pads[b * d + a]) for a in axes]
    if len(vals) == 1:
        return vals[0]
    return nearest_half_up(sum(vals), len(vals))


def padded_block(blk, mode, pads, b):
    """Block with one halo layer prepended along every axis."""
    d = blk.ndim
    P = np.zeros(tuple(n + 1 for n in blk.shape), dtype=np.int64)
    P[(slice(1, None),) * d] = blk
    for idx in itertools.product(*[range(n + 1) for n in blk.shape]):
        axes = [a for a in range(d) if idx[a] == 0]
        if axes:
            P[idx] = halo_of(mode, pads, b, d, axes)
    return P


def residuals(q, B, mode, pads):
    """Lorenzo residual of q (natural layout) with the given padding."""
    q = np.asarray(q, dtype=np.int64)
    out = np.zeros(q.shape, dtype=np.int64)
    for b, sl in enumerate(block_slices(q.shape, B)):
        P = padded_block(q[sl], mode, pads, b)
        for a in range(q.ndim):
            P = np.diff(P, axis=a)
        out[sl] = P
    return wrap32(out)


def reconstruct_zero_pad(delta, B):
    """Inverse of the zero-padded residual: cumulative sums along each axis."""
    delta = np.asarray(delta, dtype=np.int64)
    out = np.zeros(delta.shape, dtype=np.int64)
    for sl in block_slices(delta.shape, B):
        S = delta[sl]
        for a in range(delta.ndim):
            S = np.cumsum(S, axis=a)
        out[sl] = S
    return wrap32(out)


def origin_mask(shape, B):
    m = np.zeros(shape, dtype=bool)
    m[tuple(slice(0, None, B) for _ in shape)] = True
    return m


def block_major_order(shape, B):
    """Linear indices of all cells, listed block by block (row-major block
    grid), cells in local row-major order."""
    lin = np.arange(int(np.prod(shape)), dtype=np.int64).reshape(shape)
    return np.concatenate([lin[sl].ravel() for sl in block_slices(shape, B)])
