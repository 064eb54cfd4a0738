"""Pins of the entropy-stage oracle (oracle/huffman.py): a hand-worked
codebook, the Kraft equality, prefix-freeness, optimality against an
independent heap construction, the length limit and round trips."""

import heapq
import itertools

import numpy as np
import pytest

from oracle import huffman as H


def test_worked_codebook():
    """Frequencies a5 b2 c1 d1 (symbols 0..3): c and d merge (2); b (a leaf)
    goes before that node on the tie, the node and b merge (4); that node and
    a form the root. Lengths a1 b2 c3 d3; canonical codewords 0, 10, 110, 111."""
    L = H.code_lengths(np.array([5, 2, 1, 1]))
    assert L.tolist() == [1, 2, 3, 3]
    assert H.canonical_codes(L).tolist() == [0b0, 0b10, 0b110, 0b111]
    words, off = H.encode(np.array([0, 1, 2, 3, 0]), L, H.canonical_codes(L))
    # 0 10 110 111 0 -> 0101 1011 10 + zeros
    assert off.tolist() == [0, 1] and words[0] == 0b0101101110 << 22


def _optimal_cost(freq):
    """Sum of f * length of an optimal prefix code: the sum of the merged
    weights of any Huffman construction (heap, independent of tie rules)."""
    h = [int(f) for f in freq if f > 0]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


@pytest.mark.parametrize("seed", range(8))
def test_kraft_prefix_free_and_optimal(seed):
    rng = np.random.default_rng(seed)
    K = int(rng.integers(2, 60))
    freq = rng.integers(0, 1000, size=K) * (rng.random(K) < 0.7)
    if (freq > 0).sum() < 2:
        freq[:2] = [3, 5]
    L = H.code_lengths(freq)
    C = H.canonical_codes(L)
    present = np.flatnonzero(freq > 0)
    assert np.all(L[freq == 0] == 0) and np.all(L[present] >= 1)
    assert sum(2.0 ** -int(L[s]) for s in present) == 1.0  # a full binary tree
    for a, b in itertools.permutations(present, 2):
        la, lb = int(L[a]), int(L[b])
        if la <= lb:
            assert (int(C[b]) >> (lb - la)) != int(C[a])  # no codeword prefixes another
    assert int((freq * L).sum()) == _optimal_cost(freq)


def test_length_limit():
    """Fibonacci frequencies give a tree of depth n - 1; over 40 symbols the
    lengths are limited to 32 by halving the frequencies, and the code stays
    complete and decodable."""
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    freq = np.array(fib)
    assert H._lengths_once(freq).max() == 39
    L = H.code_lengths(freq)
    assert L.max() <= 32
    assert sum(2.0 ** -int(l) for l in L) == 1.0
    C = H.canonical_codes(L)
    codes = np.repeat(np.arange(40), 3)
    w, off = H.encode(codes, L, C, chunk=16)
    assert np.array_equal(H.decode(w, off, codes.size, L, C, chunk=16), codes)


def test_single_symbol_and_round_trips():
    L = H.code_lengths(np.array([0, 0, 7, 0]))
    assert L.tolist() == [0, 0, 1, 0]
    w, off = H.encode(np.full(100, 2), L, H.canonical_codes(L), chunk=64)
    assert off.tolist() == [0, 2, 4] and np.all(w == 0)  # 64 bits, then 36 bits
    rng = np.random.default_rng(1)
    for n, K, chunk in ((1, 5, 4), (1000, 33, 64), (5000, 1025, 1024)):
        codes = np.minimum(rng.geometric(0.05, size=n) - 1, K - 1)
        L = H.code_lengths(H.histogram(codes, K))
        C = H.canonical_codes(L)
        w, off = H.encode(codes, L, C, chunk=chunk)
        assert off[-1] == w.size and off.size == (n + chunk - 1) // chunk + 1
        assert np.array_equal(H.decode(w, off, n, L, C, chunk=chunk), codes)


def test_sub_chunk_offsets():
    """Sub-chunk offsets: the bits of the first 256 / 512 / 768 codewords of
    each chunk, or the chunk's bit count for a shorter chunk."""
    rng = np.random.default_rng(4)
    codes = np.minimum(rng.geometric(0.1, size=2500) - 1, 63)
    L = H.code_lengths(H.histogram(codes, 64))
    C = H.canonical_codes(L)
    w, off, sub = H.encode(codes, L, C, with_sub=True)
    for c in range(sub.shape[0]):
        part = codes[c * 1024:(c + 1) * 1024]
        for k in range(3):
            assert sub[c, k] == int(L[part[:256 * (k + 1)]].sum())
