"""Oracle of the entropy stage over the quantisation codes (TEST INFRASTRUCTURE ONLY).

Only tests/ and the benchmark's CPU baseline may import this module; the
product path never does.

SZ passes the quantisation codes to a Huffman coder (Section II-B; the paper
keeps it out of the optimised step and lists better outlier and code
compression as future work). This module states the coder the GPU path
implements, plainly:

* histogram of the codes over the alphabet 0 .. n_symbols - 1;
* code lengths by the two-queue Huffman construction: the present symbols
  sorted by (frequency, symbol) form the leaf queue; internal nodes join a
  second queue in creation order; each step takes the lighter front, a leaf
  on equal weights; a single present symbol gets length 1. If a length
  exceeds 32, every present frequency is halved (kept >= 1) and the
  construction repeats;
* canonical codewords: symbols ordered by (length, symbol), the first gets
  0, each next one (previous + 1) shifted left by the length difference;
* the bitstream: chunks of CHUNK symbols, each starting on a 32-bit word,
  codewords concatenated most significant bit first; chunk_off[c] is the
  first word of chunk c (chunk_off[n_chunks] = total words); sub_off[c, k]
  (k = 0, 1, 2) is the bit offset, from the start of chunk c, of its symbol
  (k + 1) * SUB (the chunk's bit count when the chunk is shorter), so that a
  chunk can be decoded from four places at once.
"""

from __future__ import annotations

from collections import deque

import numpy as np

CHUNK = 1024
SUB = 256
MAX_LEN = 32


def histogram(codes, n_symbols):
    return np.bincount(np.asarray(codes, dtype=np.int64).ravel(), minlength=n_symbols)[:n_symbols]


def _lengths_once(freq):
    present = [s for s in range(len(freq)) if freq[s] > 0]
    L = np.zeros(len(freq), dtype=np.int64)
    if not present:
        return L
    if len(present) == 1:
        L[present[0]] = 1
        return L
    leaves = deque(sorted(present, key=lambda s: (int(freq[s]), s)))
    nodes = deque()          # (weight, node id) in creation order
    parent = {}
    nid = len(freq)          # internal node ids follow the symbols

    def take():
        if leaves and (not nodes or int(freq[leaves[0]]) <= nodes[0][0]):
            s = leaves.popleft()
            return int(freq[s]), s
        return nodes.popleft()

    while len(leaves) + len(nodes) > 1:
        wa, a = take()
        wb, b = take()
        parent[a] = nid
        parent[b] = nid
        nodes.append((wa + wb, nid))
        nid += 1
    root = nodes[0][1]
    depth = {root: 0}
    for v in range(nid - 1, len(freq) - 1, -1):   # internal nodes, parents before children
        if v in parent:
            depth[v] = depth[parent[v]] + 1
    for s in present:
        L[s] = depth[parent[s]] + 1
    return L


def code_lengths(freq):
    f = np.asarray(freq, dtype=np.int64).copy()
    while True:
        L = _lengths_once(f)
        if L.max(initial=0) <= MAX_LEN:
            return L
        f = np.where(f > 0, np.maximum(1, f >> 1), 0)


def canonical_codes(L):
    order = sorted([s for s in range(len(L)) if L[s] > 0], key=lambda s: (int(L[s]), s))
    C = np.zeros(len(L), dtype=np.int64)
    code, prev = 0, None
    for s in order:
        if prev is not None:
            code = (code + 1) << (int(L[s]) - int(L[prev]))
        C[s] = code
        prev = s
    return C


def encode(codes, L, C, chunk=CHUNK, with_sub=False):
    """Words (uint32) and chunk word offsets (uint64, n_chunks + 1); with
    with_sub also the sub-chunk bit offsets (uint16, n_chunks x 3)."""
    codes = np.asarray(codes, dtype=np.int64).ravel()
    n = codes.size
    nch = (n + chunk - 1) // chunk
    words, off, sub = [], [0], []
    for c in range(nch):
        bits = []
        marks = []
        for j, s in enumerate(codes[c * chunk:(c + 1) * chunk]):
            if j and j % SUB == 0:
                marks.append(len(bits))
            ln, cw = int(L[s]), int(C[s])
            bits.extend((cw >> (ln - 1 - k)) & 1 for k in range(ln))
        while len(marks) < 3:
            marks.append(len(bits))
        sub.append(marks[:3])
        nw = (len(bits) + 31) // 32
        bits += [0] * (32 * nw - len(bits))
        for w in range(nw):
            v = 0
            for b in bits[32 * w:32 * w + 32]:
                v = (v << 1) | b
            words.append(v)
        off.append(off[-1] + nw)
    words, off = np.array(words, dtype=np.uint32), np.array(off, dtype=np.uint64)
    if with_sub:
        return words, off, np.array(sub, dtype=np.uint16).reshape(-1, 3)
    return words, off


def decode(words, off, n, L, C, chunk=CHUNK):
    """Codes from the bitstream (bit by bit against the codeword table)."""
    table = {(int(L[s]), int(C[s])): s for s in range(len(L)) if L[s] > 0}
    out = np.zeros(n, dtype=np.int64)
    k = 0
    for c in range(len(off) - 1):
        pos = int(off[c]) * 32
        for _ in range(min(chunk, n - c * chunk)):
            code, ln = 0, 0
            while True:
                w = int(words[pos >> 5])
                code = (code << 1) | ((w >> (31 - (pos & 31))) & 1)
                pos += 1
                ln += 1
                if (ln, code) in table:
                    out[k] = table[(ln, code)]
                    k += 1
                    break
                if ln > MAX_LEN:
                    raise ValueError("invalid codeword")
    return out
