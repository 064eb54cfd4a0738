"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: every expected value comes
from a hand-worked example, a closed form, an exact rational computation, a
textbook numpy routine (np.diff / np.cumsum on halo-padded blocks), or an
invariant of the method.
"""

import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import npref as NP
from paper_2201_04614_amd import fields as F

HERE = os.path.dirname(os.path.abspath(__file__))
PADS = ["zero", "block_mean", "edge_mean", "global_mean", "block_min", "block_max", "global_min", "global_max"]
PAD_ID = {"zero": 0, "block_mean": 1, "edge_mean": 2, "global_mean": 3,
          "block_min": 4, "block_max": 5, "global_min": 6, "global_max": 7}


def golden():
    with open(os.path.join(HERE, "golden", "worked_examples.json")) as f:
        return json.load(f)


# ------------------------------------------------------------ worked examples

@pytest.mark.parametrize("case", golden()["prequant"], ids=lambda c: f"eb{c['eb']}")
def test_prequant_worked_examples(ref, case):
    x = np.array(case["x"], dtype=np.float32)
    p = ref.params(x.shape, case["eb"], "abs", 4, "zero", 512)
    st, q = ref.prequantize(p, x, case["eb"])
    assert st == ref.OK
    assert q.tolist() == case["q"]


@pytest.mark.parametrize("case", golden()["codec"],
                         ids=lambda c: f"{len(c['shape'])}d-{c['pad']}")
def test_codec_worked_examples(ref, case):
    shape = tuple(case["shape"])
    x = np.array(case["x"], dtype=np.float32).reshape(shape)
    p = ref.params(shape, 0.5, "abs", case["block"], case["pad"], case["radius"])
    c = ref.compress(p, x)
    assert c.status == ref.OK
    assert c.codes.ravel().tolist() == case["codes"]
    assert c.out_idx.tolist() == case["out_idx"]
    assert c.out_val.tolist() == case["out_val"]
    assert c.pads.tolist() == case["pads"]
    st, xh = ref.decompress(p, c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads)
    assert st == ref.OK
    assert np.array_equal(xh, x)  # eb = 0.5: q = x and 2 eb q = x exactly


# ------------------------------------------------------------ rounding helpers

def test_round_mean_is_nearest_half_up(ref):
    rng = np.random.default_rng(7)
    cases = [(0, 1), (1, 2), (-1, 2), (3, 2), (-3, 2), (5, 3), (-5, 3), (7, 4),
             (-7, 4), (2 ** 62, 3), (-(2 ** 62), 7), (2 ** 63 - 1, 2 ** 32 - 1),
             (-(2 ** 63), 2 ** 32 - 1), (2 ** 63 - 1, 1), (-(2 ** 63), 1),
             (-(2 ** 63), 2), (2 ** 63 - 2, 4)]
    for _ in range(2000):
        n = int(rng.integers(1, 1 << 20))
        S = int(rng.integers(-(1 << 40), 1 << 40))
        cases.append((S, n))
        cases.append((n * int(rng.integers(-1000, 1000)) + n // 2, n))
    for S, n in cases:
        assert ref.round_mean(S, n) == NP.nearest_half_up(S, n), (S, n)


# ------------------------------------------------------------ P1: error bound

def _exact_bound_violations(x, eb, q, idx):
    ebf = Fraction(eb)
    bad = []
    for i in idx:
        err = Fraction(float(x.flat[i])) - 2 * ebf * int(q.flat[i])
        if abs(err) > ebf:
            bad.append(int(i))
    return bad


def _check_bound_everywhere(x, eb, q):
    """|x - 2 eb q| <= eb for every element: exact rational check on every
    element that is not far from a rounding boundary, and on a sample."""
    t = np.abs(x.astype(np.float64) / (2.0 * eb) - q.astype(np.float64))
    near = np.flatnonzero(t.ravel() > 0.5 - 1e-6)
    rng = np.random.default_rng(0)
    sample = rng.choice(x.size, size=min(x.size, 5000), replace=False)
    assert t.max() < 0.5 + 1e-6
    assert _exact_bound_violations(x, eb, q, np.concatenate([near, sample])) == []


@pytest.mark.parametrize("eb_rel", [1e-2, 1e-3, 1e-4, 1e-5])
def test_prequant_bound_sinusoid(ref, eb_rel):
    x = F.sinusoid_field((256, 256), seed=11)
    eb = eb_rel * F.field_range(x)
    p = ref.params(x.shape, eb, "abs", 16, "zero", 512)
    st, q = ref.prequantize(p, x, eb)
    assert st == ref.OK
    _check_bound_everywhere(x, eb, q)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_prequant_bound_uniform_and_tiny_eb(ref, seed):
    x = F.uniform_field((50000,), seed, -1000.0, 1000.0)
    for eb in (0.5, 1e-3, 3.3e-5, 4.7e-7):
        p = ref.params(x.shape, eb, "abs", 16, "zero", 512)
        st, q = ref.prequantize(p, x, eb)
        assert st == ref.OK
        _check_bound_everywhere(x, eb, q)


def _half_even(v):
    fl = math.floor(v)
    frac = v - fl
    if frac > Fraction(1, 2) or (frac == Fraction(1, 2) and fl % 2 == 1):
        return fl + 1
    return fl


def test_prequant_is_nearest_integer_half_even(ref):
    # q is the nearest integer to the exact x/(2 eb), halves to even: a floor,
    # a truncation, halves away from zero or an inexact quotient fail here
    rng = np.random.default_rng(5)
    cases = [(F.uniform_field((20000,), 5, -50.0, 50.0), 0.37),
             (F.uniform_field((20000,), 6, -1000.0, 1000.0), 1e-3)]
    # exact halves: eb a power of two and x on the half-integer grid of 2 eb
    for k in (-3, 0, 4):
        eb = 2.0 ** k
        m = rng.integers(-4000, 4000, size=4000)
        cases.append(((m + 0.5) * 2 * eb, eb))
    for x, eb in cases:
        x = np.ascontiguousarray(x, dtype=np.float32)
        p = ref.params(x.shape, eb, "abs", 16, "zero", 512)
        st, q = ref.prequantize(p, x, eb)
        assert st == ref.OK
        for i in range(0, x.size, 3):
            v = Fraction(float(x[i])) / (2 * Fraction(eb))
            assert int(q[i]) == _half_even(v), (float(x[i]), eb)


# ------------------------------------------------------------ P2: round trip

@pytest.mark.parametrize("pad", PADS)
def test_round_trip_sinusoid(ref, pad):
    x = F.sinusoid_field((512, 512), seed=1)
    eb = 1e-4 * F.field_range(x)
    p = ref.params(x.shape, eb, "abs", 16, pad, 512)
    c = ref.compress(p, x)
    assert c.status == ref.OK
    st, q = ref.prequantize(p, x, eb)
    st, xh = ref.decompress(p, c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads)
    assert st == ref.OK
    # decode returns q exactly, dequantised with one fp64 product
    expect = (q.astype(np.float64) * (2.0 * eb)).astype(np.float32)
    assert np.array_equal(xh.view(np.uint32), expect.view(np.uint32))
    err = np.abs(xh.astype(np.float64) - x.astype(np.float64))
    half_ulp = np.spacing(np.abs(xh)).astype(np.float64) / 2
    assert np.all(err <= eb * (1 + 1e-12) + half_ulp)


@pytest.mark.parametrize("pad", PADS)
def test_round_trip_grf_3d_rel(ref, pad):
    x = F.power_law_grf((48, 40, 36), seed=3) + np.float32(5.0)
    p = ref.params(x.shape, 1e-3, "rel", 8, pad, 512)
    c = ref.compress(p, x)
    assert c.status == ref.OK
    assert c.eb_abs == 1e-3 * (np.float64(x.max()) - np.float64(x.min()))
    st, xh = ref.decompress(p, c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads)
    assert st == ref.OK
    assert np.abs(xh.astype(np.float64) - x).max() <= c.eb_abs * (1 + 1e-6)


# ------------------------------------------------------------ P3 / P4: closed forms

def _affine_expected_delta(shape, B, q0, slopes, pad):
    """Closed form of the residual of q[u] = q0 + sum_a slopes[a] u_a."""
    d = len(shape)
    delta = np.zeros(shape, dtype=np.int64)
    for sl in NP.block_slices(shape, B):
        o = [s.start for s in sl]
        ext = [s.stop - s.start for s in sl]
        qo = q0 + sum(sa * oa for sa, oa in zip(slopes, o))
        blk = np.zeros(ext, dtype=np.int64)
        for u in itertools.product(*[range(e) for e in ext]):
            nz = [a for a in range(d) if u[a] != 0]
            if len(nz) >= 2:
                blk[u] = 0
            elif len(nz) == 1:
                blk[u] = slopes[nz[0]]
        # origin: q_o minus the effective pad
        if pad == "zero":
            peff = 0
        elif pad == "block_mean":  # mean of an arithmetic grid = centre value
            peff = math.floor(Fraction(qo) + sum(Fraction(slopes[a] * (ext[a] - 1), 2)
                                                 for a in range(d)) + Fraction(1, 2))
        elif pad == "global_mean":
            peff = math.floor(Fraction(q0) + sum(Fraction(slopes[a] * (shape[a] - 1), 2)
                                                 for a in range(d)) + Fraction(1, 2))
        elif pad in ("block_min", "block_max"):  # extreme corner of the block
            pick = min if pad == "block_min" else max
            peff = qo + sum(pick(0, slopes[a] * (ext[a] - 1)) for a in range(d))
        elif pad in ("global_min", "global_max"):  # extreme corner of the field
            pick = min if pad == "global_min" else max
            peff = q0 + sum(pick(0, slopes[a] * (shape[a] - 1)) for a in range(d))
        else:  # edge: face a mean = centre of the face; inclusion-exclusion
            E = [math.floor(Fraction(qo) + sum(Fraction(slopes[b] * (ext[b] - 1), 2)
                                                for b in range(d) if b != a) + Fraction(1, 2))
                 for a in range(d)]
            peff = 0
            for m in range(1, d + 1):
                for S in itertools.combinations(range(d), m):
                    h = E[S[0]] if m == 1 else math.floor(Fraction(sum(E[a] for a in S), m)
                                                          + Fraction(1, 2))
                    peff += (-1) ** (m + 1) * h
        blk[(0,) * d] = qo - peff
        delta[sl] = blk
    return delta


AFFINE = [((37,), 8, 5, (3,)), ((64,), 16, -700, (-2,)), ((21, 34), 8, 11, (3, -5)),
          ((32, 32), 16, -300, (1, 1)), ((9, 10, 13), 4, 7, (2, -1, 3)),
          ((16, 16, 16), 8, 1000, (-3, 2, 1)), ((5, 17, 6), 2, 0, (0, 0, 4))]


@pytest.mark.parametrize("shape,B,q0,slopes", AFFINE)
@pytest.mark.parametrize("pad", PADS)
def test_affine_fields_closed_form(ref, shape, B, q0, slopes, pad):
    x = F.affine_integer_field(shape, q0, slopes)
    R = 512
    p = ref.params(shape, 0.5, "abs", B, pad, R)
    c = ref.compress(p, x)
    assert c.status == ref.OK
    delta = _affine_expected_delta(shape, B, q0, slopes, pad)
    inl = np.abs(delta) < R
    expect_codes = np.where(inl, delta + R, 0)
    assert np.array_equal(c.codes.astype(np.int64), expect_codes)
    order = NP.block_major_order(shape, B)
    out = order[~inl.ravel()[order]]
    assert np.array_equal(c.out_idx.astype(np.int64), out)
    assert np.array_equal(c.out_val.astype(np.int64), delta.ravel()[out])


@pytest.mark.parametrize("shape,B", [((100,), 16), ((30, 45), 8), ((10, 12, 9), 4)])
@pytest.mark.parametrize("c0", [0, 7, -300, 511, 512, -512, 100000])
def test_constant_field(ref, shape, B, c0):
    x = F.constant_field(shape, c0)
    R = 512
    origins = NP.origin_mask(shape, B)
    for pad in PADS:
        p = ref.params(shape, 0.5, "abs", B, pad, R)
        c = ref.compress(p, x)
        assert c.status == ref.OK
        assert np.all(c.codes[~origins] == R)
        if pad == "zero":
            if abs(c0) < R:
                assert np.all(c.codes[origins] == R + c0) and c.n_out == 0
            else:
                assert np.all(c.codes[origins] == 0)
                assert c.n_out == origins.sum() and np.all(c.out_val == c0)
        else:  # every statistic of a constant equals it: nothing left to code
            assert np.all(c.codes[origins] == R) and c.n_out == 0


# ------------------------------------------------------------ P5 / P6 / P7 textbook

def _tiny_shapes():
    return [(1,), (7,), (16,), (33,), (1, 1), (3, 5), (9, 11), (8, 8), (4, 1),
            (2, 2, 2), (5, 6, 7), (3, 1, 4), (1, 6, 2)]


def _blocks_for(shape):
    m = max(shape)
    return sorted(set(list(range(1, min(m, 6) + 1)) + [m, m + 3]))


@pytest.mark.parametrize("shape", _tiny_shapes(), ids=str)
def test_residuals_equal_diff_of_halo_padded_blocks(ref, shape):
    rng = np.random.default_rng(len(shape) * 100 + sum(shape))
    for amp in (3, 40, 2 ** 31 - 200):
        q = rng.integers(-amp, amp + 1, size=shape).astype(np.int32)
        for B in _blocks_for(shape):
            for pad in PADS:
                p = ref.params(shape, 0.5, "abs", B, pad, 512)
                st, pads = ref.pad_values(p, q)
                assert st == ref.OK
                assert np.array_equal(pads.astype(np.int64), NP.pad_values(q, B, PAD_ID[pad]))
                st, d = ref.residuals(p, q, pads)
                assert st == ref.OK
                assert np.array_equal(d.astype(np.int64),
                                      NP.residuals(q, B, PAD_ID[pad], pads)), (B, pad)
                st, back = ref.reconstruct(p, d, pads)
                assert st == ref.OK and np.array_equal(back, q)
                if pad == "zero":
                    assert np.array_equal(NP.reconstruct_zero_pad(d, B), q.astype(np.int64))


@pytest.mark.parametrize("shape", [(33,), (9, 11), (5, 6, 7)], ids=str)
@pytest.mark.parametrize("R", [1, 2, 3, 512])
def test_codes_and_outliers_brute_force(ref, shape, R):
    rng = np.random.default_rng(R + len(shape))
    x = rng.integers(-6, 7, size=shape).astype(np.float32)
    for B in _blocks_for(shape):
        for pad in PADS:
            p = ref.params(shape, 0.5, "abs", B, pad, R)
            c = ref.compress(p, x)
            assert c.status == ref.OK
            q = x.astype(np.int64)
            delta = NP.residuals(q, B, PAD_ID[pad], NP.pad_values(q, B, PAD_ID[pad]))
            inl = (delta > -R) & (delta < R)
            assert np.array_equal(c.codes.astype(np.int64), np.where(inl, delta + R, 0))
            order = NP.block_major_order(shape, B)
            out = order[~inl.ravel()[order]]
            assert c.n_out == out.size
            assert np.array_equal(c.out_idx.astype(np.int64), out)
            assert np.array_equal(c.out_val.astype(np.int64), delta.ravel()[out])
            if R == 1:  # every non-zero residual is an outlier
                assert c.n_out == int(np.count_nonzero(delta))
            st, xh = ref.decompress(p, c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads)
            assert st == ref.OK and np.array_equal(xh, x)


@pytest.mark.parametrize("shape,B", [((200,), 16), ((40, 50), 8), ((12, 14, 10), 4)])
def test_pad_locality(ref, shape, B):
    """Any two paddings give the same residual except at block origins."""
    rng = np.random.default_rng(3)
    q = rng.integers(-5000, 5000, size=shape).astype(np.int32)
    origins = NP.origin_mask(shape, B)
    base = None
    for pad in PADS:
        p = ref.params(shape, 0.5, "abs", B, pad, 512)
        _, pads = ref.pad_values(p, q)
        _, d = ref.residuals(p, q, pads)
        if base is None:
            base = d
        else:
            assert np.array_equal(d[~origins], base[~origins])


# ------------------------------------------------------------ P8 / P9 and scale

def test_counting_and_thread_invariance_c1(ref):
    x = F.sinusoid_field((512, 512), seed=1)
    eb = 1e-4 * F.field_range(x)
    p = ref.params(x.shape, eb, "abs", 16, "zero", 512)
    c1 = ref.compress(p, x, nthreads=1)
    c8 = ref.compress(p, x, nthreads=8)
    for a, b in [(c1.codes, c8.codes), (c1.out_idx, c8.out_idx), (c1.out_val, c8.out_val)]:
        assert np.array_equal(a, b)
    st, q = ref.prequantize(p, x, eb)
    delta = NP.residuals(q, 16, 0, NP.pad_values(q, 16, 0))
    assert c1.n_out == int(np.count_nonzero(np.abs(delta) >= 512))
    assert np.all((c1.codes == 0) == (np.abs(delta) >= 512))
    st1, x1 = ref.decompress(p, c1.eb_abs, c1.codes, c1.out_idx, c1.out_val, c1.pads, nthreads=1)
    st8, x8 = ref.decompress(p, c1.eb_abs, c1.codes, c1.out_idx, c1.out_val, c1.pads, nthreads=8)
    assert st1 == st8 == ref.OK and np.array_equal(x1, x8)


def test_offset_field_padding_removes_border_outliers(ref):
    """Section IV / V-I: on a field with few near-zero values, zero padding
    leaves the block origins unpredictable; mean padding predicts them."""
    x = F.power_law_grf((64, 64, 64), seed=2)
    x = x + np.float32(2.0 * F.field_range(x))
    counts = {}
    for pad in ("zero", "block_mean", "edge_mean"):
        p = ref.params(x.shape, 1e-3, "rel", 8, pad, 512)
        c = ref.compress(p, x)
        assert c.status == ref.OK
        counts[pad] = c.n_out
    assert counts["zero"] >= (64 // 8) ** 3  # every origin
    assert counts["block_mean"] < counts["zero"] and counts["edge_mean"] < counts["zero"]


@pytest.mark.parametrize("shape,seed", [((300,), 1), ((37, 41), 2), ((9, 13, 11), 3)])
def test_global_extreme_pad_is_prequantised_extreme(ref, shape, seed):
    """Rounding to the nearest integer is monotone, so the minimum (maximum)
    of q is the prequantised minimum (maximum) of x: the global min / max
    pads need only the value range of the field."""
    x = F.power_law_grf(shape, seed=seed) * np.float32(7.0) - np.float32(3.0)
    for eb in (1e-2, 1e-3, 3.7e-5):
        xe = np.array([x.min(), x.max()], dtype=np.float32)
        pe = ref.params(xe.shape, eb, "abs", 4, "zero", 512)
        st, qe = ref.prequantize(pe, xe, eb)
        assert st == ref.OK
        for pad, want in (("global_min", qe[0]), ("global_max", qe[1])):
            p = ref.params(x.shape, eb, "abs", 4, pad, 512)
            st, q = ref.prequantize(p, x, eb)
            st, pads = ref.pad_values(p, q)
            assert st == ref.OK and pads.shape == (1,) and pads[0] == want


@pytest.mark.parametrize("shape,B", [((101,), 8), ((23, 30), 4), ((9, 10, 11), 4)])
def test_given_pads(ref, shape, B):
    """Per-block values chosen by the caller: the halo of each block is its
    value (checked against the halo-padded np.diff restatement); the block
    means reproduce block-mean padding; the origin values themselves leave
    every origin residual zero; random values round-trip."""
    rng = np.random.default_rng(sum(shape) + B)
    x = F.power_law_grf(shape, seed=7) * np.float32(50.0)
    eb = 1e-2
    pm = ref.params(shape, eb, "abs", B, "block_mean", 512)
    cm = ref.compress(pm, x)
    pg = ref.params(shape, eb, "abs", B, "given", 512)
    cg = ref.compress(pg, x, pads=cm.pads)
    assert cg.status == ref.OK and np.array_equal(cg.codes, cm.codes)
    assert np.array_equal(cg.out_idx, cm.out_idx) and np.array_equal(cg.out_val, cm.out_val)
    st, q = ref.prequantize(pg, x, eb)
    origins = NP.origin_mask(shape, B)
    qo = q[origins]  # block-major order equals the row-major order of the origins
    co = ref.compress(pg, x, pads=qo)
    assert np.all(co.codes[origins] == 512)
    assert not np.any(np.isin(co.out_idx, np.flatnonzero(origins.ravel())))
    rp = rng.integers(-3000, 3000, size=qo.size).astype(np.int32)
    cr = ref.compress(pg, x, pads=rp)
    assert cr.status == ref.OK and np.array_equal(cr.pads, rp)
    st, d = ref.residuals(pg, q, rp)
    assert np.array_equal(d.astype(np.int64), NP.residuals(q, B, NP.GIVEN, rp))
    st, xh = ref.decompress(pg, cr.eb_abs, cr.codes, cr.out_idx, cr.out_val, cr.pads)
    assert st == ref.OK
    assert np.array_equal(xh, (q.astype(np.float64) * (2 * eb)).astype(np.float32))


def test_extreme_pads_bound_the_origin_residual(ref):
    """With block min (max) padding every origin residual is q_o - min >= 0
    (q_o - max <= 0), and zero exactly where the origin holds the block's
    extreme."""
    x = F.power_law_grf((40, 36, 28), seed=9)
    for pad, sign in (("block_min", 1), ("block_max", -1)):
        p = ref.params(x.shape, 1e-3, "rel", 4, pad, 1 << 15)
        c = ref.compress(p, x)
        assert c.status == ref.OK and c.n_out == 0
        origins = NP.origin_mask(x.shape, 4)
        d0 = c.codes[origins].astype(np.int64) - (1 << 15)
        assert np.all(sign * d0 >= 0)
        st, q = ref.prequantize(p, x, c.eb_abs)
        qo = q[origins].astype(np.int64)
        assert np.array_equal(d0, qo - c.pads.astype(np.int64))


# ------------------------------------------------------------ validation and errors

def test_validation(ref):
    good = dict(shape=(10, 10), eb=1e-3, eb_mode="abs", block=4, pad="zero", radius=512)
    assert ref.validate(ref.params(**good)) == ref.OK
    bad = [dict(shape=(0, 10)), dict(shape=(2, 3, 4, 5)), dict(eb=0.0), dict(eb=-1.0),
           dict(eb=float("nan")), dict(eb=float("inf")), dict(eb=1e-320), dict(block=0),
           dict(pad=9), dict(pad=-1), dict(radius=0), dict(radius=32769), dict(eb_mode=5),
           dict(shape=(65536, 65536))]
    for b in bad:
        kw = dict(good)
        kw.update(b)
        if len(kw["shape"]) > 3:
            p = ref.params((1, 1, 1), 1.0)
            p.ndim = 4
        else:
            p = ref.params(**kw)
        assert ref.validate(p) == ref.EINVAL, b
    p = ref.params((65535, 65537), 1.0)  # 2^32 - 1 elements is the largest field
    assert ref.validate(p) == ref.OK


def test_range_and_nonfinite(ref):
    x = F.uniform_field((1000,), 1)
    for v in (np.nan, np.inf, -np.inf):
        y = x.copy()
        y[17] = v
        for mode, eb in (("abs", 1e-3), ("rel", 1e-3)):
            c = ref.compress(ref.params(y.shape, eb, mode, 16, "zero", 512), y)
            assert c.status == ref.ERANGE
    y = x.copy()
    y[3] = 1e7
    c = ref.compress(ref.params(y.shape, 1e-3, "abs", 16, "zero", 512), y)
    assert c.status == ref.ERANGE  # 1e7 / 2e-3 > 2^31
    # |q| <= 2^31 - 1 is the accepted range; eb = 0.5 makes q = x
    for v, st in ((2147483520.0, ref.OK), (2147483648.0, ref.ERANGE),
                  (-2147483520.0, ref.OK), (-2147483648.0, ref.ERANGE)):
        y = np.zeros(8, dtype=np.float32)
        y[5] = v
        c = ref.compress(ref.params(y.shape, 0.5, "abs", 4, "zero", 512), y)
        assert c.status == st, v
    c = ref.compress(ref.params(x.shape, 1e-3, "rel", 16, "zero", 512), F.constant_field((1000,), 3))
    assert c.status == ref.EINVAL  # zero value range


def test_capacity(ref):
    x = F.sinusoid_field((128, 128), seed=4)
    p = ref.params(x.shape, 1e-5 * F.field_range(x), "abs", 16, "zero", 64)
    full = ref.compress(p, x)
    assert full.status == ref.OK and full.n_out > 100
    part = ref.compress(p, x, out_cap=50)
    assert part.status == ref.ECAPACITY and part.n_out == full.n_out
    assert np.array_equal(part.out_idx, full.out_idx[:50])
    assert np.array_equal(part.codes, full.codes)


def test_corrupt_streams(ref):
    x = F.sinusoid_field((64, 64), seed=9)
    p = ref.params(x.shape, 1e-5 * F.field_range(x), "abs", 8, "block_mean", 32)
    c = ref.compress(p, x)
    assert c.status == ref.OK and c.n_out > 10

    def dec(codes, idx, val):
        return ref.decompress(p, c.eb_abs, codes, idx, val, c.pads)[0]

    assert dec(c.codes, c.out_idx, c.out_val) == ref.OK
    assert dec(c.codes, c.out_idx[1:], c.out_val[1:]) == ref.ECORRUPT  # missing outlier
    sw = c.out_idx.copy()
    sw[[3, 4]] = sw[[4, 3]]
    assert dec(c.codes, sw, c.out_val) == ref.ECORRUPT  # not block-major
    oob = c.out_idx.copy()
    oob[-1] = x.size
    assert dec(c.codes, oob, c.out_val) == ref.ECORRUPT  # index out of range
    nz = int(np.flatnonzero(c.codes.ravel())[0])
    extra_idx = np.sort(np.append(c.out_idx, nz))
    assert dec(c.codes, extra_idx, np.append(c.out_val, 0)) == ref.ECORRUPT
