"""Pins of the selector oracle (oracle/selector.py) against what the C oracle and
the mathematics fix independently of it."""

import math

import numpy as np
import pytest

import npref as NP
from oracle import selector as S
from paper_2201_04614_amd import fields as F

SHAPES = [((203,), 8), ((37, 41), 4), ((21, 18, 27), 4), ((24, 20, 16), 8), ((19, 33, 17), 16)]


def _q(ref, x, eb, B, pad="zero"):
    p = ref.params(x.shape, eb, "abs", B, pad, 512)
    st, q = ref.prequantize(p, x, eb)
    assert st == ref.OK
    return q


@pytest.mark.parametrize("shape,B", SHAPES, ids=str)
def test_candidates_are_the_oracle_pads(ref, shape, B):
    x = F.power_law_grf(shape, seed=3) * np.float32(40.0) + np.float32(9.0)
    eb = 1e-2
    q = _q(ref, x, eb, B)
    d = len(shape)
    st = S.block_stats(q, B)
    gmean = S.round_mean(int(q.astype(np.int64).sum()), q.size)
    cand = S.candidates(st, gmean, d)
    for pad, col in (("block_mean", 2), ("global_mean", 1)):
        p = ref.params(shape, eb, "abs", B, pad, 512)
        s2, pads = ref.pad_values(p, q)
        want = np.broadcast_to(pads.astype(np.int64), (len(st),)) if pad == "global_mean" else pads
        assert np.array_equal(cand[:, col], want)
    p = ref.params(shape, eb, "abs", B, "edge_mean", 512)
    s2, pads = ref.pad_values(p, q)
    e = pads.astype(np.int64).reshape(-1, d)
    # the origin's halo value along every axis set, by npref's rules
    for b in range(len(st)):
        want = 0
        for m in range(1, d + 1):
            import itertools
            for A in itertools.combinations(range(d), m):
                want += (-1) ** (m + 1) * NP.halo_of(NP.EDGE_MEAN, pads, b, d, list(A))
        assert cand[b, 3] == S.wrap32(want)
    mids = [NP.nearest_half_up(s["min"] + s["max"], 2) for s in st]
    assert np.array_equal(cand[:, 4], mids)
    assert np.all(cand[:, 0] == 0)


@pytest.mark.parametrize("shape,B", SHAPES, ids=str)
@pytest.mark.parametrize("R", [2, 40, 512])
def test_origin_flags_and_totals_match_the_codec(ref, shape, B, R):
    """The flags equal the origin codes of real compressions with each
    candidate as the padding, and the per-block best choice compressed with
    the given-pads mode has exactly the predicted outlier count."""
    x = F.power_law_grf(shape, seed=4) * np.float32(30.0) + np.float32(25.0)
    eb = 1e-2
    q = _q(ref, x, eb, B)
    d = len(shape)
    st = S.block_stats(q, B)
    gmean = S.round_mean(int(q.astype(np.int64).sum()), q.size)
    cand = S.candidates(st, gmean, d)
    flags = S.origin_outlier_flags(st, cand, R)
    origins = NP.origin_mask(shape, B)
    pg = ref.params(shape, eb, "abs", B, "given", R)
    for c in range(S.N_PAD):
        cc = ref.compress(pg, x, pads=cand[:, c].astype(np.int32))
        assert cc.status == ref.OK
        assert np.array_equal(cc.codes[origins] == 0, flags[:, c]), c
    z = ref.compress(ref.params(shape, eb, "abs", B, "zero", R), x)
    nonorig = S.nonorigin_outliers(z.codes, B)
    lab = S.pad_labels(flags)
    best = ref.compress(pg, x, pads=cand[np.arange(len(st)), lab].astype(np.int32))
    assert best.n_out == int(nonorig.sum() + flags[np.arange(len(st)), lab].sum())
    assert best.n_out == int(nonorig.sum() + flags.min(axis=1).sum())
    assert best.n_out <= z.n_out


def test_block_size_costs(ref):
    shape = (40, 36, 33)
    x = F.power_law_grf(shape, seed=6) * np.float32(60.0) + np.float32(100.0)
    eb, R = 1e-2, 64
    per_b, nout = [], []
    for B in S.BSIZES:
        q = _q(ref, x, eb, B)
        st = S.block_stats(q, B)
        gmean = S.round_mean(int(q.astype(np.int64).sum()), q.size)
        cand = S.candidates(st, gmean, 3)
        flags = S.origin_outlier_flags(st, cand, R)
        z = ref.compress(ref.params(shape, eb, "abs", B, "zero", R), x)
        lab = S.pad_labels(flags)
        per_b.append(S.nonorigin_outliers(z.codes, B) + flags[np.arange(len(st)), lab])
        c = ref.compress(ref.params(shape, eb, "abs", B, "given", R), x,
                         pads=cand[np.arange(len(st)), lab].astype(np.int32))
        nout.append(c.n_out)
    lab, cost = S.block_size_labels(shape, per_b)
    for i, B in enumerate(S.BSIZES):
        nb = int(np.prod([(n + B - 1) // B for n in shape]))
        assert cost[i].sum() == 8 * nout[i] + 4 * nb
    assert np.all(cost[lab, np.arange(cost.shape[1])] == cost.min(axis=0))


@pytest.mark.parametrize("shape,B,slopes", [((64,), 8, (3,)), ((20, 24), 4, (2, -5)), ((16, 12, 8), 4, (1, -2, 7))])
def test_features_affine_closed_form(ref, shape, B, slopes):
    """q = q0 + sum s_a u_a: every in-block difference along axis a is s_a, the
    range is sum |s_a| (ext_a - 1), and the midrange / mean sit at the centre."""
    q0, R = 1000, 256
    x = F.affine_integer_field(shape, q0, slopes)
    q = _q(ref, x, 0.5, B)
    d = len(shape)
    st = S.block_stats(q, B)
    gmean = S.round_mean(int(q.astype(np.int64).sum()), q.size)
    cand = S.candidates(st, gmean, d)
    f = S.features(st, cand, gmean, R, d, B)
    for b, sl in enumerate(NP.block_slices(shape, B)):
        ext = [s.stop - s.start for s in sl]
        for a in range(d):
            want = abs(slopes[a]) / R if ext[a] > 1 else 0.0
            assert f[b, 18 + a] == np.float32(min(want, S.CLAMP))
        rng_ = sum(abs(slopes[a]) * (ext[a] - 1) for a in range(d))
        assert f[b, 10] == np.float32(min(rng_ / R, S.CLAMP))
        assert cand[b, 4] == cand[b, 2]  # symmetric range: midrange = mean
    assert np.all(f[:, 22] == np.float32(d / 3.0)) and np.all(f[:, 23] == np.float32(math.log2(B) / 4))


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = S.init_params(1) * 0.5 + rng.normal(0, 0.05, S.n_params())
    X = rng.normal(0, 1, (7, S.N_FEAT))
    yp = rng.integers(0, S.N_PAD, 7)
    yb = rng.integers(0, S.N_BSZ, 7)
    g = S.grad(theta, X, yp, yb)
    idx = rng.choice(S.n_params(), 300, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (S.loss(theta + e, X, yp, yb) - S.loss(theta - e, X, yp, yb)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), i


def test_mlp_zero_network_and_adam_first_step():
    theta = np.zeros(S.n_params())
    X = np.ones((3, S.N_FEAT))
    assert math.isclose(S.loss(theta, X, [0, 1, 2], [0, 1, 2]), math.log(5) + math.log(3), rel_tol=1e-12)
    rng = np.random.default_rng(3)
    g = rng.normal(0, 1, S.n_params())
    th, m, v = S.adam_step(np.zeros_like(g), np.zeros_like(g), np.zeros_like(g), g, 1, 1e-3)
    # first step: m_hat = g, v_hat = g^2, so the update is lr * g / (|g| + eps)
    assert np.allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_bf16_rounding_worked_values():
    """bfloat16 keeps 7 fraction bits: at [1, 2) its step is 2^-7; exact ties
    go to the even neighbour."""
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, 1 + 2 ** -7 + 2 ** -8, -2.5, 0.1], dtype=np.float32)
    want = np.array([1.0, 1.0, 1 + 2 ** -7, 1 + 2 ** -6, -2.5, 0.10009765625], dtype=np.float32)
    assert np.array_equal(S.bf16_round(v), want)


# ------------------------------------------------- hand-worked statistics and features

def _golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "selector_worked.json")) as f:
        return json.load(f)["cases"]


def _fval(v):
    return np.float32(2.0 / 3.0) if v == "2/3" else np.float32(v)


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c["cite"][-22:])
def test_worked_statistics_candidates_features(case):
    """Every statistic, candidate, flag, label and feature of two tiny fields
    equals its hand-derived value (tests/golden/selector_worked.json)."""
    q = np.array(case["q"], dtype=np.int64)
    B, R, d = case["block"], case["radius"], q.ndim
    st = S.block_stats(q, B)
    gmean = S.round_mean(int(q.sum()), q.size)
    assert gmean == case["gmean"]
    assert len(st) == len(case["blocks"])
    for s, want in zip(st, case["blocks"]):
        for k in ("qo", "cells", "sum", "min", "max", "mad", "fsum", "fcnt", "rough", "npairs"):
            assert s[k] == want[k], k
    cand = S.candidates(st, gmean, d)
    assert np.array_equal(cand, [w["cand"] for w in case["blocks"]])
    f = S.features(st, cand, gmean, R, d, B)
    want = np.array([[_fval(v) for v in w["feat"]] for w in case["blocks"]], dtype=np.float32)
    for j in range(S.N_FEAT):
        assert np.array_equal(f[:, j], want[:, j]), f"feature {j}: {f[:, j]} != {want[:, j]}"
    flags = S.origin_outlier_flags(st, cand, 2)
    assert np.array_equal(flags, case["flags_r2"])
    assert np.array_equal(S.pad_labels(flags), case["labels_r2"])
    f1 = S.features(st, S.candidates(st, gmean, d), gmean, 1, d, B)
    assert np.array_equal(f1[:, 10], np.array(case["f10_r1"], dtype=np.float32))  # the clamp


def _rm_frac(v):
    """Nearest integer to the rational v, halves toward +infinity."""
    import fractions
    return math.floor(fractions.Fraction(v) + fractions.Fraction(1, 2))


@pytest.mark.parametrize("shape,B,slopes,q0,R", [
    ((50,), 8, (3,), 1000, 64),
    ((50,), 16, (-5,), -300, 32),
    ((20, 27), 4, (2, 5), 700, 16),
    ((23, 17), 8, (-3, -1), 40, 128),
    ((20, 27), 8, (4, -7), 900, 8),
    ((12, 10, 9), 4, (1, 2, 3), 500, 64),
    ((11, 13, 9), 4, (-2, -1, -4), -50, 16),
    ((9, 12, 10), 8, (3, -2, 1), 2000, 256)], ids=str)
def test_features_affine_closed_forms(shape, B, slopes, q0, R):
    """q = q0 + sum_a s_a u_a: every statistic and feature has a closed form
    in the block's origin o and extents e (partial blocks included):
      min / max = q_o + sum of the negative / positive s_a (e_a - 1);
      block mean = q_o + sum s_a (e_a - 1) / 2, the mean of the face u_a = 0
      lacks axis a's term; the field mean is q0 + sum s_a (n_a - 1) / 2;
      with slopes of one sign, mad = cells * sum |s_a| (e_a - 1) / 2."""
    from fractions import Fraction as Fr
    d = len(shape)
    x = F.affine_integer_field(shape, q0, slopes)
    q = x.astype(np.int64)  # eb = 0.5: q = x for integer x
    st = S.block_stats(q, B)
    gmean = S.round_mean(int(q.sum()), q.size)
    assert gmean == _rm_frac(q0 + sum(Fr(s * (n - 1), 2) for s, n in zip(slopes, shape)))
    cand = S.candidates(st, gmean, d)
    f = S.features(st, cand, gmean, R, d, B)
    one_sign = all(s >= 0 for s in slopes) or all(s <= 0 for s in slopes)

    def cl(v):
        return np.float32(min(max(float(v), -S.CLAMP), S.CLAMP))

    for b, sl in enumerate(NP.block_slices(shape, B)):
        o = [s.start for s in sl]
        e = [s.stop - s.start for s in sl]
        cells = int(np.prod(e))
        qo = q0 + sum(s * oa for s, oa in zip(slopes, o))
        lo = qo + sum(min(0, s * (ea - 1)) for s, ea in zip(slopes, e))
        hi = qo + sum(max(0, s * (ea - 1)) for s, ea in zip(slopes, e))
        bmean = _rm_frac(qo + sum(Fr(s * (ea - 1), 2) for s, ea in zip(slopes, e)))
        assert (st[b]["qo"], st[b]["min"], st[b]["max"]) == (qo, lo, hi)
        assert cand[b, 2] == bmean and cand[b, 4] == _rm_frac(Fr(lo + hi, 2))
        if one_sign:
            mad = cells * sum(Fr(abs(s) * (ea - 1), 2) for s, ea in zip(slopes, e))
            assert st[b]["mad"] == mad
            assert f[b, 17] == cl(Fr(mad) / (cells * R))
        assert f[b, 15] == cl(Fr(qo - lo, R)) and f[b, 16] == cl(Fr(hi - qo, R))
        assert f[b, 10] == cl(Fr(hi - lo, R))
        assert f[b, 11] == cl(Fr(bmean - gmean, R))
        for a in range(d):
            ea_mean = _rm_frac(qo + sum(Fr(s * (eb - 1), 2) for k, (s, eb) in enumerate(zip(slopes, e)) if k != a))
            assert f[b, 12 + a] == cl(Fr(ea_mean - bmean, R)), (b, a)
        for a in range(d, 3):
            assert f[b, 12 + a] == 0 and f[b, 18 + a] == 0
        # origin residual against each candidate: zero, global mean, block mean,
        # edge-mean effective value (pinned against the codec oracle above), midrange
        for c, P in enumerate([0, gmean, bmean, int(cand[b, 3]), _rm_frac(Fr(lo + hi, 2))]):
            assert f[b, c] == cl(Fr(qo - P, R)), (b, c)
            assert f[b, 5 + c] == cl(Fr(abs(qo - P), R)), (b, c)
        assert f[b, 21] == cl(Fr(gmean, 64 * R))


# ------------------------------------------------- the network's forward passes

def _sparse_theta(entries):
    P = {name: np.zeros(shp) for name, shp in S.param_layout()}
    for (name, idx), v in entries.items():
        P[name][idx] = v
    return S.pack(P)


def test_forward_worked_network():
    """A hand-built network: hidden-1 unit 0 reads feature 3 with weight 2 and
    bias -1; hidden-2 unit 5 reads hidden-1 unit 0 with weight 3; logit 6 reads
    hidden-2 unit 5; logit 2 is the bias 0.5. Weights are stored (out, in)."""
    theta = _sparse_theta({("W1", (0, 3)): 2.0, ("b1", 0): -1.0, ("W2", (5, 0)): 3.0,
                           ("W3", (6, 5)): 1.0, ("b3", 2): 0.5})
    X = np.zeros((4, S.N_FEAT))
    X[0, 3] = 4.0      # a1 = 7, h2 = 21
    X[1, 3] = 0.0      # a1 = -1: ReLU gives 0
    X[2, 4] = 100.0    # another feature: no path to the logits
    X[3, 3] = 129.0    # a1 = 257: a bfloat16 tie between 256 and 258
    z, _ = S.forward(theta, X)
    want = np.zeros((4, S.N_OUT))
    want[:, 2] = 0.5
    want[0, 6] = 21.0
    want[3, 6] = 771.0
    assert np.array_equal(z, want)
    zb = S.forward_bf16(theta, X)
    want[3, 6] = 768.0  # 257 rounds to the even neighbour 256, times 3
    assert np.array_equal(zb, want)
    assert np.array_equal(S.forward_bf16_f32(theta, X), want.astype(np.float32))


def test_forward_bf16_equals_forward_when_every_value_is_representable():
    """Integer inputs and sparse integer weights keep every activation an
    integer below 256, which bfloat16 holds exactly: the bf16 forward (fp64
    sums) and the fp32-accumulating one then equal the exact forward."""
    rng = np.random.default_rng(11)
    P = {}
    for name, shp in S.param_layout():
        if name.startswith("W"):
            w = np.zeros(shp)
            fan = 3 if name == "W1" else 4
            for r in range(shp[0]):
                cols = rng.choice(shp[1], fan, replace=False)
                w[r, cols] = rng.choice([-1.0, 1.0, 2.0], fan)
            P[name] = w
        else:
            P[name] = rng.integers(-3, 4, shp).astype(np.float64)
    theta = S.pack(P)
    X = rng.integers(0, 4, (500, S.N_FEAT)).astype(np.float64)
    z, (_, a1, h1, a2, h2) = S.forward(theta, X)
    assert np.abs(h1).max() < 256 and np.abs(h2).max() < 256 and h2.max() > 0
    assert np.array_equal(S.forward_bf16(theta, X), z)
    assert np.array_equal(S.forward_bf16_f32(theta, X).astype(np.float64), z)


def test_forward_bf16_f32_sums_in_order_in_fp32():
    """The fp32 accumulation starts from the bias and adds the products in
    input order: 1 + 2^24 rounds to 2^24 (a tie, to even), and - 2^24 then
    leaves 0, where the exact sum is 1."""
    theta = _sparse_theta({("b1", 0): 1.0, ("W1", (0, 0)): 1.0, ("W1", (0, 1)): -1.0,
                           ("W2", (0, 0)): 1.0, ("W3", (0, 0)): 1.0})
    X = np.zeros((1, S.N_FEAT))
    X[0, 0] = X[0, 1] = 2.0 ** 24
    assert S.forward_bf16(theta, X)[0, 0] == 1.0
    assert S.forward_bf16_f32(theta, X)[0, 0] == 0.0


def test_forward_bf16_f32_within_the_summation_bound():
    """On random networks the fp32-accumulating forward differs from the
    fp64-summing one only by rounding: with the same bf16 hidden activations
    (recomputed from the fp32 pass), each logit is within the recursive
    summation bound n u sum |terms| (u = 2^-24, n = 65 terms)."""
    rng = np.random.default_rng(12)
    theta = (S.init_params(4) + rng.normal(0, 0.05, S.n_params())).astype(np.float32)
    X = rng.normal(0, 2, (400, S.N_FEAT)).astype(np.float32)
    P = S.unpack(S.bf16_round(theta).astype(np.float64))
    x = S.bf16_round(X).astype(np.float64)
    h1 = S.bf16_round(np.maximum(S._f32_layer(x, P["W1"], P["b1"]), 0)).astype(np.float64)
    h2 = S.bf16_round(np.maximum(S._f32_layer(h1, P["W2"], P["b2"]), 0)).astype(np.float64)
    z32 = S.forward_bf16_f32(theta, X).astype(np.float64)
    exact = h2 @ P["W3"].T + P["b3"]
    bound = 65 * 2.0 ** -24 * (np.abs(h2) @ np.abs(P["W3"]).T + np.abs(P["b3"]))
    assert np.all(np.abs(z32 - exact) <= bound)
