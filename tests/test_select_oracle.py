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
