"""GPU parity of the per-block padding / block-size selector against its oracle,
and what the trained network gains over zero padding."""

import numpy as np
import pytest

import gpu_util as G
from oracle import selector as S
from paper_2201_04614_amd import binding as dq
from paper_2201_04614_amd import fields as F
from paper_2201_04614_amd import selector as SEL

pytestmark = pytest.mark.gpu

CASES = [((203,), 8, 512), ((1000,), 64, 40), ((37, 41), 4, 64), ((64, 70), 16, 512), ((21, 18, 27), 4, 40),
         ((24, 20, 16), 8, 512), ((19, 33, 17), 16, 64), ((5, 7, 9), 2, 2)]


def _field(shape, seed):
    x = F.power_law_grf(shape, seed=seed) * np.float32(30.0) + np.float32(25.0)
    if len(shape) == 1 or min(shape) < 4:
        x = F.uniform_field(shape, seed=seed, lo=-40.0, hi=90.0)
    return np.ascontiguousarray(x, dtype=np.float32)


def _oracle_block_data(ref, x, eb, B, R, codes):
    p = ref.params(x.shape, eb, "abs", B, "zero", R)
    st, q = ref.prequantize(p, x, eb)
    assert st == ref.OK
    stats = S.block_stats(q, B)
    gmean = S.round_mean(int(q.astype(np.int64).sum()), q.size)
    cand = S.candidates(stats, gmean, x.ndim)
    flags = S.origin_outlier_flags(stats, cand, R)
    feat = S.features(stats, cand, gmean, R, x.ndim, B)
    return stats, cand, flags, S.pad_labels(flags), feat, S.nonorigin_outliers(codes, B)


@pytest.mark.parametrize("shape,B,R", CASES, ids=str)
def test_block_features_bit_exact(ref, shape, B, R):
    import torch
    x = _field(shape, sum(shape) + B)
    eb = 1e-2
    G.say(f"selector features {shape} B={B} R={R}")
    z = G.gpu_compress(x, eb, "abs", B, "zero", R)
    xd = torch.from_numpy(x).cuda()
    info = SEL.block_features(xd, eb, B, R, codes=z["codec"].codes)
    torch.cuda.synchronize()
    assert int(info.status.item()) == 0
    stats, cand, flags, lab, feat, nonorig = _oracle_block_data(ref, x, eb, B, R, z["codes"])
    gs = info.stats_host()
    for k in ("qo", "sum", "mad"):
        assert np.array_equal(gs[k].astype(np.int64), [s[k] for s in stats]), k
    assert np.array_equal(gs["mn"], [s["min"] for s in stats]) and np.array_equal(gs["mx"], [s["max"] for s in stats])
    assert np.array_equal(gs["fsum"], [s["fsum"] for s in stats])
    assert np.array_equal(gs["rough"], [s["rough"] for s in stats])
    assert np.array_equal(gs["nonorig"], nonorig)
    assert np.array_equal(info.cand.cpu().numpy(), cand)
    gf = info.flags.cpu().numpy()
    assert np.array_equal(np.stack([(gf >> c) & 1 for c in range(S.N_PAD)], 1).astype(bool), flags)
    assert np.array_equal(info.label.cpu().numpy(), lab)
    assert np.array_equal(info.feat.cpu().numpy().view(np.uint32), feat.view(np.uint32))
    # the chosen candidates compress (given mode) to the predicted outlier count
    pads = SEL.gather_pads(info, info.label).cpu().numpy()
    assert np.array_equal(pads, cand[np.arange(len(stats)), lab])
    c = G.parity(ref, x, eb, "abs", B, "given", R, pads=pads)
    assert c.n_out == int(nonorig.sum() + flags[np.arange(len(stats)), lab].sum())


def test_super_block_costs(ref):
    import torch
    shape, R, eb = (40, 36, 33), 64, 1e-2
    x = _field(shape, 6)
    xd = torch.from_numpy(x).cuda()
    per_b = []
    gpu_costs = []
    for B in S.BSIZES:
        z = G.gpu_compress(x, eb, "abs", B, "zero", R)
        info = SEL.block_features(xd, eb, B, R, codes=z["codec"].codes)
        gpu_costs.append(SEL.super_cost(shape, B, info, info.label).cpu().numpy())
        stats, cand, flags, lab, feat, nonorig = _oracle_block_data(ref, x, eb, B, R, z["codes"])
        per_b.append(nonorig + flags[np.arange(len(stats)), lab])
    lab, cost = S.block_size_labels(shape, per_b)
    assert np.array_equal(np.stack(gpu_costs), cost)
    srch = SEL.exhaustive_search(xd, eb, "abs", R)
    assert np.array_equal(srch.super_label.cpu().numpy(), lab)
    assert np.array_equal(srch.super_cost.cpu().numpy(), cost)


@pytest.mark.parametrize("n", [1, 31, 32, 100, 4099])
def test_mlp_gradient_and_adam(n):
    import torch
    rng = np.random.default_rng(n)
    theta = (S.init_params(2) * 0.7 + rng.normal(0, 0.02, S.n_params())).astype(np.float32)
    X = rng.normal(0, 1, (n, S.N_FEAT)).astype(np.float32)
    yp = rng.integers(0, S.N_PAD, n).astype(np.int32)
    yb = rng.integers(0, S.N_BSZ, n).astype(np.int32)
    G.say(f"mlp grad n={n}")
    td = torch.from_numpy(theta).cuda()
    g, loss, _ = SEL.mlp_grad(td, torch.from_numpy(X).cuda(), torch.from_numpy(yp).cuda(), torch.from_numpy(yb).cuda())
    want = S.grad(theta.astype(np.float64), X.astype(np.float64), yp, yb)
    got = g.cpu().numpy().astype(np.float64)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 2e-5 * scale + 1e-7, np.abs(got - want).max() / scale
    wl = S.loss(theta.astype(np.float64), X.astype(np.float64), yp, yb)
    assert abs(float(loss.item()) - wl) <= 1e-5 * abs(wl)
    # one Adam step from zero moments
    m = torch.zeros_like(td)
    v = torch.zeros_like(td)
    SEL.mlp_adam(td, m, v, g, 1, 1e-3)
    th2, _, _ = S.adam_step(theta.astype(np.float64), 0.0, 0.0, got, 1, 1e-3)
    assert np.allclose(td.cpu().numpy(), th2, rtol=0, atol=2e-6)


def test_bf16_inference():
    """bf16 parameters, inputs and activations with fp32 accumulation: the
    logits equal the oracle's fp32-order forward bit for bit, and both heads'
    choices equal its argmax on every sample."""
    import torch
    rng = np.random.default_rng(5)
    theta = (S.init_params(3) + rng.normal(0, 0.05, S.n_params())).astype(np.float32)
    X = rng.normal(0, 2, (3000, S.N_FEAT)).astype(np.float32)
    tb = SEL.to_bf16(torch.from_numpy(theta).cuda())
    assert np.array_equal(tb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16,
                          S.bf16_round(theta).view(np.uint32))
    pc, bc, lg = SEL.infer(tb, torch.from_numpy(X).cuda(), logits=True)
    want = S.forward_bf16_f32(theta, X)
    got = lg.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), np.abs(got - want).max()
    assert np.array_equal(pc.cpu().numpy(), np.argmax(want[:, :S.N_PAD], axis=1))
    assert np.array_equal(bc.cpu().numpy(), np.argmax(want[:, S.N_PAD:], axis=1))


def _training_fields(n, shape, seed):
    """Seeded fields where the padding matters: k^-2..k^-4 backgrounds with
    offsets of up to a few ranges and large-scale ramps (with radius 64 a
    single global value cannot predict every origin)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        slope = float(rng.uniform(2.0, 4.0))
        x = F.power_law_grf(shape, slope=slope, seed=int(seed * 1000 + i)).astype(np.float64)
        ramp = rng.normal(0, 1.0, size=3)
        g = np.meshgrid(*[np.linspace(-1, 1, s) for s in shape], indexing="ij")
        x += sum(r * gi for r, gi in zip(ramp, g)) * float(rng.uniform(0, 12))
        x += float(rng.choice([0.0, 0.5, 2.0, 5.0])) * (x.max() - x.min())
        out.append((x.astype(np.float32), float(10 ** rng.uniform(-3, -2))))
    return out


def test_learned_padding_gain(ref):
    """Trained on exhaustive labels of generated fields, the network's pads
    keep >= 95 % of the exhaustive search's outlier reduction over zero padding
    on held-out fields, and decode exactly (given mode)."""
    import torch
    R, B = 64, 8
    Xs, yps, ybs = [], [], []
    G.say("selector: labels of 48 training fields 64^3")
    for x, eb in _training_fields(48, (64, 64, 64), 1):
        s = SEL.exhaustive_search(torch.from_numpy(x).cuda(), eb, "rel", R, base=B)
        Xs.append(s.info.feat)
        yps.append(s.info.label)
        ybs.append(s.sample_bsz)
    X = torch.cat(Xs)
    yp = torch.cat(yps)
    yb = torch.cat(ybs)
    G.say(f"selector: training on {X.shape[0]} blocks")
    theta = SEL.train(X, yp, yb, epochs=30, batch=2048, lr=3e-3)
    tb = SEL.to_bf16(theta)
    zero_tot = best_tot = learned_tot = 0
    for i, (x, eb) in enumerate(_training_fields(6, (48, 40, 56), 2)):
        xd = torch.from_numpy(x).cuda()
        s = SEL.exhaustive_search(xd, eb, "rel", R, base=B)
        pads, pc, bc = SEL.learned_pads(tb, s.info)
        pads_h = pads.cpu().numpy()
        G.say(f"selector: held-out field {i}")
        c = G.parity(ref, x, s.eb_abs, "abs", B, "given", R, pads=pads_h)
        zero_tot += s.zero_out
        best_tot += s.best_out
        learned_tot += c.n_out
    G.say(f"selector: zero {zero_tot} exhaustive {best_tot} learned {learned_tot} labels {np.bincount(yp.cpu().numpy(), minlength=5)}")
    assert best_tot < zero_tot
    assert (yp != 0).float().mean() > 0.2 and (yp > 1).float().mean() > 0.02  # not a one-candidate problem
    assert zero_tot - learned_tot >= 0.95 * (zero_tot - best_tot)
