"""Learned padding / block-size selection against the exhaustive search and
plain zero padding, on one GPU:

    python -m paper_2201_04614_amd.selector_eval [--train 2000] [--eval-shape 512 512 512]

Training data: seeded 64^3 fields synthesised on the device - k^-2..k^-4
Gaussian random backgrounds, up to five planar steps and five spherical
shocks, large-scale ramps and offsets of up to five value ranges (the
offsets are what make zero padding fail at block origins, Section IV; the
ramps make a single global value fail where the q range exceeds the radius),
relative bounds 1e-4..1e-2 and radii 32..512, labelled by the exhaustive
search at block edges 4, 8 and 16 (every block is a sample; the block-size
label is its 16^3 super-block's). The network is trained with libdq's
kernels (fp32, Adam) and evaluated in bf16 on held-out 512^3 fields.
Printed: per field and block edge the
outliers of zero padding, of the exhaustive per-block choice and of the
learned choice (encoded with the given-pads mode), the share of the
exhaustive reduction the network keeps, the block-size head's agreement with
the exhaustive super-block labels, and the GPU time of the exhaustive search
and of the learned selection.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import binding as dq
from . import fields as F
from . import selector as SEL


def _field(shape, seed, device="cuda", planes=None, ramp_amp=None, offset=None):
    """A seeded training / test field, its relative bound and radius."""
    import torch
    rng = np.random.default_rng([seed, 0xF1E1D])
    k = int(rng.integers(0, 6)) if planes is None else planes
    x = F.sharp_feature_field_device(shape, seed=seed, n_planes=k, n_spheres=k,
                                     slope=float(rng.uniform(2.0, 4.0)), device=device)
    g = [torch.linspace(-1.0, 1.0, s, device=device) for s in shape]
    amp = float(rng.uniform(0, 20)) if ramp_amp is None else ramp_amp
    ramp = rng.normal(0, 1.0, size=3) * amp
    x += float(ramp[0]) * g[0][:, None, None] + float(ramp[1]) * g[1][None, :, None] + float(ramp[2]) * g[2][None, None, :]
    rng_x = float(x.max() - x.min())
    x += (float(rng.choice([0.0, 0.5, 2.0, 5.0])) if offset is None else offset) * rng_x
    eb = float(10 ** rng.uniform(-4.0, -2.0))
    R = int(rng.choice([32, 64, 128, 256, 512]))
    return x.contiguous(), eb, R


def _sync():
    import torch
    torch.cuda.synchronize()


def collect(n_fields, shape, seed0=1000, log=None):
    import torch
    X, yp, yb = [], [], []
    for i in range(n_fields):
        x, eb, R = _field(shape, seed0 + i)
        s = SEL.exhaustive_search(x, eb, "rel", R)
        for B in SEL.BSIZES:
            X.append(s.infos[B].feat)
            yp.append(s.infos[B].label)
            yb.append(s.sample_bszs[B])
        if log and (i + 1) % 250 == 0:
            log(f"labelled {i + 1} fields")
    return torch.cat(X), torch.cat(yp), torch.cat(yb)


def evaluate(theta_bf16, x, eb_rel, radius, name, base=8, log=None):
    """Zero / exhaustive / learned outliers per block edge; the block-size
    head's per-super-block choice priced with the exhaustive cost table."""
    import torch
    shape = tuple(x.shape)
    eb_abs = SEL.resolve_eb(x, eb_rel, "rel")
    _sync()
    t0 = time.perf_counter()
    s = SEL.exhaustive_search(x, eb_abs, "abs", radius, base=base)
    _sync()
    t_search = time.perf_counter() - t0
    rows = []
    for B in SEL.BSIZES:
        _sync()
        t0 = time.perf_counter()
        info = SEL.block_features(x, eb_abs, B, radius)
        pads, pc, bc = SEL.learned_pads(theta_bf16, info)
        _sync()
        t_learned = time.perf_counter() - t0
        codec = dq.Codec(shape, eb_abs, "abs", B, "given", radius, out_cap=x.numel() // 4, device=x.device)
        codec.pads[:pads.numel()].copy_(pads)
        codec.compress_async(x)
        r = codec.result()
        assert r.status == dq.DQ_OK, dq.strerror(r.status)
        learned = int(r.n_out)
        red_ex = s.zero_outs[B] - s.best_outs[B]
        rows.append(dict(field=name, block=B, zero=s.zero_outs[B], exhaustive=s.best_outs[B], learned=learned,
                         kept=(s.zero_outs[B] - learned) / red_ex if red_ex else 1.0,
                         learned_select_ms=1e3 * t_learned))
        if log:
            log(json.dumps(rows[-1]))
        del codec, info
    # block-size head at the base edge: its logits summed over each super-block's blocks
    info = s.infos[base]
    _, _, lg = SEL.infer(theta_bf16, info.feat, logits=True)
    sb = SEL._super_of_blocks(shape, base, x.device)
    agg = torch.zeros((s.super_cost.shape[1], 3), device=x.device).index_add_(0, sb, lg[:, 5:])
    pred = torch.argmax(agg, dim=1)
    cols = torch.arange(s.super_cost.shape[1], device=x.device)
    summ = dict(field=name, search_ms=1e3 * t_search,
                side_bytes_fixed_edge={B: int(s.super_cost[i].sum()) for i, B in enumerate(SEL.BSIZES)},
                side_bytes_exhaustive_per_super_block=int(s.super_cost.min(dim=0).values.sum()),
                side_bytes_learned_per_super_block=int(s.super_cost[pred, cols].sum()),
                bsz_head_agreement=float((pred == s.super_label).float().mean()),
                exhaustive_edge_share={B: float((s.super_label == i).float().mean())
                                       for i, B in enumerate(SEL.BSIZES)})
    if log:
        log(json.dumps(summ))
    return rows, summ


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--train", type=int, default=2000, help="64^3 training fields")
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--eval-shape", type=int, nargs=3, default=[512, 512, 512])
    args = ap.parse_args(argv)

    def log(m):
        print(m, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    X, yp, yb = collect(args.train, (64, 64, 64), log=log)
    _sync()
    t_label = time.perf_counter() - t0
    log(f"{X.shape[0]} samples labelled in {t_label:.1f} s; pad labels "
        f"{torch.bincount(yp, minlength=5).tolist()}, block labels {torch.bincount(yb, minlength=3).tolist()}")
    t0 = time.perf_counter()
    theta = SEL.train(X, yp, yb, epochs=args.epochs, batch=4096, lr=2e-3, log=log)
    _sync()
    t_train = time.perf_counter() - t0
    tb = SEL.to_bf16(theta)
    del X, yp, yb
    shape = tuple(args.eval_shape)
    results, summary = [], []
    # held-out fields: a k^-3 background with a ramp and an offset, radius 64,
    # relative bound 1e-3; the sharp-feature field (25 planar steps, 25
    # spherical shocks) at 1e-4 of its range and radius 512
    tests = (("grf-ramp-offset-R64", dict(seed=7, planes=0, ramp_amp=8.0, offset=2.0), 1e-3, 64),
             ("sharp-features-R512", dict(seed=5, planes=25, ramp_amp=0.0, offset=0.0), 1e-4, 512))
    for name, kw, eb_rel, R in tests:
        x, _, _ = _field(shape, **kw)
        rows, summ = evaluate(tb, x, eb_rel, R, name, log=log)
        results += rows
        summary.append(summ)
        del x
    out = dict(train_fields=args.train, train_samples_per_field=sum((64 // b) ** 3 for b in SEL.BSIZES),
               label_s=t_label, train_s=t_train, results=results, block_size_search=summary)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
