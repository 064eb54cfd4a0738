"""Block-size and vector-width autotuner (the paper's Section III-E on the GPU).

The paper picks the block size and vector length of vecSZ by running the
dual-quantisation on a sample of blocks with every configuration, repeating
the test and keeping the fastest on average. Here the configurations are the
block edges the kernels support for the field's dimensionality and the cells
per lane (1, 2, 4; the `vec` hint), the sample is a contiguous slab of about
`frac` of the field along its slowest axis (whole blocks), and each
configuration is timed with HIP events around compress + decompress,
`iters` times after one warm-up. Only timing decides; every configuration
is exact. The block edge changes the compressed stream (not its accuracy).
"""

from __future__ import annotations

import numpy as np

from . import binding as dq

BLOCKS = {1: (256, 1024, 4096), 2: (8, 16, 32), 3: (4, 8, 16)}
VECS = (1, 2, 4)


def _sample(x, frac, B):
    n0 = x.shape[0]
    rows = max(B, int(round(n0 * frac / B)) * B)
    return x[:min(n0, rows)].contiguous()


def tune(x, eb, eb_mode="rel", pad="zero", radius=512, frac=0.1, iters=3, blocks=None, vecs=VECS):
    """Fastest (block, vec) for the field x (contiguous fp32 CUDA tensor);
    returns (block, vec, table of mean ms per configuration)."""
    import torch
    d = x.dim()
    eb_abs = float(eb)
    if eb_mode == "rel":  # the bound of the whole field (resolved by the codec), not of the sample
        c = dq.Codec(tuple(x.shape), eb, "rel", BLOCKS[d][0], "zero", radius, out_cap=0, device=x.device)
        c.compress_async(x)
        r = c.result()
        if r.status not in (dq.DQ_OK, dq.DQ_ECAPACITY):
            raise dq.DQError(r.status, "value range")
        eb_abs = float(r.eb_abs)
        del c
    table = {}
    for B in (blocks or BLOCKS[d]):
        xs = _sample(x, frac, B)
        for V in vecs:
            if xs.shape[-1] % V:
                continue
            try:
                cd = dq.Codec(tuple(xs.shape), eb_abs, "abs", B, pad, radius, out_cap=xs.numel(),
                              device=x.device, vec=V)
            except dq.DQError:
                continue
            ms = []
            for it in range(iters + 1):
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record()
                cd.compress_async(xs)
                cd.decompress_dev_async()
                ev1.record()
                ev1.synchronize()
                if it:
                    ms.append(ev0.elapsed_time(ev1))
            r = cd.result()
            if r.status != dq.DQ_OK:
                continue
            table[(B, V)] = float(np.mean(ms)) * x.numel() / xs.numel()  # scaled to the whole field
    best = min(table, key=table.get)
    return best[0], best[1], table


DEFAULT_BLOCK = {1: 1024, 2: 16, 3: 8}


def tune_batch(xs, ebs, eb_mode="rel", pad="zero", radius=512, frac=0.1, iters=3, margin=0.10):
    """One (block, vec) per dimensionality for a batch of fields: each field's
    configurations are timed as in tune() (scaled to the whole field) and the
    per-dimensionality sums decide, so the batch has one persistent kernel
    class per dimensionality. A configuration replaces the default block edge
    (its fastest width) only when it is faster by more than `margin`, so
    timing noise does not flip the choice from run to run. Returns
    {ndim: (block, vec)} and the per-field tables."""
    totals, tables = {}, []
    for x, eb in zip(xs, ebs):
        _, _, table = tune(x, eb, eb_mode, pad, radius, frac, iters)
        tables.append(table)
        acc = totals.setdefault(x.dim(), {})
        for cfg, ms in table.items():
            acc[cfg] = acc.get(cfg, 0.0) + ms
    best = {}
    for d, acc in totals.items():
        n_fields = sum(1 for x in xs if x.dim() == d)
        # configurations every field of the dimensionality could run
        full = [cfg for cfg in acc if sum(1 for x, t in zip(xs, tables) if x.dim() == d and cfg in t) == n_fields]
        cands = full or list(acc)
        pick = min(cands, key=acc.get)
        dflt = [c for c in cands if c[0] == DEFAULT_BLOCK[d]]
        if dflt:
            base = min(dflt, key=acc.get)
            if acc[pick] > (1.0 - margin) * acc[base]:
                pick = base
        best[d] = pick
    return best, tables
