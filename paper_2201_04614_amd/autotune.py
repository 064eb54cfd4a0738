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
    if eb_mode == "rel":  # the bound of the whole field, not of the sample
        eb_abs = float(eb) * float(x.max() - x.min())
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
