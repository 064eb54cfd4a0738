"""Side-information budget of the padding modes (Section IV, results in V-I).

For each synthetic field and every padding mode, compress on the GPU and
report the outlier count, the bytes of stored padding values and the net
side bytes (8 per outlier - uint32 index + int32 residual - plus the pads),
next to zero padding on the same field and bound:

    python -m paper_2201_04614_amd.padreport [--json]

Fields (seeded, the shapes of the measured workloads):
  c1         512 x 512 sum of 8 sinusoids + noise, abs eb 1e-4 * range, 16^2 blocks
  c2         256^3 k^-3 Gaussian random field, rel eb 1e-3, 8^3 blocks
  c2-offset  the same field + 2 * range (few near-zero values), 8^3 blocks
  c2-b4/b16  c2-offset with 4^3 and 16^3 blocks
"""

from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import binding as dq
from . import fields as F

MODES = ["zero", "global_mean", "global_min", "global_max", "block_mean", "block_min", "block_max",
         "edge_mean"]


def _fields():
    c1 = F.sinusoid_field((512, 512), seed=1)
    c2 = F.power_law_grf((256, 256, 256), slope=3.0, seed=2).astype(np.float32)
    c2o = c2 + np.float32(2.0 * F.field_range(c2))
    return [
        ("c1", c1, 1e-4 * F.field_range(c1), "abs", 16),
        ("c2", c2, 1e-3, "rel", 8),
        ("c2-offset", c2o, 1e-3, "rel", 8),
        ("c2-offset-b4", c2o, 1e-3, "rel", 4),
        ("c2-offset-b16", c2o, 1e-3, "rel", 16),
    ]


def report(radius=512):
    import torch

    rows = []
    for name, x, eb, mode, B in _fields():
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        base = None
        for pad in MODES:
            codec = dq.Codec(x.shape, eb, mode, B, pad, radius, out_cap=x.size)
            codec.compress_async(xd)
            r = codec.result()
            if r.status != dq.DQ_OK:
                raise dq.DQError(r.status, f"{name} {pad}")
            n_out = int(r.n_out)
            pad_bytes = 4 * dq.pad_count(codec.p)
            side = 8 * n_out + pad_bytes
            if base is None:
                base = (n_out, side)
            rows.append(dict(field=name, shape=list(x.shape), block=B, pad=pad, n_out=n_out,
                             outlier_pct=100.0 * n_out / x.size, pad_bytes=pad_bytes, side_bytes=side,
                             outliers_saved=base[0] - n_out, side_bytes_saved=base[1] - side))
            del codec
        del xd
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--json", action="store_true", help="one JSON object per line")
    ap.add_argument("--radius", type=int, default=512)
    args = ap.parse_args(argv)
    rows = report(args.radius)
    if args.json:
        for r in rows:
            print(json.dumps(r))
        return 0
    print(f"{'field':14s} {'B':>3s} {'pad':12s} {'outliers':>10s} {'%':>8s} {'pad B':>9s} "
          f"{'side B':>10s} {'saved out':>10s} {'saved B':>10s}")
    for r in rows:
        print(f"{r['field']:14s} {r['block']:3d} {r['pad']:12s} {r['n_out']:10d} {r['outlier_pct']:8.4f} "
              f"{r['pad_bytes']:9d} {r['side_bytes']:10d} {r['outliers_saved']:10d} {r['side_bytes_saved']:10d}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
