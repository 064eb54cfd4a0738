"""Randomized parity sweep: seeded random shapes (1-D, 2-D, 3-D, ragged),
block edges, vector-width hints, padding modes, radii, absolute and relative
bounds, value distributions (uniform, power-law random fields, integers,
magnitudes from 1e-20 to 1e20) and outlier capacities (the cell count, which
gives every cell a staging slot; a sixteenth of it; the exact count, which
sends entries to the overflow list; one short, which must fail with
ECAPACITY); every output of the HIP path must equal the oracle's bit for bit
(codes, outliers, pads, bound, decoded floats, status)."""

import numpy as np
import pytest

import gpu_util as G
from paper_2201_04614_amd import binding as dq
from paper_2201_04614_amd import fields as F

pytestmark = pytest.mark.gpu

BLOCKS = {1: [1, 2, 8, 16, 64, 256, 1024, 4096], 2: [1, 2, 4, 8, 16, 32, 64, 128, 256],
          3: [1, 2, 4, 8, 16, 32, 64]}
PADS = ["zero", "block_mean", "edge_mean", "global_mean", "block_min", "block_max", "global_min", "global_max"]


def _case(rng):
    d = int(rng.integers(1, 4))
    B = int(rng.choice(BLOCKS[d]))
    if d == 1:
        shape = (int(rng.integers(1, 400000)),)
    elif d == 2:
        shape = tuple(int(v) for v in rng.integers(1, 700, size=2))
    else:
        shape = tuple(int(v) for v in rng.integers(1, 90, size=3))
    vec = int(rng.choice([0, 1, 2, 4]))
    pad = str(rng.choice(PADS))
    R = int(rng.choice([1, 2, 7, 64, 512, 32768]))
    kind = int(rng.integers(0, 4))
    seed = int(rng.integers(0, 1 << 30))
    if kind == 0:
        x = F.uniform_field(shape, seed, -float(rng.uniform(0.1, 1e4)), float(rng.uniform(0.1, 1e4)))
    elif kind == 1:
        x = F.power_law_grf(shape, slope=float(rng.uniform(2, 4)), seed=seed).astype(np.float32)
        x += np.float32(rng.uniform(-3, 3))
    elif kind == 2:
        x = F.integer_field(shape, seed, int(rng.integers(1, 100000)))
    else:
        x = F.uniform_field(shape, seed, -1.0, 1.0) * np.float32(10.0 ** rng.uniform(-20, 20))
    x = np.ascontiguousarray(x, dtype=np.float32)
    if rng.random() < 0.5:
        mode, eb = "rel", float(10.0 ** rng.uniform(-6, -1))
    else:
        span = float(np.max(x) - np.min(x))
        mode, eb = "abs", float(max(span, 1e-30) * 10.0 ** rng.uniform(-7, -1))
    return x, eb, mode, B, pad, R, vec, kind


def ref_count(ref, x, eb, mode, B, pad, R):
    c = ref.compress(ref.params(x.shape, eb, mode, B, pad, R), x)
    return c.status, int(c.n_out)


@pytest.mark.parametrize("seed", [101, 202, 303])
def test_random_configurations(ref, seed):
    rng = np.random.default_rng(seed)
    ran = 0
    for case in range(20):
        x, eb, mode, B, pad, R, vec, kind = _case(rng)
        if dq.validate(dq.make_params(x.shape, eb, mode, B, pad, R)) == dq.DQ_ENOTSUP:
            continue  # outside the GPU kernels' coverage (checked on the host)
        cap_kind = int(rng.integers(0, 4))
        cap = None
        if cap_kind:
            st, n_out = ref_count(ref, x, eb, mode, B, pad, R)
            if st == 0:
                cap = [max(n_out, x.size // 16), n_out, max(n_out - 1, 0)][cap_kind - 1]
        G.say(f"random seed={seed} case={case} shape={x.shape} B={B} vec={vec} pad={pad} R={R} "
              f"kind={kind} {mode} eb={eb:.3g} cap={cap}")
        G.parity(ref, x, eb, mode, B, pad, R, vec=vec, out_cap=cap)
        ran += 1
    assert ran >= 15
