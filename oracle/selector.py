"""Oracle of the per-block padding / block-size selector (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke check and the CPU baseline of the benchmark may import
this module; the product path never does.

The paper chooses padding values from statistics of the data (Section IV-A:
mean, minimum, maximum; Section IV-B: per field, per block or per block and
axis) and tunes the block size by searching the configurations (Section
III-E autotuning). This module states, plainly and slowly, what the GPU
selector computes:

* block statistics of the pre-quantised field q (integers, exact);
* five candidate padding values per block and, by pad locality (a constant
  halo only enters the residual of the block origin, where it equals
  q_o - P_eff), whether each candidate leaves the origin an outlier;
* the exhaustive labels: the first candidate that keeps the origin
  predictable, and per 16^d super-block the block size in {4, 8, 16} with the
  lowest side cost (8 bytes per outlier + 4 bytes per stored pad);
* 24 features per block, each an fp64 expression of exact integers rounded
  once to fp32, so a GPU implementation can match them bit for bit;
* the MLP 24 -> 64 -> 64 -> 8 (ReLU; a 5-way padding head and a 3-way block
  size head, softmax cross-entropy each), its gradients and one Adam step,
  in fp64; its bfloat16 inference with fp64 sums and with fp32 accumulation
  in input order.

Pins (tests/test_select_oracle.py): statistics, candidates, flags, labels
and all 24 features of two hand-worked fields (tests/golden); closed forms of
every statistic and feature on integer-affine fields, partial blocks
included; candidates and flags against the codec oracle's pads and the origin
codes of real compressions; super-block costs against real outlier counts;
the forward passes on a hand-built network (bfloat16 ties, ReLU, the (out, in)
weight layout), exact agreement of the bf16 forwards with the exact one where
every value is representable, the fp32 accumulation order on a hand-worked
cancellation and within the recursive-summation bound; the gradients against
central finite differences; the first Adam step in closed form.
"""

from __future__ import annotations

import itertools
import math

import numpy as np

N_FEAT = 24
N_HID = 64
N_PAD = 5      # zero, global mean, block mean, edge-mean effective value, block midrange
N_BSZ = 3      # block edge 4, 8, 16
N_OUT = N_PAD + N_BSZ
SUPER = 16     # super-block edge of the block-size choice
BSIZES = (4, 8, 16)
CLAMP = 8.0


def round_mean(S, n):
    """Nearest integer to S / n (n > 0), halves toward +infinity."""
    return (2 * int(S) + int(n)) // (2 * int(n))


def wrap32(v):
    return ((int(v) + 2 ** 31) % 2 ** 32) - 2 ** 31


def _block_slices(shape, B):
    grids = [range(0, n, B) for n in shape]
    for origin in itertools.product(*grids):
        yield tuple(slice(o, min(o + B, n)) for o, n in zip(origin, shape))


def block_stats(q, B):
    """Per block (row-major block order): dict of exact integer statistics."""
    q = np.asarray(q, dtype=np.int64)
    d = q.ndim
    out = []
    for sl in _block_slices(q.shape, B):
        blk = q[sl]
        qo = int(blk[(0,) * d])
        st = dict(cells=int(blk.size), qo=qo, sum=int(blk.sum()), min=int(blk.min()), max=int(blk.max()),
                  mad=int(np.abs(blk - qo).sum()))
        fs, fc, rough, npairs = [], [], [], []
        for a in range(3):
            if a < d:
                face = np.take(blk, 0, axis=a)
                fs.append(int(face.sum()))
                fc.append(int(face.size))
                df = np.diff(blk, axis=a)
                rough.append(int(np.abs(df).sum()))
                npairs.append(int(df.size))
            else:
                fs.append(0)
                fc.append(0)
                rough.append(0)
                npairs.append(0)
        st.update(fsum=fs, fcnt=fc, rough=rough, npairs=npairs)
        out.append(st)
    return out


def edge_effective(e):
    """Effective padding at the origin for per-axis values e (the halo cell in
    front along the axis set S takes e_a for |S| = 1, else the rounded mean
    of the e_a, a in S); inclusion-exclusion over the corners."""
    d = len(e)
    P = 0
    for m in range(1, d + 1):
        for S in itertools.combinations(range(d), m):
            h = e[S[0]] if m == 1 else round_mean(sum(e[a] for a in S), m)
            P += (-1) ** (m + 1) * h
    return wrap32(P)


def candidates(stats, gmean, d):
    """Five candidate padding values of every block."""
    out = []
    for st in stats:
        e = [round_mean(st["fsum"][a], st["fcnt"][a]) for a in range(d)]
        out.append([0, gmean, round_mean(st["sum"], st["cells"]), edge_effective(e),
                    round_mean(st["min"] + st["max"], 2)])
    return np.array(out, dtype=np.int64)


def origin_outlier_flags(stats, cand, R):
    """flags[b, c]: the origin residual q_o - P_c (mod 2^32) is not in (-R, R)."""
    f = np.zeros(cand.shape, dtype=bool)
    for b, st in enumerate(stats):
        for c in range(cand.shape[1]):
            dl = wrap32(st["qo"] - int(cand[b, c]))
            f[b, c] = not (-R < dl < R)
    return f


def pad_labels(flags):
    """First candidate whose origin is predictable (0 if none is)."""
    lab = np.zeros(flags.shape[0], dtype=np.int64)
    for b in range(flags.shape[0]):
        ok = np.flatnonzero(~flags[b])
        lab[b] = ok[0] if ok.size else 0
    return lab


def _clampf(v):
    return np.float32(min(max(v, -CLAMP), CLAMP))


def features(stats, cand, gmean, R, d, B):
    """24 fp32 features per block (each one fp64 expression rounded once)."""
    F = np.zeros((len(stats), N_FEAT), dtype=np.float32)
    R = float(R)
    for b, st in enumerate(stats):
        qo, cells = st["qo"], st["cells"]
        bmean = round_mean(st["sum"], cells)
        f = [0.0] * N_FEAT
        for c in range(N_PAD):
            dl = wrap32(qo - int(cand[b, c]))
            f[c] = _clampf(dl / R)
            f[N_PAD + c] = _clampf(abs(dl) / R)
        f[10] = _clampf((st["max"] - st["min"]) / R)
        f[11] = _clampf((bmean - gmean) / R)
        for a in range(3):
            if a < d and st["fcnt"][a] > 0:
                f[12 + a] = _clampf((round_mean(st["fsum"][a], st["fcnt"][a]) - bmean) / R)
                if st["npairs"][a] > 0:
                    f[18 + a] = _clampf(st["rough"][a] / (st["npairs"][a] * R))
        f[15] = _clampf((qo - st["min"]) / R)
        f[16] = _clampf((st["max"] - qo) / R)
        f[17] = _clampf(st["mad"] / (cells * R))
        f[21] = _clampf(gmean / (64.0 * R))
        f[22] = np.float32(d / 3.0)
        f[23] = np.float32(math.log2(B) / 4.0)
        F[b] = np.array(f, dtype=np.float32)
    return F


def nonorigin_outliers(codes, B):
    """Per block: zero codes (outliers) away from the block origin."""
    codes = np.asarray(codes)
    d = codes.ndim
    out = []
    for sl in _block_slices(codes.shape, B):
        blk = codes[sl]
        z = int(np.count_nonzero(blk == 0))
        if blk[(0,) * d] == 0:
            z -= 1
        out.append(z)
    return np.array(out, dtype=np.int64)


def super_of_blocks(shape, B):
    """Super-block index (row-major over the 16^d super-block grid) of every block."""
    nsb = [(n + SUPER - 1) // SUPER for n in shape]
    out = []
    for sl in _block_slices(shape, B):
        c = [s.start // SUPER for s in sl]
        k = 0
        for a in range(len(shape)):
            k = k * nsb[a] + c[a]
        out.append(k)
    return np.array(out, dtype=np.int64)


def block_size_labels(shape, per_b):
    """per_b[i] = (block outliers under the best padding, per block) for
    B = BSIZES[i]; returns the label (index into BSIZES) per super-block:
    lowest 8 * outliers + 4 * blocks, ties to the larger block."""
    nsb = int(np.prod([(n + SUPER - 1) // SUPER for n in shape]))
    cost = np.zeros((N_BSZ, nsb), dtype=np.int64)
    for i, B in enumerate(BSIZES):
        sb = super_of_blocks(shape, B)
        np.add.at(cost[i], sb, 8 * per_b[i] + 4)
    lab = np.zeros(nsb, dtype=np.int64)
    for s in range(nsb):
        best = None
        for i in reversed(range(N_BSZ)):  # larger blocks first: ties keep them
            if best is None or cost[i, s] < cost[best, s]:
                best = i
        lab[s] = best
    return lab, cost


# ------------------------------------------------------------------ MLP

def param_layout():
    """(name, shape) of the parameters in their packed order."""
    return [("W1", (N_HID, N_FEAT)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
            ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]


def n_params():
    return sum(int(np.prod(s)) for _, s in param_layout())


def unpack(theta):
    out, k = {}, 0
    for name, shp in param_layout():
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[k:k + n], dtype=np.float64).reshape(shp)
        k += n
    return out


def pack(P):
    return np.concatenate([np.asarray(P[name], dtype=np.float64).reshape(-1) for name, _ in param_layout()])


def _log_softmax(z):
    m = z.max(axis=1, keepdims=True)
    return z - m - np.log(np.exp(z - m).sum(axis=1, keepdims=True))


def forward(theta, X):
    """Logits (n x 8) and the hidden activations."""
    P = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["W3"].T + P["b3"]
    return z, (X, a1, h1, a2, h2)


def loss(theta, X, y_pad, y_bsz):
    """Mean over samples of the two heads' cross-entropies."""
    z, _ = forward(theta, X)
    n = z.shape[0]
    lp = _log_softmax(z[:, :N_PAD])
    lb = _log_softmax(z[:, N_PAD:])
    return float(-(lp[np.arange(n), y_pad].sum() + lb[np.arange(n), y_bsz].sum()) / n)


def grad(theta, X, y_pad, y_bsz):
    """Gradient of loss() with respect to the packed parameters (backprop)."""
    P = unpack(theta)
    z, (X, a1, h1, a2, h2) = forward(theta, X)
    n = z.shape[0]
    dz = np.zeros_like(z)
    dz[:, :N_PAD] = np.exp(_log_softmax(z[:, :N_PAD]))
    dz[np.arange(n), y_pad] -= 1.0
    dz[:, N_PAD:] = np.exp(_log_softmax(z[:, N_PAD:]))
    dz[np.arange(n), N_PAD + np.asarray(y_bsz)] -= 1.0
    dz /= n
    G = {"W3": dz.T @ h2, "b3": dz.sum(axis=0)}
    d2 = (dz @ P["W3"]) * (a2 > 0)
    G["W2"], G["b2"] = d2.T @ h1, d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (a1 > 0)
    G["W1"], G["b1"] = d1.T @ X, d1.sum(axis=0)
    return pack(G)


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1), step t >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-uniform weights, zero biases (a seeded starting point)."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, shp in param_layout():
        if name.startswith("W"):
            lim = math.sqrt(6.0 / shp[1])
            P[name] = rng.uniform(-lim, lim, size=shp)
        else:
            P[name] = np.zeros(shp)
    return pack(P)


def bf16_round(a):
    """fp32 values rounded to bfloat16 (nearest, ties to even), as fp32."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def forward_bf16(theta, X):
    """Logits of the network with its parameters, inputs and hidden
    activations rounded to bfloat16, the products summed exactly (fp64)."""
    P = unpack(bf16_round(np.asarray(theta, dtype=np.float32)).astype(np.float64))
    x = bf16_round(np.asarray(X, dtype=np.float32)).astype(np.float64)
    h1 = bf16_round(np.maximum(x @ P["W1"].T + P["b1"], 0.0).astype(np.float32)).astype(np.float64)
    h2 = bf16_round(np.maximum(h1 @ P["W2"].T + P["b2"], 0.0).astype(np.float32)).astype(np.float64)
    return h2 @ P["W3"].T + P["b3"]


def _f32_layer(x, W, b):
    """One layer in fp32: each output starts from its bias and adds the
    products w_k x_k in input order k = 0, 1, ..., every addition rounded to
    fp32. x and W hold bfloat16 values, so every product is exact in fp32."""
    x = np.asarray(x, dtype=np.float32)
    W = np.asarray(W, dtype=np.float32)
    acc = np.broadcast_to(np.asarray(b, dtype=np.float32), (x.shape[0], W.shape[0])).copy()
    for k in range(W.shape[1]):
        acc = (acc + np.outer(x[:, k], W[:, k]).astype(np.float32)).astype(np.float32)
    return acc


def forward_bf16_f32(theta, X):
    """Logits of the bfloat16 network (parameters, inputs and hidden
    activations rounded to bfloat16, as forward_bf16) with fp32 accumulation:
    the reading of BF16 inference with FP32 accumulation in which each sum is
    taken in input order from the bias, one fp32 rounding per addition."""
    P = unpack(bf16_round(np.asarray(theta, dtype=np.float32)).astype(np.float64))
    x = bf16_round(np.asarray(X, dtype=np.float32))
    h1 = bf16_round(np.maximum(_f32_layer(x, P["W1"], P["b1"]), np.float32(0)))
    h2 = bf16_round(np.maximum(_f32_layer(h1, P["W2"], P["b2"]), np.float32(0)))
    return _f32_layer(h2, P["W3"], P["b3"])



def super_vote(shape, base, logits):
    """Edge index (0, 1, 2 for 4, 8, 16) of every super-block from the
    block-size logits (outputs 5, 6, 7) of the blocks at edge `base`: each
    super-block's logits summed in fp32 over its blocks in row-major order,
    the largest sum, ties to the larger edge."""
    logits = np.asarray(logits, dtype=np.float32)
    nb = [(n + base - 1) // base for n in shape]
    nsb = [(n + SUPER - 1) // SUPER for n in shape]
    per = SUPER // base
    out = []
    for sc in itertools.product(*[range(k) for k in nsb]):
        acc = np.zeros(3, dtype=np.float32)
        ranges = [range(c * per, min(nb[a], (c + 1) * per)) for a, c in enumerate(sc)]
        for bc in itertools.product(*ranges):
            b = 0
            for a in range(len(shape)):
                b = b * nb[a] + bc[a]
            acc = (acc + logits[b, N_PAD:N_OUT]).astype(np.float32)
        best = 2
        for i in (1, 0):
            if acc[i] > acc[best]:
                best = i
        out.append(best)
    return np.array(out, dtype=np.int64)
