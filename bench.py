"""Benchmark of the dual-quantisation hot path on one MI355X.

Default workload (one step): a batch of 64 fp32 fields of uneven shape
(1-D 2^20..2^24 cells, 2-D up to 1800 x 3600, 3-D up to 512^3; k^-2..k^-4
Gaussian random fields synthesised on the device, seed 3; relative bounds
1e-5..1e-2 per field, radius 512, zero padding), compressed and decompressed
by one graph launch - every stage of the path for every field: value-range
pass, prequantisation + Lorenzo + codes + outlier staging, outlier
placement, prefix-sum decode + dequantisation. Block edge and cells per lane
come from the autotuner, one configuration per dimensionality. Both batch
forms are timed (a graph replaying every field's own kernels, and the
persistent kernels draining a (field, tile) queue); the faster one gives the
step time. The line also carries the outlier counts of the 256^3 field per
padding mode and, on the 512 x 1024 x 1024 sharp-feature field, the learned
per-block padding against plain zero padding (--no-extras skips both).

--workload c2 / c1 / c5 measure one field at a time: the 256^3 k^-3 field
(rel eb 1e-3, 8^3 blocks, zero / block-mean / edge-mean padding), the 512^2
sinusoid field and the 512 x 1024 x 1024 sharp-feature field (abs eb 1e-4 *
range, zero padding); every call reads and writes its own buffers, rotating
over enough sets that the working set (> 1 GiB) cannot stay in the 256 MB
Infinity Cache.

Inputs are resident in HBM before the timed region. Prints one JSON line:
value = 4N bytes of fp32 input (every field, every padding mode) / step
time, the roofline of the dominant kernel (HIP events recorded around it on
its own stream, in a second pass of the same steps), and the CPU oracle
timed on bounded samples at one thread and on every host core.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# name -> shape, bound (factor, mode: "rel" or "abs" times the field range),
# block edge, padding modes, radius, rotating buffer sets, description
WORKLOADS = {
    "c2": dict(shape=(256, 256, 256), eb=1e-3, eb_mode="rel", block=8, radius=512, sets=4,
               pads=("zero", "block_mean", "edge_mean"),
               desc="256^3 fp32 k^-3 Gaussian random field (seed 2), rel eb 1e-3, 8^3 blocks, radius 512, "
                    "padding zero/block_mean/edge_mean; step = compress+decompress per mode"),
    "c1": dict(shape=(512, 512), eb=1e-4, eb_mode="abs", block=16, radius=512, sets=400, pads=("zero",),
               desc="512^2 fp32 sum of 8 sinusoids + N(0,1e-3) noise (seed 1), abs eb 1e-4*range, 16^2 blocks, "
                    "radius 512, zero padding; step = compress+decompress"),
    "c5": dict(shape=(512, 1024, 1024), eb=1e-4, eb_mode="abs", block=8, radius=512, sets=1, pads=("zero",),
               desc="512x1024x1024 fp32 k^-3 background + 25 planar steps + 25 spherical shocks (seed 5, "
                    "device synthesis), abs eb 1e-4*range, 8^3 blocks, radius 512, zero padding; "
                    "step = compress+decompress"),
    "c3": dict(batch=True, sets=1, pads=("zero",), radius=512,
               desc="64 fp32 fields of uneven shape (1-D 2^20..2^24, 2-D up to 1800x3600, 3-D up to 512^3; "
                    "k^-2..k^-4 Gaussian random fields, device synthesis, seed 3), rel eb 1e-5..1e-2 per field, "
                    "radius 512, zero padding, block edge and cells per lane per dimensionality from the autotuner; "
                    "step = one graph launch compressing and decompressing every field"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("dq_device.hpp", "dq_kernels.hpp", "dq_fastdiv.hpp", "dq_encode.hip", "dq_decode.hip", "dq_aux.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "encode_256cubed_traffic.txt")


def kernel_source_hash():
    """Hash of the kernel sources, to tell whether a stored counter reading
    still describes the kernels being timed."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2201_04614_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic():
    """HBM bytes per encode launch from the committed FETCH_SIZE / WRITE_SIZE
    reading, or None when it was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(reps=20):
    """A plain device copy of known size (256 MiB read, 256 MiB written):
    the reference that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 64 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": 4 * n, "reps": reps}), flush=True)


def cpu_baseline(x, W, eb_abs):
    """The oracle, as it stands, on a bounded sample of the same step: the
    whole field up to 2^24 cells, else a block-aligned sub-box of 2^24 cells
    (blocks are independent) with the bound of the full field."""
    from oracle import dqref
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    sample = "whole field"
    if x.size > (1 << 24):
        x = np.ascontiguousarray(x[: max(W["block"], (1 << 24) // (x.shape[1] * x.shape[2]))])
        sample = f"sub-box {x.shape[0]}x{x.shape[1]}x{x.shape[2]} of the field"
    n = x.size
    reps = max(1, int(2e6 // n))  # small fields: repeat to a measurable time
    t0 = time.perf_counter()
    for _ in range(reps):
        for pad in W["pads"]:
            if W["eb_mode"] == "rel" and sample == "whole field":
                p = dqref.params(x.shape, W["eb"], "rel", W["block"], pad, W["radius"])
            else:
                p = dqref.params(x.shape, eb_abs, "abs", W["block"], pad, W["radius"])
            c = dqref.compress(p, x, out_cap=n // 16, nthreads=threads)
            st, _ = dqref.decompress(p, c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads, nthreads=threads)
            assert c.status == 0 and st == 0
    dt = time.perf_counter() - t0
    npad = len(W["pads"])
    return {"value": round(reps * npad * 4.0 * n / dt / 1e9, 4), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} x ({sample}, {npad} padding mode(s), compress+decompress), {dt:.1f} s wall"}


def batch_specs(seed=3, n=64):
    """The uneven batch: field kinds in rotation, seeded shapes, spectra and bounds."""
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(n):
        kind = k % 3
        if kind == 0:
            shape = (int(2 ** rng.uniform(20, 24)),)
        elif kind == 1:
            shape = (int(rng.integers(256, 1801)), int(rng.integers(256, 3601)))
        else:
            shape = tuple(int(rng.integers(64, 513)) for _ in range(3))
        specs.append(dict(shape=shape, slope=float(rng.uniform(2.0, 4.0)), eb=float(10 ** rng.uniform(-5, -2)),
                          seed=1000 + k))
    return specs


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_batch(xs, specs, cfg, W, all_cells=1 << 28, one_cells=1 << 25):
    """The oracle, as it stands, on bounded samples of the batch: the first
    fields in batch order (all dimensionalities interleave) up to all_cells
    cells on every host core, up to one_cells cells on one thread; each field
    compressed and decompressed with its own bound, block and padding."""
    from oracle import dqref
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)

    def run(limit, nthreads):
        host, n = [], 0
        for x, s in zip(xs, specs):
            if host and n + x.numel() > limit:
                break
            host.append((x.cpu().numpy(), s))
            n += x.numel()
        t0 = time.perf_counter()
        for x, s in host:
            B, _ = cfg[x.ndim]
            p = dqref.params(x.shape, s["eb"], "rel", B, "zero", W["radius"])
            c = dqref.compress(p, x, out_cap=x.size, nthreads=nthreads)
            st, _ = dqref.decompress(p, c.eb_abs, c.codes, c.out_idx, c.out_val, c.pads, nthreads=nthreads)
            assert c.status == 0 and st == 0
        dt = time.perf_counter() - t0
        return round(4.0 * n / dt / 1e9, 4), f"first {len(host)} fields of the batch, {n} cells, {dt:.1f} s wall"

    v_all, s_all = run(all_cells, threads)
    v_one, s_one = run(one_cells, 1)
    return {"value": v_all, "unit": "GB/s", "cores": threads, "kind": "oracle", "sample": s_all,
            "cpu_model": cpu_model(),
            "single_thread": {"value": v_one, "unit": "GB/s", "cores": 1, "sample": s_one}}


BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batch_64fields_persistent_traffic.txt")


def stored_batch_traffic(kernel):
    """HBM bytes per launch of the named batch kernel (a line
    "traffic_bytes_per_launch[<kernel>]: <bytes>") from the committed counter
    reading, or None when it was taken on other kernel sources or does not
    cover that kernel."""
    try:
        with open(BATCH_TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv[f"traffic_bytes_per_launch[{kernel}]"])
    except (KeyError, ValueError):
        return None


def c2_outlier_counts(W):
    """Outliers per padding mode on the 256^3 k^-3 field (seed 2) and on the
    same field offset by two value ranges (rel eb 1e-3, 8^3 blocks, R 512)."""
    import torch
    from paper_2201_04614_amd import binding as dq
    from paper_2201_04614_amd import fields
    x = fields.power_law_grf((256, 256, 256), slope=3.0, seed=2)
    out = {}
    for name, xx in (("c2", x), ("c2_offset", (x + np.float32(2.0 * fields.field_range(x))).astype(np.float32))):
        xd = torch.from_numpy(np.ascontiguousarray(xx)).cuda()
        row = {}
        for pad in ("zero", "block_mean", "edge_mean", "global_mean"):
            cd = dq.Codec(xd.shape, 1e-3, "rel", 8, pad, 512, out_cap=xd.numel())
            cd.compress_async(xd)
            r = cd.result()
            assert r.status == dq.DQ_OK
            row[pad] = int(r.n_out)
        out[name] = row
    return out


def train_selector(n_train=2000, log=log):
    """The selector network trained on the GPU with libdq's kernels on the
    exhaustive labels of n_train generated 64^3 fields (bf16 for inference)."""
    import torch
    from paper_2201_04614_amd import selector as SEL
    from paper_2201_04614_amd import selector_eval as SE
    t0 = time.perf_counter()
    X, yp, yb = SE.collect(n_train, (64, 64, 64))
    theta = SEL.train(X, yp, yb, epochs=6, batch=4096, lr=2e-3)
    tb = SEL.to_bf16(theta)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del X, yp, yb
    log(f"bench: selector trained on {n_train} fields in {t_train:.1f} s")
    return tb, n_train, t_train


def c4_mixed_report(tb, log=log):
    """Held-out 512^3 fields, rel eb 1e-3: plain zero padding (8^3 blocks)
    against mixed-edge streams (an edge in {4, 8, 16} per 16^3 super-block
    and a padding per block) chosen by the exhaustive search and by the
    network; outliers, side bytes (8 per outlier + 4 per pad + 1 per edge),
    GPU times, and every mixed stream decoded and compared bit for bit with
    the zero-padding stream's x_hat (the same q, so the same floats)."""
    import torch
    from paper_2201_04614_amd import binding as dq
    from paper_2201_04614_amd import mixed as MX
    from paper_2201_04614_amd import selector as SEL
    from paper_2201_04614_amd import selector_eval as SE
    shape = (512, 512, 512)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def gpu_ms(f):
        torch.cuda.synchronize()
        ev[0].record()
        r = f()
        ev[1].record()
        torch.cuda.synchronize()
        return r, ev[0].elapsed_time(ev[1])

    out = []
    for name, kw, R in (("k^-3 + ramp + offset", dict(seed=7, planes=0, ramp_amp=8.0, offset=2.0), 64),
                        ("sharp features", dict(seed=5, planes=25, ramp_amp=0.0, offset=0.0), 32)):
        x, _, _ = SE._field(shape, **kw)
        eb = SEL.resolve_eb(x, 1e-3, "rel")
        n = x.numel()
        ns = MX.num_super(shape)
        zero = dq.Codec(shape, eb, "abs", 8, "zero", R, out_cap=n)
        zero.compress_async(x)
        zx = zero.decompress_dev_async()
        rz = zero.result()
        assert rz.status == dq.DQ_OK
        row = {"field": name, "radius": R, "eb_abs": eb,
               "zero_pad": {"outliers": int(rz.n_out), "side_bytes": 8 * int(rz.n_out)}}
        zero_side = 8 * int(rz.n_out)
        for kind in ("exhaustive", "learned"):
            if kind == "exhaustive":
                (edges, pads, off, _), ms_sel = gpu_ms(lambda: SEL.mixed_exhaustive(x, eb, "abs", R))
            else:
                (edges, pads, off), ms_sel = gpu_ms(lambda: SEL.mixed_learned(tb, x, eb, R))
            st, ms_c = gpu_ms(lambda: MX.compress(x, eb, R, edges, pads, pad_off=off))
            assert st.status == dq.DQ_OK
            xh, ms_d = gpu_ms(lambda: MX.decompress(st))
            n_pads = int(off[-1].item())
            side = 8 * st.n_out + 4 * n_pads + ns
            share = {int(E): round(float((edges == E).float().mean()), 4) for E in (4, 8, 16)}
            row[kind] = {"outliers": st.n_out, "pads": n_pads, "side_bytes": side, "edge_share": share,
                         "select_ms": round(ms_sel, 2), "compress_ms": round(ms_c, 3), "decompress_ms": round(ms_d, 3),
                         "decoded_equals_zero_pad_x_hat": bool(torch.equal(xh.view(torch.int32),
                                                                           zx.view(torch.int32)))}
            del st, xh, edges, pads, off
        ex_side = row["exhaustive"]["side_bytes"]
        red = zero_side - ex_side
        row["learned"]["share_of_exhaustive_side_byte_reduction"] = \
            round((zero_side - row["learned"]["side_bytes"]) / red, 4) if red else 1.0
        log(f"bench: c4 {name}: {json.dumps(row)}")
        out.append(row)
        del x, zero, zx
        torch.cuda.empty_cache()
    return out


def c5_selector_report(tb, n_train, t_train, log=log):
    """The 512 x 1024 x 1024 sharp-feature field (seed 5, eb 1e-4 * range,
    8^3 blocks, R 512): plain zero padding against the learned per-block
    padding (bf16 inference, given-pads stream), with the exhaustive
    search's outliers as the reference; GPU times of compress + decompress
    and of the learned selection."""
    import torch
    from paper_2201_04614_amd import binding as dq
    from paper_2201_04614_amd import fields
    from paper_2201_04614_amd import selector as SEL
    shape = (512, 1024, 1024)
    x = fields.sharp_feature_field_device(shape, seed=5)
    eb = 1e-4 * float(x.max().double() - x.min().double())
    n = x.numel()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def timed(cd, reps=5):
        ms = []
        for _ in range(reps + 1):
            ev[0].record()
            cd.compress_async(x)
            cd.decompress_dev_async()
            ev[1].record()
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
        r, rd = cd.result(), cd.decompress_result()
        assert r.status == dq.DQ_OK and rd.status == dq.DQ_OK
        return float(np.median(ms[1:])), int(r.n_out)

    zero = dq.Codec(shape, eb, "abs", 8, "zero", 512, out_cap=n // 8)
    ms_zero, out_zero = timed(zero)
    ev[2].record()
    info = SEL.block_features(x, eb, 8, 512)
    pads, _, _ = SEL.learned_pads(tb, info)
    ev[3].record()
    torch.cuda.synchronize()
    ms_select = ev[2].elapsed_time(ev[3])
    # the exhaustive reference: per block the zero-pad outliers away from the
    # origin plus the best candidate's origin (statistics given the zero-pad codes)
    info_ex = SEL.block_features(x, eb, 8, 512, codes=zero.codes)
    del zero
    learned = dq.Codec(shape, eb, "abs", 8, "given", 512, out_cap=n // 8)
    learned.pads[:pads.numel()].copy_(pads)
    ms_learned, out_learned = timed(learned)
    st = info_ex.stats_host()
    fl = info_ex.flags.cpu().numpy()
    lab = info_ex.label.cpu().numpy()
    out_best = int(st["nonorig"].astype(np.int64).sum() + ((fl >> lab) & 1).astype(np.int64).sum())
    del learned, info, info_ex, x
    torch.cuda.empty_cache()
    red = out_zero - out_best
    return {"workload": "512x1024x1024 sharp features (seed 5), eb 1e-4*range, 8^3 blocks, R 512",
            "zero_pad": {"outliers": out_zero, "outlier_pct": round(100.0 * out_zero / n, 4),
                         "ms": round(ms_zero, 4), "GBps": round(4.0 * n / (ms_zero * 1e-3) / 1e9, 1)},
            "learned_pad": {"outliers": out_learned, "outlier_pct": round(100.0 * out_learned / n, 4),
                            "ms": round(ms_learned, 4), "GBps": round(4.0 * n / (ms_learned * 1e-3) / 1e9, 1),
                            "select_ms": round(ms_select, 4),
                            "share_of_exhaustive_reduction": round((out_zero - out_learned) / red, 4) if red else 1.0},
            "exhaustive_pad_outliers": out_best, "train_fields": n_train, "train_s": round(t_train, 1)}


def run_batch(args, W):
    """The batched workload: one step = one graph launch compressing and
    decompressing every field (the persistent form when faster)."""
    import torch
    from paper_2201_04614_amd import autotune as AT
    from paper_2201_04614_amd import batch as BT
    from paper_2201_04614_amd import fields

    specs = batch_specs()
    log(f"bench: synthesising {len(specs)} fields")
    xs = []
    for k, s in enumerate(specs):
        xs.append(fields.power_law_grf_device(s["shape"], s["slope"], s["seed"]))
        if k % 16 == 15:
            torch.cuda.synchronize()
            log(f"bench: {k + 1} fields synthesised")
    N = sum(x.numel() for x in xs)
    torch.cuda.synchronize()
    log(f"bench: {N} cells; autotuning block edge and vector width per dimensionality")
    t0 = time.perf_counter()
    if args.batch_config:
        cfg = {int(d): (int(b), int(v)) for d, b, v in (c.split(":") for c in args.batch_config.split(","))}
    else:
        cfg, _ = AT.tune_batch(xs, [s["eb"] for s in specs], "rel", frac=0.1, iters=3)
    t_tune = time.perf_counter() - t0
    log(f"bench: tuned {cfg} in {t_tune:.1f} s")

    def items(c):
        return [(x, dict(eb=s["eb"], eb_mode="rel", block=c[x.dim()][0], pad="zero", radius=W["radius"],
                         out_cap=x.numel(), vec=c[x.dim()][1])) for x, s in zip(xs, specs)]

    def time_graph(b, steps, warmup):
        for _ in range(max(1, warmup)):
            b.launch()
        torch.cuda.synchronize()
        bad = [(i, r.status, rd.status) for i, (r, rd) in enumerate(b.results()) if r.status or rd.status]
        assert not bad, bad
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            b.launch()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # the graph of per-field launches
    b = BT.Batch(items(cfg), branches=4)
    ms_graph = time_graph(b, args.steps, args.warmup)
    per_out = [int(r.n_out) for r, _ in b.results()]
    b.close()
    del b
    torch.cuda.empty_cache()
    # the persistent form, with events around the largest class's kernels
    pb = BT.PersistentBatch(items(cfg), hooks=True)
    ms_pers = time_graph(pb, args.steps, args.warmup)
    assert [int(r.n_out) for r, _ in pb.results()] == per_out
    # per-kernel durations: the same launches again, each followed by a read
    # of the events (kept out of the step time)
    enc_ms, dec_ms = [], []
    for _ in range(args.steps):
        pb.run()  # the graph's kernels on torch's stream, events around the largest class's
        torch.cuda.synchronize()
        enc_ms.append(pb.enc_hook.elapsed_ms())
        dec_ms.append(pb.dec_hook.elapsed_ms())
    plans = [(x.dim(), cd.block, v) for x, cd, v in zip(xs, pb.codecs, pb.field_vec)]
    big = next(pl for pl, c in zip(plans, pb.field_class) if c == 0)  # the class the hooks time
    pb.close()
    del pb
    torch.cuda.empty_cache()
    ms_untuned = None
    if not args.no_extras:
        default = {1: (1024, 0), 2: (16, 0), 3: (8, 0)}
        b0 = BT.PersistentBatch(items(default))
        ms_untuned = time_graph(b0, args.steps, args.warmup)
        b0.close()
        del b0
        torch.cuda.empty_cache()
    n_out = sum(per_out)
    ms = min(ms_graph, ms_pers)
    # the largest class: its fields' algorithmic bytes per encode / decode launch
    cells_of = {}
    for (d, B, V), x in zip(plans, xs):
        cells_of[(d, B, V)] = cells_of.get((d, B, V), 0) + x.numel()
    big_bytes = sum(6.0 * x.numel() + 8.0 * o for pl, x, o in zip(plans, xs, per_out) if pl == big)
    e_ms, d_ms = float(np.mean(enc_ms)), float(np.mean(dec_ms))
    kname, kms = (f"k_encode_batch<{big[0]},{big[1]},{big[2]}>", e_ms) if e_ms >= d_ms else \
        (f"k_decode_batch<{big[0]},{big[1]},{big[2]}>", d_ms)
    achieved = big_bytes / (kms * 1e-3) / 1e9
    # algorithmic bytes of the whole step: value range 4N, encode and decode 6N + 8 n_out each
    alg = 16.0 * N + 16.0 * n_out
    value = 4.0 * N / (ms * 1e-3) / 1e9
    out = {
        "metric": "dual-quant compress+decompress GB/s on 1 MI355X; % HBM peak; outlier %",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+i32", "data": "synthetic",
        "config": {"workload": W["desc"], "fields": len(specs), "cells": N, "radius": W["radius"],
                   "path": "persistent" if ms_pers <= ms_graph else "graph of per-field launches",
                   "tuned": {str(d): list(c) for d, c in sorted(cfg.items())}},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": stored_batch_traffic(kname), "avg_kernel_ms": round(kms, 5),
                     "kernel_cells": cells_of[big], "kernel_source_hash": kernel_source_hash()},
        "outlier_pct": round(100.0 * n_out / N, 4), "n_out": n_out,
        "step_algorithmic_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
        "step_pct_hbm_peak": round(100.0 * alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 2),
        "ms_per_step_graph": round(ms_graph, 4), "ms_per_step_persistent": round(ms_pers, 4),
        "ms_per_step_persistent_untuned": round(ms_untuned, 4) if ms_untuned else None,
        "kernels_ms": {f"k_encode_batch<{big[0]},{big[1]},{big[2]}>": round(e_ms, 5),
                       f"k_decode_batch<{big[0]},{big[1]},{big[2]}>": round(d_ms, 5)},
        "autotune_s": round(t_tune, 2),
        "fields": [{"shape": list(s["shape"]), "eb_rel": round(s["eb"], 8), "slope": round(s["slope"], 3),
                    "outlier_pct": round(100.0 * po / x.numel(), 3)} for s, po, x in zip(specs, per_out, xs)],
    }
    if not args.no_extras:
        log("bench: 256^3 outlier counts")
        out["c2_outliers"] = c2_outlier_counts(W)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline_batch(xs, specs, {d: c for d, c in cfg.items()}, W)
    del xs
    torch.cuda.empty_cache()
    if not args.no_extras:
        tb, n_train, t_train = train_selector()
        log("bench: 512^3 fields, mixed-edge streams (exhaustive, learned) against zero padding")
        out["c4_mixed_edges"] = c4_mixed_report(tb)
        log("bench: 512x1024x1024 field, learned padding against zero padding")
        out["c5_learned_vs_zero"] = c5_selector_report(tb, n_train, t_train)
    print(json.dumps(out), flush=True)


def entropy_report(codecs, pads, n_out, reps=10):
    """Huffman stage on each mode's codes (outside the timed step): bits per
    code, compression ratio of the whole stream against fp32, and the GPU
    times of the codebook, encode and decode."""
    import torch
    from paper_2201_04614_amd import binding as dq
    from paper_2201_04614_amd import huffman as HF
    out = {}
    for pi, pad in enumerate(pads):
        cd = codecs[pi][0]
        codes = cd.codes.reshape(-1)
        n = codes.numel()
        K = 2 * cd.radius
        ws = HF._ws(n, codes.device)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        t = {"codebook": 0.0, "encode": 0.0, "decode": 0.0}
        for r in range(reps + 1):
            ev[0].record()
            cb = HF.codebook(codes, K)
            ev[1].record()
            bs = HF.encode(codes, cb, ws=ws)
            ev[2].record()
            back, st = HF.decode(bs, cb, ws=ws)
            ev[3].record()
            torch.cuda.synchronize()
            if r:
                t["codebook"] += ev[0].elapsed_time(ev[1]) / reps
                t["encode"] += ev[1].elapsed_time(ev[2]) / reps
                t["decode"] += ev[2].elapsed_time(ev[3]) / reps
        assert int(cb.status.item()) == 0 and int(bs.status.item()) == 0 and int(st.item()) == 0
        assert torch.equal(back, codes)
        words = int(bs.chunk_off[-1].item())
        nch = bs.chunk_off.numel() - 1
        stream = 4 * words + 8 * (nch + 1) + 6 * nch + K + 8 * n_out[pad] + 4 * dq.pad_count(cd.p) + 64
        out[pad] = {"bits_per_code": round(32.0 * words / n, 4), "ratio_vs_fp32": round(4.0 * n / stream, 3),
                    "codebook_ms": round(t["codebook"], 4), "encode_ms": round(t["encode"], 4),
                    "decode_ms": round(t["decode"], 4),
                    "encode_GBps_of_codes": round(2.0 * n / (t["encode"] * 1e-3) / 1e9, 1),
                    "decode_GBps_of_codes": round(2.0 * n / (t["decode"] * 1e-3) / 1e9, 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sets", type=int, default=0, help="rotating buffer sets per padding mode (0 = workload's)")
    ap.add_argument("--vec", type=int, default=0, help="cells per lane hint (0 = automatic)")
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-config", default="",
                    help="batch workload: fixed block edge and cells per lane per dimensionality instead of the "
                         "autotuner's, e.g. 1:1024:4,2:16:1,3:4:1 (to profile the configuration a run chose)")
    ap.add_argument("--no-extras", action="store_true",
                    help="batch workload: skip the untuned run, the 256^3 outlier counts and the learned-padding "
                         "report on the 512x1024x1024 field")
    ap.add_argument("--entropy", action="store_true",
                    help="also time the Huffman stage on each mode's codes and report the compression ratio")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the plain copy used to scale the byte counters")
    args = ap.parse_args()
    if args.copy_only:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the path has no "
              "multi-GPU code in this build; see the sharding notes in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2201_04614_amd import binding as dq
    from paper_2201_04614_amd import fields

    W = WORKLOADS[args.workload]
    if W.get("batch"):
        run_batch(args, W)
        return
    SHAPE, BLOCK, RADIUS, PADS = W["shape"], W["block"], W["radius"], W["pads"]
    sets = args.sets or W["sets"]
    dev = torch.device("cuda:0")
    log(f"bench: generating the {args.workload} field {SHAPE}")
    if args.workload == "c2":
        x = fields.power_law_grf(SHAPE, slope=3.0, seed=2)
        xd = None
    elif args.workload == "c1":
        x = fields.sinusoid_field(SHAPE, seed=1)
        xd = None
    else:
        xd = fields.sharp_feature_field_device(SHAPE, seed=5)
        x = xd.cpu().numpy()
    n = x.size
    eb_arg = W["eb"] if W["eb_mode"] == "rel" else W["eb"] * fields.field_range(x)
    xs = [[(xd if xd is not None else torch.from_numpy(x).to(dev)) for _ in range(sets)] for _ in PADS]
    codecs = [[dq.Codec(SHAPE, eb_arg, W["eb_mode"], BLOCK, pad, RADIUS, out_cap=max(1024, n // 16), device=dev,
                        vec=args.vec)
               for _ in range(sets)] for pad in PADS]
    torch.cuda.synchronize()

    # warmup: also fixes each mode's outlier count and bound (identical every step)
    n_out, eb_abs = {}, {}
    for w in range(max(1, args.warmup)):
        for pi, pad in enumerate(PADS):
            for s in range(sets):
                cd = codecs[pi][s]
                cd.compress_async(xs[pi][s])
                r = cd.result()
                assert r.status == dq.DQ_OK, dq.strerror(r.status)
                n_out[pad], eb_abs[pad] = int(r.n_out), float(r.eb_abs)
                cd.decompress_async(eb_abs[pad], n_out[pad])
                rd = cd.decompress_result()
                assert rd.status == dq.DQ_OK, dq.strerror(rd.status)
    torch.cuda.synchronize()
    log(f"bench: warmup done, outliers per mode {n_out}")

    def run_steps(hooks=None):
        for k in range(args.steps):
            s = k % sets
            for pi, pad in enumerate(PADS):
                cd = codecs[pi][s]
                he, hd = hooks[k][pi] if hooks else (None, None)
                cd.compress_async(xs[pi][s], hooks=he)
                cd.decompress_async(eb_abs[pad], n_out[pad], hooks=hd)

    # timed region: K steps, every kernel enqueued back to back on one stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    run_steps()
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"bench: {args.steps} steps, {ms_step:.4f} ms/step")

    # per-kernel durations: the same K steps again with HIP events recorded
    # right before and after each encode and decode launch (event records
    # add gaps between kernels, so this pass is kept out of the step time)
    hooks = [[(dq.Hook(), dq.Hook()) for _ in PADS] for _ in range(args.steps)]
    torch.cuda.synchronize()
    run_steps(hooks)
    torch.cuda.synchronize()

    # the timed results are the warmup's: same field, same outliers
    for pi, pad in enumerate(PADS):
        for s in range(sets):
            r = codecs[pi][s].result()
            assert r.status == dq.DQ_OK and int(r.n_out) == n_out[pad]
            assert codecs[pi][s].decompress_result().status == dq.DQ_OK

    enc_ms = {pad: np.mean([hooks[k][pi][0].elapsed_ms() for k in range(args.steps)])
              for pi, pad in enumerate(PADS)}
    dec_ms = {pad: np.mean([hooks[k][pi][1].elapsed_ms() for k in range(args.steps)])
              for pi, pad in enumerate(PADS)}
    for row in hooks:
        for he, hd in row:
            he.close()
            hd.close()

    nb = dq.num_blocks(codecs[0][0].p)
    pads_bytes = {"zero": 0, "block_mean": 4 * nb, "edge_mean": 4 * len(SHAPE) * nb, "global_mean": 4}
    # algorithmic bytes per launch: encode reads x, writes codes, outliers
    # (index + value) and pads; decode reads the same stream and writes x_hat
    enc_bytes = {pad: 6.0 * n + 8.0 * n_out[pad] + pads_bytes[pad] for pad in PADS}
    dec_bytes = {pad: 6.0 * n + 8.0 * n_out[pad] + pads_bytes[pad] for pad in PADS}
    enc_tot, dec_tot = sum(enc_ms.values()), sum(dec_ms.values())
    if enc_tot >= dec_tot:
        kname, kms, kbytes = "encode", enc_tot / len(PADS), np.mean(list(enc_bytes.values()))
    else:
        kname, kms, kbytes = "decode", dec_tot / len(PADS), np.mean(list(dec_bytes.values()))
    achieved = kbytes / (kms * 1e-3) / 1e9

    value = len(PADS) * 4.0 * n / (ms_step * 1e-3) / 1e9
    # bytes the whole step must move: value-range pass (4N, relative bound) + encode + decode per mode
    rel_pass = 4.0 * n if W["eb_mode"] == "rel" else 0.0
    step_bytes = sum(rel_pass + enc_bytes[p] + dec_bytes[p] for p in PADS)
    out = {
        "metric": "dual-quant compress+decompress GB/s on 1 MI355X; % HBM peak; outlier %",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+i32",
        "data": "synthetic",
        "config": {"workload": W["desc"], "shape": list(SHAPE), "block": BLOCK, "radius": RADIUS,
                   "eb": W["eb"], "eb_mode": W["eb_mode"] + ("" if W["eb_mode"] == "rel" else " (x range)"),
                   "buffer_sets": sets, "vec_hint": args.vec},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": stored_traffic() if (kname == "encode" and args.workload == "c2") else None,
                     "avg_kernel_ms": round(kms, 5), "kernel_source_hash": kernel_source_hash()},
        "kernels_ms": {"encode": {p: round(v, 5) for p, v in enc_ms.items()},
                       "decode": {p: round(v, 5) for p, v in dec_ms.items()}},
        "outlier_pct": {p: round(100.0 * n_out[p] / n, 5) for p in PADS},
        "n_out": n_out,
        "eb_abs": eb_abs[PADS[0]],
        "step_algorithmic_GBps": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
        "step_pct_hbm_peak": round(100.0 * step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 2),
    }
    if args.entropy:
        log("bench: Huffman stage on the codes")
        out["entropy"] = entropy_report(codecs, PADS, n_out)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(x, W, eb_abs[PADS[0]])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
