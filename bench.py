"""Benchmark of the dual-quantisation hot path on one MI355X.

Default workload (one step): the 256^3 fp32 Gaussian random field with a k^-3
power spectrum (seed 2), relative error bound 1e-3, 8^3 blocks, radius 512,
run through compress + decompress once per padding mode (zero, block mean,
edge mean) - every stage of the path: value-range pass, prequantisation +
Lorenzo + codes + outlier staging (bound resolved per wave), outlier
placement, outlier index, prefix-sum decode + dequantisation.

--workload c1 / c5 measure the 512^2 sinusoid field (abs eb 1e-4 * range,
16^2 blocks, zero padding) and the 512 x 1024 x 1024 sharp-feature field
(abs eb 1e-4 * range, 8^3 blocks, zero padding) the same way. --workload c3
measures a batch of 64 uneven fields run as one HIP graph launch (block edge
and vector width per field from the autotuner).

Every call reads and writes its own buffers: inputs and outputs rotate over
enough distinct sets that the working set (> 1 GiB) cannot stay in the 256 MB
Infinity Cache, so the figure is HBM throughput. Inputs are resident in HBM
before the timed region.

Prints one JSON line: value = (padding modes) * 4N bytes / step time (GB/s of
fp32 input through compress + decompress), the roofline of the dominant
kernel (timed with HIP events recorded around it), and the CPU oracle timed
on a bounded sample.
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
                    "radius 512, zero padding, block edge and vector width per field from the autotuner; "
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


def run_batch(args, W):
    """The batched workload: one graph launch = compress + decompress of every field."""
    import torch
    from paper_2201_04614_amd import autotune as AT
    from paper_2201_04614_amd import batch as BT
    from paper_2201_04614_amd import binding as dq
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
    log(f"bench: {N} cells; autotuning block edge and vector width per field")
    t0 = time.perf_counter()
    tuned = []
    for k, (x, s) in enumerate(zip(xs, specs)):
        tuned.append(AT.tune(x, s["eb"], "rel", frac=0.1, iters=3)[:2])
        if k % 16 == 15:
            log(f"bench: {k + 1} fields tuned")
    t_tune = time.perf_counter() - t0

    def items(cfg):
        return [(x, dict(eb=s["eb"], eb_mode="rel", block=B, pad="zero", radius=W["radius"], out_cap=x.numel(),
                         vec=V)) for x, s, (B, V) in zip(xs, specs, cfg)]

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

    b = BT.Batch(items(tuned), branches=4)
    ms = time_graph(b, args.steps, args.warmup)
    res = b.results()
    per_out = [int(r.n_out) for r, _ in res]
    n_out = sum(per_out)
    # the same calls enqueued one by one on one stream (no graph)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        for cd, (x, _) in zip(b.codecs, items(tuned)):
            cd.compress_async(x)
            cd.decompress_dev_async()
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / args.steps
    b.close()
    del b
    default = [({1: 1024, 2: 16, 3: 8}[x.dim()], 0) for x in xs]
    b0 = BT.Batch(items(default), branches=4)
    ms_default = time_graph(b0, args.steps, args.warmup)
    b0.close()
    del b0
    # algorithmic bytes: value-range pass 4N, encode 6N + 8 n_out, decode 6N + 8 n_out
    alg = 16.0 * N + 16.0 * n_out
    value = 4.0 * N / (ms * 1e-3) / 1e9
    achieved = alg / (ms * 1e-3) / 1e9
    out = {
        "metric": "dual-quant compress+decompress GB/s on 1 MI355X; % HBM peak; outlier %",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+i32", "data": "synthetic",
        "config": {"workload": W["desc"], "fields": len(specs), "cells": N, "radius": W["radius"],
                   "graph_branches": 4},
        "roofline": {"bound": "hbm", "kernel": "whole batch graph (all kernels)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None},
        "outlier_pct": round(100.0 * n_out / N, 4),
        "ms_per_step_untuned": round(ms_default, 4), "ms_per_step_no_graph": round(ms_eager, 4),
        "autotune_s": round(t_tune, 2),
        "tuned": [{"shape": list(s["shape"]), "block": B, "vec": V, "eb_rel": round(s["eb"], 8),
                   "slope": round(s["slope"], 3), "outlier_pct": round(100.0 * po / n, 3)}
                  for s, (B, V), po, n in zip(specs, tuned, per_out, [x.numel() for x in xs])],
    }
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
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sets", type=int, default=0, help="rotating buffer sets per padding mode (0 = workload's)")
    ap.add_argument("--vec", type=int, default=0, help="cells per lane hint (0 = automatic)")
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
