"""Benchmark: compress + decompress of a 512^3 float32 field on one MI355X.

Workload (one "step"): the 512^3 Gaussian random field with P(k) ~ k^-3
(seeded FFT synthesis, scaled to [0, 1]) is compressed and decompressed at
value-range-relative error bounds 1e-2, 1e-3 and 1e-4 - three full round
trips of the whole path (value range, prequantisation + Lorenzo + codes +
histogram, Huffman code, encode, container; decode + inverse Lorenzo +
patches).  Inputs and output buffers are resident in HBM before timing.

Prints one JSON line.  `value` is round-trip throughput: input bytes
(3 x 4 N per step) divided by the wall time of the timed steps.
Per-stage times come from HIP events the library records on the stream
the kernels run on, inside the timed region.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Other workloads (not the headline line; same JSON keys):
  --workload selector   1024^3 k^-11/3 field + 64 tanh fronts + 1% log-normal
                        spikes at rel 1e-4: compress with first-order Lorenzo,
                        exhaustive per-block trial and the learned selector
                        (trained first on disjoint seeds, outside the timing)
  --workload batch2d    64 uneven 2D fields (per-field offset, scale, bound):
                        one graph-captured batch call vs per-field calls
  --workload batchmixed 256 mixed 1D/2D/3D fields: batched first-order Lorenzo
                        vs batched learned selector
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
EBS = (1e-2, 1e-3, 1e-4)
SHAPE = (512, 512, 512)
LINK_GBPS = 35.7  # the paper's measured GPU-to-host bandwidth on its H100 node (Table 1), for Eq. (1)


# stage -> (kernel as rocprofv3 names it on the 512^3 first-order Lorenzo
# workload, the source file that holds it)
STAGE_KERNEL = {
    "compress:minmax": ("fz::k_minmax", "fz_quant.hip"),
    "compress:quant": ("fz::k_quant<3, 0>", "fz_quant.hip"),
    "compress:encode": ("fz::k_encode<3>", "fz_huffman.hip"),
    "compress:finalize": ("fz::k_finalize", "fz_huffman.hip"),
    "decompress:oindex": ("fz::k_outlier_index", "fz_decode.hip"),
    "decompress:decode": ("fz::k_decode_fast<3, false, true>", "fz_decode.hip"),
}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_512cubed_grf_lorenzo1.md")


def source_digest(fname: str) -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_2509_20563_amd", "csrc", fname), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(stage: str):
    """HBM bytes per launch of a stage's kernel from the committed PMC
    summary (calibrated FETCH_SIZE + WRITE_SIZE), or None when there is
    none or the kernel's source changed since the counters were taken."""
    if stage not in STAGE_KERNEL or not os.path.exists(TRAFFIC_PROFILE):
        return None
    kern, src = STAGE_KERNEL[stage]
    digest = source_digest(src)
    with open(TRAFFIC_PROFILE) as f:
        for line in f:
            cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            if len(cells) >= 7 and cells[0] == kern:
                return int(float(cells[4])) if cells[6] == digest else None
    return None


def stage_bytes(stage: str, n: int, nblocks: int, h: dict, total: int) -> float:
    """Algorithmic bytes one launch of a stage must move (see the design notes)."""
    ntiles = (nblocks + 3) // 4
    side = 8 * (h["n_outliers"] + h["n_patches"])
    stream = 4 * h["stream_words"]
    return {
        "minmax": 4 * n,
        "quant": 4 * n + 2 * n + side,
        "encode": 2 * n + 2 * nblocks + stream,
        "scan_counts": 4 * ntiles + 8 * ntiles,
        "finalize": 2 * side + 12 * ntiles,
        "lut": 512,
        "scan": 2 * nblocks + 8 * nblocks,
        "oindex": 4 * h["n_outliers"] + (8 * nblocks if h["n_outliers"] else 0),
        "decode": stream + 10 * nblocks + 4 * h["n_outliers"] + (8 * nblocks if h["n_outliers"] else 0) + 4 * n,
        "patch": 8 * h["n_patches"] + 4 * h["n_patches"],
    }.get(stage, 0.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--shape", type=str, default=None)
    ap.add_argument("--workload", default="roundtrip", choices=["roundtrip", "selector", "batch2d", "batchmixed"])
    ap.add_argument("--fields", type=int, default=None)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (sharding is a design note only)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from inputs import fields
    from paper_2509_20563_amd import fz, metrics

    if args.workload != "roundtrip":
        return {"selector": bench_selector, "batch2d": bench_batch2d, "batchmixed": bench_batchmixed}[args.workload](args)
    shape = tuple(int(s) for s in (args.shape or "512,512,512").split(","))
    n = int(np.prod(shape))
    print(f"[bench] generating {shape} k^-3 field", file=sys.stderr, flush=True)
    x_host = fields.grf(shape, alpha=3.0, seed=2)
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(x_host).to(dev)
    # a plain device copy of the field (4N bytes read, 4N written): the
    # reference kernel against which HBM byte counters are calibrated
    calib = torch.empty_like(x)
    calib.copy_(x)
    torch.cuda.synchronize()
    del calib
    ctx = fz.Context(0, max_elems=n)
    cap = ctx.compress_bound(shape)
    outs = [torch.empty(cap, dtype=torch.uint8, device=dev) for _ in EBS]
    recs = [torch.empty(shape, dtype=torch.float32, device=dev) for _ in EBS]
    headers = [None] * len(EBS)
    sizes = [0] * len(EBS)

    def step(timed_stages=None):
        for i, eb in enumerate(EBS):
            c = ctx.compress(x, eb, fz.EB_REL, out=outs[i])
            if timed_stages is not None:
                for name, ms in ctx.stage_times():
                    timed_stages.setdefault(("c", i, name), []).append(ms)
            sizes[i] = c.numel()
            if headers[i] is None:
                headers[i] = c[:128].cpu().numpy().tobytes()
            ctx.decompress(c, header=headers[i], out=recs[i])
            if timed_stages is not None:
                for name, ms in ctx.stage_times():
                    timed_stages.setdefault(("d", i, name), []).append(ms)

    nblocks = (-(-shape[-1] // 8)) * (-(-shape[-2] // 8)) * (-(-shape[0] // 8)) if len(shape) == 3 else 0

    def per_stage(st: dict) -> dict:
        out: dict = {}
        for (d, i, name), ms in st.items():
            h = fz.header_fields(headers[i])
            key = ("compress:" if d == "c" else "decompress:") + name
            e = out.setdefault(key, {"ms": 0.0, "bytes": 0.0, "launches": 0})
            e["ms"] += sum(ms)
            e["launches"] += len(ms)
            e["bytes"] += len(ms) * stage_bytes(name, n, nblocks, h, sizes[i])
        return out

    # warmup with every stage timed (events between all kernels): the stage
    # breakdown and the dominant stage; the timed steps then record events
    # around the dominant stage alone, so the other kernels run back to back
    print("[bench] warmup", file=sys.stderr, flush=True)
    warm: dict = {}
    for k in range(args.warmup):
        # the last warmup step times every stage (earlier ones carry the
        # first-call costs)
        if k == args.warmup - 1:
            ctx.set_timing(True)
            step(warm)
        else:
            step()
    ctx.set_timing(True)
    dom_stage = None
    if warm:
        dom_key = max(per_stage(warm).items(), key=lambda kv: kv[1]["ms"])[0]
        dom_stage = dom_key.split(":", 1)[1]
        ctx.set_timing_stage(dom_stage)
    stages: dict = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(stages)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_timing_stage(None)
    ctx.set_timing(False)
    print("[bench] timed steps done", file=sys.stderr, flush=True)

    # whole calls on the GPU clock (after the timed region): one event before
    # each call's first kernel and one after its last, none in between
    call_ms = {"compress": [0.0] * len(EBS), "decompress": [0.0] * len(EBS)}
    ctx.set_timing(True)
    ctx.set_timing_stage("call")
    for i, eb in enumerate(EBS):
        for _ in range(3):
            c = ctx.compress(x, eb, fz.EB_REL, out=outs[i])
            call_ms["compress"][i] += ctx.stage_times()[0][1] / 3
            ctx.decompress(c, header=headers[i], out=recs[i])
            call_ms["decompress"][i] += ctx.stage_times()[0][1] / 3
    ctx.set_timing_stage(None)
    ctx.set_timing(False)

    # per-direction throughput (separate passes, after the timed region)
    per_eb = []
    parse_header = fz.header_fields
    for i, eb in enumerate(EBS):
        h = parse_header(headers[i])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            ctx.compress(x, eb, fz.EB_REL, out=outs[i])
        torch.cuda.synchronize()
        tc = (time.perf_counter() - t) / 3
        c = outs[i][: sizes[i]]
        t = time.perf_counter()
        for _ in range(3):
            ctx.decompress(c, header=headers[i], out=recs[i])
        torch.cuda.synchronize()
        td = (time.perf_counter() - t) / 3
        err = (recs[i].double() - x.double()).abs().max().item()
        rng = float(x_host.max()) - float(x_host.min())
        mse = ((recs[i].double() - x.double()) ** 2).mean().item()
        cr = metrics.compression_ratio(n, sizes[i])
        comp = metrics.throughput_gbps(n, tc)
        per_eb.append({
            "eb_rel": eb, "eb_abs": h["eb_abs"], "bytes": sizes[i], "cr": round(cr, 4),
            "bit_rate": round(metrics.bit_rate(n, sizes[i]), 4),
            "psnr_db": round(20 * math.log10(rng / math.sqrt(mse)), 3) if mse > 0 else None,
            "max_err_over_eb": err / h["eb_abs"],
            "compress_gbps": round(comp, 2), "decompress_gbps": round(metrics.throughput_gbps(n, td), 2),
            "n_outliers": h["n_outliers"], "n_patches": h["n_patches"], "verbatim": bool(h["flags"] & 1),
            "eq1_speedup_at_35.7GBps": round(metrics.overall_speedup(LINK_GBPS, cr, comp), 3),
        })

    # dominant kernel and its roofline (HIP events around it inside the timed region)
    by_stage = per_stage(stages)
    dom_name, dom = max(by_stage.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(dom_name),
                "avg_launch_ms": round(avg_ms, 4), "alg_bytes_per_launch": int(bytes_per_launch)}
    full = per_stage(warm if warm else stages)
    stage_summary = {k: {"avg_ms": round(v["ms"] / v["launches"], 4),
                         "gbps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
                     for k, v in sorted(full.items())}
    # whole calls: the call's algorithmic bytes (the sum over its stages) over
    # the call's own GPU time (events around the whole call), per direction
    call_roofline = {}
    call_stages = {"compress": ("minmax", "quant", "scan_counts", "encode", "finalize"),
                   "decompress": ("lut", "scan", "oindex", "decode", "patch")}
    for d, names in call_stages.items():
        by = sum(stage_bytes(name, n, nblocks, fz.header_fields(headers[i]), sizes[i])
                 for i in range(len(EBS)) for name in names)
        ms = sum(call_ms[d])
        if ms > 0:
            a = by / (ms * 1e-3) / 1e9
            call_roofline[d] = {"achieved": round(a, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                "frac": round(a / HBM_PEAK_GBPS, 4),
                                "avg_call_ms": [round(v, 4) for v in call_ms[d]]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(x_host)

    value = 3 * 4.0 * n * args.steps / wall / 1e9
    line = {
        "metric": "compress/decompress GB/s and % HBM roofline on 1 MI355X; ratio at fixed eb",
        "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, shape))} k^-3 Gaussian random field, rel eb 1e-2/1e-3/1e-4, "
                               "compress + decompress per eb (first-order Lorenzo, radius 512, Huffman)",
                   "n_values": n, "ebs": list(EBS)},
        "per_eb": per_eb,
        "stages": stage_summary,
        "stages_timed_in": "the last warmup step (every stage); the timed steps time the dominant stage alone"
                           if warm else "timed steps",
        "roofline": roofline,
        "call_roofline": call_roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(x_host):
    """The CPU oracle, single-threaded, on the first half (z) of the same field
    at all three bounds: round-trip GB/s of input."""
    import numpy as np

    import oracle

    sample = np.ascontiguousarray(x_host[: x_host.shape[0] // 2])
    print(f"[bench] cpu baseline on {sample.shape}", file=sys.stderr, flush=True)
    t = time.perf_counter()
    for eb in EBS:
        c = oracle.compress(sample, eb, 1)
        oracle.decompress(c)
    dt = time.perf_counter() - t
    return {"value": round(3 * 4.0 * sample.size / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample.shape[0]} z-planes ({'x'.join(map(str, sample.shape))}) of the same field, "
                      f"compress + decompress at rel eb 1e-2/1e-3/1e-4, single-threaded C oracle",
            "seconds": round(dt, 2)}


# ------------------------------------------------------------------ helpers
def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / steps


def _line(metric, value, unit, args, ms, config, higher=True, **extra):
    d = {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1, "steps": args.steps,
         "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": higher, "scaling": "weak",
         "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": config}
    d.update(extra)
    print(json.dumps(d), flush=True)


def train_selector(ctx, fz, device, seeds=(101, 102, 103, 104), edge=128, ebs=(1e-2, 1e-3, 1e-4), epochs=200):
    """Train the context's selector on fronts/spikes fields of seeds disjoint
    from the evaluation fields; returns (seconds, first loss, last loss, samples)."""
    import torch
    from inputs import fields_gpu
    feats, costs = [], []
    for sd in seeds:
        x = fields_gpu.fronts_spikes((edge, edge, edge), seed=sd, n_fronts=8, device=device)
        for eb in ebs:
            feats.append(ctx.block_features(x, eb, fz.EB_REL))
            costs.append(ctx.block_trial(x, eb, fz.EB_REL)[1])
    f = torch.cat(feats).contiguous()
    c = torch.cat(costs).contiguous()
    torch.cuda.synchronize()
    t = time.perf_counter()
    loss = ctx.selector_train(f, c, epochs=epochs, batch=1024, seed=1)
    torch.cuda.synchronize()
    return time.perf_counter() - t, float(loss[0]), float(loss[-1]), int(f.shape[0])


def bench_selector(args):
    import torch
    from inputs import fields_gpu
    from paper_2509_20563_amd import fz, metrics
    dev = torch.device("cuda", 0)
    shape = tuple(int(s) for s in (args.shape or "1024,1024,1024").split(","))
    ctx = fz.Context(0)
    print("[bench] training the selector", file=sys.stderr, flush=True)
    tsec, l0, l1, ns = train_selector(ctx, fz, dev)
    print(f"[bench] generating {shape} fronts/spikes field", file=sys.stderr, flush=True)
    x = fields_gpu.fronts_spikes(shape, seed=3, device=dev)
    n = x.numel()
    eb = 1e-4
    out = torch.empty(ctx.compress_bound(shape), dtype=torch.uint8, device=dev)
    res = {}
    for name, pred in (("lorenzo1", fz.PRED_LORENZO1), ("trial", fz.PRED_AUTO_TRIAL), ("selector", fz.PRED_AUTO_MLP)):
        print(f"[bench] {name}", file=sys.stderr, flush=True)
        sizes = []
        dt = _timed(lambda: sizes.append(ctx.compress(x, eb, fz.EB_REL, out=out, pred=pred).numel()),
                    args.steps, args.warmup)
        c = out[: sizes[-1]]
        y = ctx.decompress(c)
        h = fz.header_fields(c[:128].cpu().numpy().tobytes())
        err = (y.double() - x.double()).abs().max().item()
        res[name] = {"compress_gbps": round(metrics.throughput_gbps(n, dt), 2), "bytes": sizes[-1],
                     "cr": round(metrics.compression_ratio(n, sizes[-1]), 4),
                     "max_err_over_eb": err / h["eb_abs"], "ms": round(dt * 1e3, 3)}
        del y
    # the selection stage alone (the same min/max pass first in both): the
    # selector's features + network pass against the trial's reference
    # first-order pass, codebook and three-predictor cost pass
    print("[bench] selection stage alone", file=sys.stderr, flush=True)
    t_sel = _timed(lambda: ctx.block_select(x, eb, fz.EB_REL), args.steps, args.warmup)
    t_tri = _timed(lambda: ctx.block_trial(x, eb, fz.EB_REL), args.steps, args.warmup)
    # breakdown: the same pass with the features written out and no network
    t_feat = _timed(lambda: ctx.block_features(x, eb, fz.EB_REL), args.steps, args.warmup)
    ch_sel, _ = ctx.block_select(x, eb, fz.EB_REL)
    ch_tri, _ = ctx.block_trial(x, eb, fz.EB_REL)
    selection = {"selector_ms": round(t_sel * 1e3, 3), "trial_ms": round(t_tri * 1e3, 3),
                 "features_only_ms": round(t_feat * 1e3, 3),
                 "speed_selector_over_trial": round(t_tri / t_sel, 3),
                 "agreement_with_trial": round(float((ch_sel == ch_tri).float().mean().item()), 4),
                 "selector_choice_counts": [int((ch_sel == k).sum().item()) for k in range(3)],
                 "trial_choice_counts": [int((ch_tri == k).sum().item()) for k in range(3)]}
    sel, tri, p0 = res["selector"], res["trial"], res["lorenzo1"]
    _line("learned per-block predictor selector: compress GB/s; CR vs exhaustive trial", sel["compress_gbps"],
          "GB/s", args, sel["ms"],
          {"workload": f"{'x'.join(map(str, shape))} k^-11/3 field + 64 tanh fronts + 1% log-normal spikes, "
                       "rel eb 1e-4, 8^3 blocks choose first/second-order Lorenzo or regression", "n_values": n},
          modes=res, cr_selector_over_trial=round(sel["cr"] / tri["cr"], 4),
          speed_selector_over_trial_end_to_end=round(sel["compress_gbps"] / tri["compress_gbps"], 3),
          selection_stage=selection,
          cr_gain_over_lorenzo1=round(sel["cr"] / p0["cr"], 4),
          training={"seconds": round(tsec, 2), "samples": ns, "loss_first_epoch": l0, "loss_last_epoch": l1,
                    "fields": "4 fronts/spikes fields 128^3, seeds 101-104 (evaluation seed 3), rel 1e-2/1e-3/1e-4"})


def _bench_batch(args, fz, ctx, batch, label, preds=None):
    import torch
    from paper_2509_20563_amd import metrics
    xs = [f for f, _ in batch]
    ebs = [eb for _, eb in batch]
    nf = len(xs)
    preds = preds or [fz.PRED_LORENZO1] * nf
    n = sum(x.numel() for x in xs)
    modes = [fz.EB_REL] * nf
    print(f"[bench] {label}: autotune", file=sys.stderr, flush=True)
    try:
        k, w = ctx.batch_autotune(xs, ebs, modes, preds)
    except fz.FZError as e:  # the autotuner is switched off: default launch knobs
        print(f"[bench] {label}: autotune unavailable ({e}); default knobs", file=sys.stderr, flush=True)
        k, w = ctx.batch_tuning(xs, ebs, modes, preds)
    out = torch.empty(ctx.compress_batch_bound([x.shape for x in xs], preds), dtype=torch.uint8, device=xs[0].device)
    holder = {}

    def run_batch():
        holder["packed"], holder["offs"] = ctx.compress_batch(xs, ebs, modes, preds, out=out)

    print(f"[bench] {label}: batched", file=sys.stderr, flush=True)
    tb = _timed(run_batch, args.steps, args.warmup)
    packed, offs = holder["packed"], holder["offs"]
    singles = [torch.empty(ctx.compress_bound(x.shape), dtype=torch.uint8, device=x.device) for x in xs]

    def run_single():
        for i, x in enumerate(xs):
            ctx.compress(x, ebs[i], fz.EB_REL, out=singles[i], pred=preds[i])

    print(f"[bench] {label}: per-field calls", file=sys.stderr, flush=True)
    ts = _timed(run_single, args.steps, args.warmup)
    recs = [torch.empty_like(x) for x in xs]
    td = _timed(lambda: ctx.decompress_batch(packed, offs, recs), args.steps, args.warmup)
    hdrs = [packed[offs[i]:offs[i] + 128].cpu().numpy().tobytes() for i in range(nf)]

    def run_single_d():
        for i in range(nf):
            ctx.decompress(packed[offs[i]:offs[i + 1]], header=hdrs[i], out=recs[i])

    tsd = _timed(run_single_d, args.steps, args.warmup)
    worst = 0.0
    for i in range(nf):
        h = fz.header_fields(hdrs[i])
        worst = max(worst, (recs[i].double() - xs[i].double()).abs().max().item() / h["eb_abs"])
    return {"n_fields": nf, "n_values": n, "bytes_in": 4 * n, "bytes_out": int(offs[-1]),
            "cr": round(metrics.compression_ratio(n, int(offs[-1])), 4),
            "tuned_chains": k, "tuned_wg_per_cu": sorted(set(w)),
            "batch_compress_gbps": round(4 * n / tb / 1e9, 2), "per_field_compress_gbps": round(4 * n / ts / 1e9, 2),
            "batch_decompress_gbps": round(4 * n / td / 1e9, 2),
            "per_field_decompress_gbps": round(4 * n / tsd / 1e9, 2),
            "compress_speedup_batch_over_per_field": round(ts / tb, 3), "max_err_over_eb": worst,
            "ms_batch_compress": round(tb * 1e3, 3)}


def bench_batch2d(args):
    import torch
    from inputs import fields_gpu
    from paper_2509_20563_amd import fz
    dev = torch.device("cuda", 0)
    nf = args.fields or 64
    print(f"[bench] generating {nf} uneven 2D fields", file=sys.stderr, flush=True)
    batch = fields_gpu.batch_2d(n_fields=nf, device=dev)
    ctx = fz.Context(0)
    r = _bench_batch(args, fz, ctx, batch, "batch2d")
    _line("batched compress GB/s of uneven 2D fields (one graph-captured call) vs per-field calls",
          r["batch_compress_gbps"], "GB/s", args, r["ms_batch_compress"],
          {"workload": f"{nf} 2D k^-3 fields, height 256-3600, width 256-1800, per-field offset/scale "
                       "log-uniform 1e-3..1e3 and rel eb log-uniform 1e-5..1e-2, first-order Lorenzo",
           "n_values": r["n_values"]}, batch=r)


def bench_batchmixed(args):
    import torch
    from inputs import fields_gpu
    from paper_2509_20563_amd import fz
    dev = torch.device("cuda", 0)
    nf = args.fields or 256
    ctx = fz.Context(0)
    print("[bench] training the selector", file=sys.stderr, flush=True)
    tsec, l0, l1, ns = train_selector(ctx, fz, dev)
    print(f"[bench] generating {nf} mixed fields", file=sys.stderr, flush=True)
    batch = fields_gpu.batch_mixed(n_fields=nf, device=dev)
    r0 = _bench_batch(args, fz, ctx, batch, "batchmixed lorenzo1")
    r1 = _bench_batch(args, fz, ctx, batch, "batchmixed selector", preds=[fz.PRED_AUTO_MLP] * nf)
    _line("batched compress GB/s of a mixed 1D/2D/3D batch with the learned selector; CR vs first-order Lorenzo",
          r1["batch_compress_gbps"], "GB/s", args, r1["ms_batch_compress"],
          {"workload": f"{nf} fields: 1D sorted positions 1M-64M values, 2D k^-3 (as the 2D batch), 3D 64^3-384^3 "
                       "k^-3..k^-5; rel eb log-uniform 1e-5..1e-2", "n_values": r1["n_values"]},
          selector=r1, lorenzo1=r0, cr_gain_over_lorenzo1=round(r1["cr"] / r0["cr"], 4),
          training={"seconds": round(tsec, 2), "samples": ns, "loss_first_epoch": l0, "loss_last_epoch": l1})


if __name__ == "__main__":
    main()
