"""Benchmark: compress + decompress of a 1024^3 float32 field on one MI355X.

Workload (one "step"): the 1024^3 field built from a P(k) ~ k^-11/3 Gaussian
random field scaled to [0, 1], 64 seeded tanh fronts (width about 2 cells)
and 1% of the cells set to log-normal spikes (sigma 2), at the
value-range-relative bound 1e-4, is compressed and decompressed once per
predictor mode: first-order Lorenzo in every 8^3 block (the paper's path),
the learned per-block selector, and exhaustive per-block trial.  Every
stage of the path runs in each round trip (value range, prequantisation +
prediction + codes + histogram, Huffman code, encode, container; decode +
inverse prediction + patches).  Inputs and output buffers are resident in
HBM before timing; the selector is trained beforehand on fields of other
seeds, outside the timing.

Prints one JSON line.  `value` is round-trip throughput: input bytes
(3 x 4 N per step) divided by the wall time of the timed steps.  Per-stage
times come from HIP events the library records on the stream the kernels
run on, inside the timed region.  Extra keys: per-mode compression and
decompression rates and whole-call rooflines, the same field with the
bound taken from the range without the spikes, the 512^3 k^-3 field at
1e-2/1e-3/1e-4 (first-order Lorenzo), and the CPU oracle on slabs of the
same field.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Other workloads (--workload; same JSON keys):
  c2          512^3 k^-3 field at rel 1e-2/1e-3/1e-4, first-order Lorenzo
  selector    the 1024^3 field: selection stage alone, selector vs trial
  batch2d     64 uneven 2D fields (per-field offset, scale, bound):
              one graph-captured batch call vs per-field calls
  batchmixed  256 mixed 1D/2D/3D fields: batched first-order Lorenzo vs
              batched learned selector
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
C3_SHAPE = (1024, 1024, 1024)
C3_EB = 1e-4
LINK_GBPS = 35.7  # the paper's measured GPU-to-host bandwidth on its H100 node (Table 1), for Eq. (1)
MODES = (("lorenzo1", 0), ("selector", 3), ("trial", 4))

# stage -> (kernel as rocprofv3 names it on the 1024^3 first-order Lorenzo
# round trip, the source file that holds it)
STAGE_KERNEL = {
    "compress:minmax": ("fz::k_minmax", "fz_quant.hip"),
    "compress:quant": ("fz::k_quant<3, 0>", "fz_quant.hip"),
    "compress:encode": ("fz::k_encode<3>", "fz_huffman.hip"),
    "compress:finalize": ("fz::k_finalize", "fz_huffman.hip"),
    "decompress:oindex": ("fz::k_outlier_index", "fz_decode.hip"),
    "decompress:decode": ("fz::k_decode_fast<3, false, true, true, false, false>", "fz_decode.hip"),
}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_1024cubed_fronts_spikes.md")


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
    """Bytes one launch of a first-order Lorenzo stage's kernel must move in
    this design (the kernel table of the design notes): the roofline of a
    single kernel."""
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


def call_bytes(direction: str, mode: str, n: int, container: int, rel: bool = True) -> float:
    """Algorithmic bytes of a whole call: what the method itself must move.
    Compression: the value range (4N, relative bound only), the field read
    for prediction (4N), the code round trip the histogram -> code barrier
    forces (2N written + 2N read, or a second 4N read of the field), the
    container (S); the selector adds its sample pass (a quarter of the
    field, N), trial its first-order histogram pass and its cost pass (8N).
    The bit-shuffle codec (mode "shuffle") has no histogram barrier, so its
    compression needs the range and one read of the field (4N [REL] + 4N +
    S).  Decompression: the container and the field written (S + 4N)."""
    if direction == "decompress":
        return container + 4.0 * n
    if mode == "shuffle":
        # no histogram barrier: the bit-shuffle codec needs one pass over
        # the field after the range
        return (4.0 * n if rel else 0.0) + 4.0 * n + container
    extra = {"lorenzo1": 0.0, "selector": 1.0 * n, "trial": 8.0 * n}[mode]
    return (4.0 * n if rel else 0.0) + 8.0 * n + container + extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the C3' and 512^3 extra keys")
    ap.add_argument("--modes", type=str, default=None,
                    help="comma list of predictor modes of the 1024^3 step (default: lorenzo1,selector,trial)")
    ap.add_argument("--shape", type=str, default=None)
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "selector", "batch2d", "batchmixed"])
    ap.add_argument("--fields", type=int, default=None)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (sharding is a design note only)",
              file=sys.stderr)
        sys.exit(2)
    return {"c3": bench_c3, "c2": bench_c2, "selector": bench_selector, "batch2d": bench_batch2d,
            "batchmixed": bench_batchmixed}[args.workload](args)


def _call_ms(ctx, fn, reps=3):
    """GPU time of whole calls (one event before a call's first kernel, one
    after its last), averaged over reps."""
    ctx.set_timing(True)
    ctx.set_timing_stage("call")
    t = 0.0
    for _ in range(reps):
        fn()
        t += ctx.stage_times()[0][1] / reps
    ctx.set_timing_stage(None)
    ctx.set_timing(False)
    return t


def _roof(bytes_, ms):
    a = bytes_ / (ms * 1e-3) / 1e9
    return {"achieved": round(a, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(a / HBM_PEAK_GBPS, 4),
            "avg_call_ms": round(ms, 4), "alg_bytes": int(bytes_)}


def bench_c3(args):
    import numpy as np
    import torch

    from inputs import fields_gpu
    from paper_2509_20563_amd import fz, metrics

    dev = torch.device("cuda", 0)
    shape = tuple(int(s) for s in (args.shape or ",".join(map(str, C3_SHAPE))).split(","))
    ctx = fz.Context(0)
    global MODES
    if args.modes:
        want = args.modes.split(",")
        MODES = tuple((m, p) for m, p in MODES if m in want)
    names = [m for m, _ in MODES]
    training = None
    if "selector" in names:
        print("[bench] training the selector", file=sys.stderr, flush=True)
        training = train_selector(ctx, fz, dev)
    print(f"[bench] generating {shape} fronts/spikes field", file=sys.stderr, flush=True)
    x, base_range = fields_gpu.fronts_spikes(shape, seed=3, device=dev, with_base_range=True)
    n = x.numel()
    # a plain device copy of the field (4N bytes read, 4N written): the
    # reference kernel against which HBM byte counters are calibrated
    calib = torch.empty_like(x)
    calib.copy_(x)
    torch.cuda.synchronize()
    del calib
    cap = ctx.compress_bound(shape)
    outs = {m: torch.empty(cap, dtype=torch.uint8, device=dev) for m, _ in MODES}
    rec = torch.empty(shape, dtype=torch.float32, device=dev)
    headers = {m: None for m, _ in MODES}
    sizes = {m: 0 for m, _ in MODES}
    nblocks = (-(-shape[-1] // 8)) * (-(-shape[-2] // 8)) * (-(-shape[0] // 8))

    def step(timed_stages=None):
        for m, pred in MODES:
            c = ctx.compress(x, C3_EB, fz.EB_REL, out=outs[m], pred=pred)
            if timed_stages is not None:
                for name, ms in ctx.stage_times():
                    timed_stages.setdefault(("c", m, name), []).append(ms)
            sizes[m] = c.numel()
            if headers[m] is None:
                headers[m] = c[:128].cpu().numpy().tobytes()
            ctx.decompress(c, header=headers[m], out=rec)
            if timed_stages is not None:
                for name, ms in ctx.stage_times():
                    timed_stages.setdefault(("d", m, name), []).append(ms)

    def per_stage(st: dict, mode="lorenzo1") -> dict:
        out: dict = {}
        for (d, m, name), ms in st.items():
            if m != mode:
                continue
            h = fz.header_fields(headers[m])
            key = ("compress:" if d == "c" else "decompress:") + name
            e = out.setdefault(key, {"ms": 0.0, "bytes": 0.0, "launches": 0})
            e["ms"] += sum(ms)
            e["launches"] += len(ms)
            e["bytes"] += len(ms) * stage_bytes(name, n, nblocks, h, sizes[m])
        return out

    # warmup; the last warmup step times every stage (events between all
    # kernels): the stage breakdown and the dominant first-order Lorenzo
    # stage.  The timed steps record events around that stage alone, so the
    # other kernels run back to back.
    print("[bench] warmup", file=sys.stderr, flush=True)
    warm: dict = {}
    for k in range(args.warmup):
        if k == args.warmup - 1:
            ctx.set_timing(True)
            step(warm)
            ctx.set_timing(False)
        else:
            step()
    dom_stage = None
    ctx.set_timing(True)
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

    # per mode: whole-call GPU times, rates, ratio, errors (after the timed region)
    modes = {}
    xd = None
    for m, pred in MODES:
        h = fz.header_fields(headers[m])
        tc = _call_ms(ctx, lambda: ctx.compress(x, C3_EB, fz.EB_REL, out=outs[m], pred=pred))
        c = outs[m][: sizes[m]]
        td = _call_ms(ctx, lambda: ctx.decompress(c, header=headers[m], out=rec))
        if xd is None:
            xd = x.double()
        diff = rec.double() - xd
        err = diff.abs().max().item()
        mse = (diff * diff).mean().item()
        del diff
        rng = float(x.max()) - float(x.min())
        cr = metrics.compression_ratio(n, sizes[m])
        modes[m] = {
            "bytes": sizes[m], "cr": round(cr, 4), "bit_rate": round(metrics.bit_rate(n, sizes[m]), 4),
            "eb_abs": h["eb_abs"], "max_err_over_eb": err / h["eb_abs"],
            "psnr_db": round(20 * math.log10(rng / math.sqrt(mse)), 3) if mse > 0 else None,
            "n_outliers": h["n_outliers"], "n_patches": h["n_patches"], "n_regression_blocks": h["n_reg"],
            "compress_gbps": round(4.0 * n / (tc * 1e-3) / 1e9, 2),
            "decompress_gbps": round(4.0 * n / (td * 1e-3) / 1e9, 2),
            "call_roofline": {"compress": _roof(call_bytes("compress", m, n, sizes[m]), tc),
                              "decompress": _roof(call_bytes("decompress", m, n, sizes[m]), td)},
            "eq1_speedup_at_35.7GBps": round(metrics.overall_speedup(LINK_GBPS, cr, 4.0 * n / (tc * 1e-3) / 1e9), 3),
        }
    del xd
    selector_vs = None
    if all(m in modes for m in ("lorenzo1", "selector", "trial")):
        selector_vs = selector_summary(ctx, fz, x, modes)


    # the bit-shuffle codec (FZMod-Speed) on the same field
    print("[bench] bit-shuffle codec", file=sys.stderr, flush=True)
    sbuf = outs[MODES[-1][0]]
    cs = ctx.compress(x, C3_EB, fz.EB_REL, out=sbuf, codec="shuffle")
    ssize = cs.numel()
    shdr = cs[:128].cpu().numpy().tobytes()
    ctx.decompress(cs, header=shdr, out=rec)
    tc = _call_ms(ctx, lambda: ctx.compress(x, C3_EB, fz.EB_REL, out=sbuf, codec="shuffle"))
    td = _call_ms(ctx, lambda: ctx.decompress(sbuf[:ssize], header=shdr, out=rec))
    sh = fz.header_fields(shdr)
    shuffle_mode = {
        "bytes": ssize, "cr": round(metrics.compression_ratio(n, ssize), 4),
        "max_err_over_eb": (rec.double() - x.double()).abs().max().item() / sh["eb_abs"],
        "compress_gbps": round(4.0 * n / (tc * 1e-3) / 1e9, 2),
        "decompress_gbps": round(4.0 * n / (td * 1e-3) / 1e9, 2),
        "call_roofline": {"compress": _roof(call_bytes("compress", "shuffle", n, ssize), tc),
                          "decompress": _roof(call_bytes("decompress", "shuffle", n, ssize), td)}}

    # the interpolation predictor (FZMod-Quality front end) on the same field
    print("[bench] interpolation predictor", file=sys.stderr, flush=True)
    interp_mode = quality_mode(ctx, fz, metrics, x, C3_EB, sbuf, rec)
    print("[bench] global Lorenzo", file=sys.stderr, flush=True)
    global_mode = quality_mode(ctx, fz, metrics, x, C3_EB, sbuf, rec, pred=fz.PRED_GLOBAL)

    # dominant first-order Lorenzo kernel and its roofline (HIP events
    # around it inside the timed region)
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

    # the same field with the bound taken from its range before the spikes
    # (absolute bound 1e-4 x that range): the selector on the structure
    extras = {}
    if not args.no_extras:
        print("[bench] C3' (bound from the range without the spikes)", file=sys.stderr, flush=True)
        eb_abs = C3_EB * base_range
        c3p = {}
        for m, pred in MODES:
            tc = _call_ms(ctx, lambda: ctx.compress(x, eb_abs, fz.EB_ABS, out=outs[m], pred=pred), reps=2)
            size = int(fz.header_fields(outs[m][:128].cpu().numpy().tobytes())["total"])
            c3p[m] = {"bytes": size, "cr": round(metrics.compression_ratio(n, size), 4),
                      "compress_gbps": round(4.0 * n / (tc * 1e-3) / 1e9, 2),
                      "compress_call_roofline": _roof(call_bytes("compress", m, n, size, rel=False), tc)}
        extras["c3_prime"] = {"eb_abs": eb_abs, "range_without_spikes": base_range, "modes": c3p}
        if all(m in c3p for m in ("lorenzo1", "selector", "trial")):
            extras["c3_prime"]["cr_selector_over_trial"] = round(c3p["selector"]["cr"] / c3p["trial"]["cr"], 4)
            extras["c3_prime"]["cr_selector_over_lorenzo1"] = round(c3p["selector"]["cr"] / c3p["lorenzo1"]["cr"], 4)

    cpu = None
    if not args.no_cpu_baseline:
        w = ctx.selector_get() if "selector" in names else None
        slabs_needed = _cpu_threads()
        nz = shape[0]
        slab = max(1, min(32, nz // max(1, slabs_needed)))
        host_slabs = [x[k * slab:(k + 1) * slab].cpu().numpy() for k in range(min(slabs_needed, nz // slab))]
    del x, outs, rec
    torch.cuda.empty_cache()
    if not args.no_extras:
        extras["c2_512cubed"] = c2_extra(ctx, fz, metrics, dev)
        extras["graph_mode"] = graph_extra(fz, dev)
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(host_slabs, w, shape)

    value = len(MODES) * 4.0 * n * args.steps / wall / 1e9
    line = {
        "metric": "compress/decompress GB/s and % HBM roofline on 1 MI355X; ratio at fixed eb",
        "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, shape))} k^-11/3 field + 64 tanh fronts + 1% log-normal spikes, "
                               "rel eb 1e-4; one compress + decompress round trip per predictor mode (first-order "
                               "Lorenzo; learned per-8^3-block selector of first/second-order Lorenzo or "
                               "regression; exhaustive per-block trial), radius 512, Huffman",
                   "n_values": n, "eb_rel": C3_EB, "modes": [m for m, _ in MODES]},
        "modes": modes,
        "shuffle_codec": shuffle_mode,
        "interp_predictor": interp_mode,
        "global_lorenzo": global_mode,
        "selector": selector_vs,
        "training": training,
        "stages": stage_summary,
        "stages_timed_in": "the last warmup step (every stage, first-order Lorenzo); the timed steps time the "
                           "dominant stage alone" if warm else "timed steps",
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


def selector_summary(ctx, fz, x, modes):
    """The learned selector against trial and first-order Lorenzo on the
    1024^3 field: ratios, speeds, and the selection stage alone."""
    p0, sel, tri = modes["lorenzo1"], modes["selector"], modes["trial"]
    selector_vs = {
        "cr_selector_over_trial": round(sel["cr"] / tri["cr"], 4),
        "cr_selector_over_lorenzo1": round(sel["cr"] / p0["cr"], 4),
        "compress_speed_selector_over_trial": round(sel["compress_gbps"] / tri["compress_gbps"], 3),
        "compress_speed_selector_over_lorenzo1": round(sel["compress_gbps"] / p0["compress_gbps"], 3),
    }
    # the selection stage alone: the selector's sample features + network
    # against trial's first-order pass, reference code and cost pass
    print("[bench] selection stage alone", file=sys.stderr, flush=True)
    t_sel = _timed(lambda: ctx.block_select(x, C3_EB, fz.EB_REL), 3, 1)
    t_tri = _timed(lambda: ctx.block_trial(x, C3_EB, fz.EB_REL), 3, 1)
    ch_sel, _ = ctx.block_select(x, C3_EB, fz.EB_REL)
    ch_tri, _ = ctx.block_trial(x, C3_EB, fz.EB_REL)
    selector_vs["selection_stage"] = {
        "selector_ms": round(t_sel * 1e3, 3), "trial_ms": round(t_tri * 1e3, 3),
        "speed_selector_over_trial": round(t_tri / t_sel, 3),
        "agreement_with_trial": round(float((ch_sel == ch_tri).float().mean().item()), 4),
        "selector_choice_counts": [int((ch_sel == k).sum().item()) for k in range(3)],
        "trial_choice_counts": [int((ch_tri == k).sum().item()) for k in range(3)]}
    del ch_sel, ch_tri
    return selector_vs


def quality_mode(ctx, fz, metrics, x, eb, buf, rec, pred=None):
    """One field through a whole-field predictor (the interpolation
    predictor by default, or global Lorenzo; Huffman codec): ratio, error,
    PSNR, whole-call rates and rooflines.  The algorithmic bytes are
    first-order Lorenzo's (the method reads the field once for the
    prediction and writes it once on decompression; halo reads and the
    decoder's residual and prefix-sum passes are implementation traffic)."""
    pred = fz.PRED_INTERP if pred is None else pred
    n = x.numel()
    c = ctx.compress(x, eb, fz.EB_REL, out=buf, pred=pred)
    size = c.numel()
    hdr = c[:128].cpu().numpy().tobytes()
    ctx.decompress(c, header=hdr, out=rec)
    tc = _call_ms(ctx, lambda: ctx.compress(x, eb, fz.EB_REL, out=buf, pred=pred))
    td = _call_ms(ctx, lambda: ctx.decompress(buf[:size], header=hdr, out=rec))
    h = fz.header_fields(hdr)
    diff = rec.double() - x.double()
    err = diff.abs().max().item()
    mse = (diff * diff).mean().item()
    del diff
    rng = float(x.max()) - float(x.min())
    return {"bytes": size, "cr": round(metrics.compression_ratio(n, size), 4),
            "max_err_over_eb": err / h["eb_abs"],
            "psnr_db": round(20 * math.log10(rng / math.sqrt(mse)), 3) if mse > 0 else None,
            "n_outliers": h["n_outliers"],
            "compress_gbps": round(4.0 * n / (tc * 1e-3) / 1e9, 2),
            "decompress_gbps": round(4.0 * n / (td * 1e-3) / 1e9, 2),
            "call_roofline": {"compress": _roof(call_bytes("compress", "lorenzo1", n, size), tc),
                              "decompress": _roof(call_bytes("decompress", "lorenzo1", n, size), td)}}


def c2_extra(ctx, fz, metrics, dev):
    """The 512^3 k^-3 field at rel 1e-2/1e-3/1e-4, first-order Lorenzo:
    whole-call rates and rooflines per bound."""
    import torch

    from inputs import fields
    shape = (512, 512, 512)
    print("[bench] 512^3 k^-3 field", file=sys.stderr, flush=True)
    x = torch.from_numpy(fields.grf(shape, alpha=3.0, seed=2)).to(dev)
    n = x.numel()
    out = torch.empty(ctx.compress_bound(shape), dtype=torch.uint8, device=dev)
    out2 = torch.empty_like(out)
    rec = torch.empty_like(x)
    rows = []
    for eb in EBS:
        for _ in range(2):
            c = ctx.compress(x, eb, fz.EB_REL, out=out)
            hdr = c[:128].cpu().numpy().tobytes()
            ctx.decompress(c, header=hdr, out=rec)
        size = c.numel()
        tc = _call_ms(ctx, lambda: ctx.compress(x, eb, fz.EB_REL, out=out))
        td = _call_ms(ctx, lambda: ctx.decompress(out[:size], header=hdr, out=rec))
        h = fz.header_fields(hdr)
        # the bit-shuffle codec at the same bound (separate output buffer)
        cs = ctx.compress(x, eb, fz.EB_REL, out=out2, codec="shuffle")
        ssize = cs.numel()
        shdr = cs[:128].cpu().numpy().tobytes()
        ctx.decompress(cs, header=shdr, out=rec)
        stc = _call_ms(ctx, lambda: ctx.compress(x, eb, fz.EB_REL, out=out2, codec="shuffle"))
        std = _call_ms(ctx, lambda: ctx.decompress(out2[:ssize], header=shdr, out=rec))
        shuffle = {"bytes": ssize, "cr": round(metrics.compression_ratio(n, ssize), 4),
                   "compress_gbps": round(4.0 * n / (stc * 1e-3) / 1e9, 2),
                   "decompress_gbps": round(4.0 * n / (std * 1e-3) / 1e9, 2),
                   "call_roofline": {"compress": _roof(call_bytes("compress", "shuffle", n, ssize), stc),
                                     "decompress": _roof(call_bytes("decompress", "shuffle", n, ssize), std)}}
        interp = quality_mode(ctx, fz, metrics, x, eb, out2, rec)
        glob = quality_mode(ctx, fz, metrics, x, eb, out2, rec, pred=fz.PRED_GLOBAL)
        ctx.decompress(out[:size], header=hdr, out=rec)
        rows.append({"eb_rel": eb, "bytes": size, "cr": round(metrics.compression_ratio(n, size), 4),
                     "max_err_over_eb": (rec.double() - x.double()).abs().max().item() / h["eb_abs"],
                     "n_outliers": h["n_outliers"], "n_patches": h["n_patches"],
                     "compress_gbps": round(4.0 * n / (tc * 1e-3) / 1e9, 2),
                     "decompress_gbps": round(4.0 * n / (td * 1e-3) / 1e9, 2),
                     "call_roofline": {"compress": _roof(call_bytes("compress", "lorenzo1", n, size), tc),
                                       "decompress": _roof(call_bytes("decompress", "lorenzo1", n, size), td)},
                     "shuffle_codec": shuffle, "interp_predictor": interp, "global_lorenzo": glob})
    del x, out, out2, rec
    torch.cuda.empty_cache()
    return {"workload": "512x512x512 k^-3 Gaussian random field, first-order Lorenzo", "per_eb": rows}


def graph_extra(fz, dev):
    """Eager calls against graph mode (stage tasks captured with concurrent
    branches, replayed): the calls' GPU time (events around each whole
    call) and host wall time, small to mid-size fields at rel 1e-3."""
    import torch

    from inputs import fields
    rows = []
    for shape in ((64, 64, 64), (128, 128, 128), (256, 256, 256)):
        x = torch.from_numpy(fields.grf(shape, alpha=3.0, seed=2)).to(dev)
        row = {"shape": list(shape)}
        for mode, streams in (("eager", 0), ("graph_one_stream", 1), ("graph", 4)):
            ctx = fz.Context(0)
            ctx.set_graph_mode(streams)
            out = torch.empty(ctx.compress_bound(shape), dtype=torch.uint8, device=dev)
            y = torch.empty_like(x)
            c = ctx.compress(x, 1e-3, fz.EB_REL, out=out)
            hdr = c[:128].cpu().numpy().tobytes()
            ctx.decompress(c, header=hdr, out=y)
            tc = _call_ms(ctx, lambda: ctx.compress(x, 1e-3, fz.EB_REL, out=out), reps=10)
            td = _call_ms(ctx, lambda: ctx.decompress(c, header=hdr, out=y), reps=10)
            wc = _timed(lambda: ctx.compress(x, 1e-3, fz.EB_REL, out=out), 20, 3)
            wd = _timed(lambda: ctx.decompress(c, header=hdr, out=y), 20, 3)
            row[mode] = {"compress_gpu_us": round(tc * 1e3, 1), "decompress_gpu_us": round(td * 1e3, 1),
                         "compress_wall_us": round(wc * 1e6, 1), "decompress_wall_us": round(wd * 1e6, 1)}
            ctx.close()
        rows.append(row)
    return {"eb_rel": 1e-3, "fields": "k^-3 Gaussian random fields", "rows": rows}


def bench_c2(args):
    """The 512^3 field alone, as its own line (round trips at three bounds)."""
    import torch

    from paper_2509_20563_amd import fz, metrics
    dev = torch.device("cuda", 0)
    ctx = fz.Context(0)
    t = time.perf_counter()
    r = c2_extra(ctx, fz, metrics, dev)
    dt = time.perf_counter() - t
    per = r["per_eb"]
    n = 512 ** 3
    ms = sum(row["call_roofline"]["compress"]["avg_call_ms"] + row["call_roofline"]["decompress"]["avg_call_ms"]
             for row in per)
    _line("compress/decompress GB/s and % HBM roofline on 1 MI355X; ratio at fixed eb", 3 * 4.0 * n / (ms * 1e-3) / 1e9,
          "GB/s", args, ms, {"workload": r["workload"] + ", rel eb 1e-2/1e-3/1e-4, one round trip per bound",
                             "n_values": n}, per_eb=per, seconds=round(dt, 2))


def _cpu_threads():
    n = os.environ.get("OMP_NUM_THREADS")
    try:
        t = int(n) if n else (os.cpu_count() or 1)
    except ValueError:
        t = os.cpu_count() or 1
    return max(1, min(t, 32))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(slabs, w, shape):
    """The CPU oracle as it is (plain C, one thread per call) on slabs of the
    same field: one slab single-threaded, then one slab per thread run
    concurrently; each slab is a field of its own (its own range and
    containers), round trips in the three predictor modes."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    preds = (0, 3, 4) if w is not None else (0, 4)

    def roundtrip(s):
        for pred in preds:
            if pred == 3:
                f = oracle.features(s, C3_EB, 1)
                _, ch = oracle.mlp_infer(w, f)
                c = oracle.compress(s, C3_EB, 1, pred=3, choice=ch)
            else:
                c = oracle.compress(s, C3_EB, 1, pred=pred)
            oracle.decompress(c)
        return len(preds) * 4.0 * s.size

    print(f"[bench] cpu baseline: {len(slabs)} slabs of {slabs[0].shape}", file=sys.stderr, flush=True)
    t = time.perf_counter()
    b1 = roundtrip(slabs[0])
    t1 = time.perf_counter() - t
    threads = len(slabs)
    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        bn = sum(ex.map(roundtrip, slabs))
    tn = time.perf_counter() - t
    return {"value": round(bn / tn / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{threads} slabs of {slabs[0].shape[0]} z-planes ({'x'.join(map(str, slabs[0].shape))}) of the "
                      f"{'x'.join(map(str, shape))} field, each a field of its own at rel eb 1e-4, compress + "
                      "decompress with first-order Lorenzo, the selector's choices (oracle features and network) "
                      "and exhaustive trial; the plain C oracle, one call per thread, threads run concurrently",
            "seconds": round(tn, 2), "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": round(b1 / t1 / 1e9, 4), "unit": "GB/s", "cores": 1,
                              "seconds": round(t1, 2)}}


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


# training fields: every family of the evaluated workloads, seeds disjoint
# from the evaluation seeds (2, 3, 4000+, 5000+)
TRAIN_FIELDS = (
    [("fronts_spikes", (128, 128, 128), sd, None) for sd in (101, 102, 103, 104)]
    + [("grf3", (128, 128, 128), sd, a) for sd, a in ((111, 3.0), (112, 3.0), (113, 11.0 / 3.0), (114, 5.0))]
    + [("grf2", (1024, 1024), sd, 3.0) for sd in (121, 122)]
    + [("positions", (1 << 21,), sd, None) for sd in (131, 132)])
TRAIN_EBS = (1e-2, 1e-3, 1e-4, 1e-5)


def train_selector(ctx, fz, device, epochs=200):
    """Train the context's selector on the training fields (features and
    trial costs from the library); returns a summary dict."""
    import torch
    from inputs import fields_gpu
    feats, costs = [], []
    t0 = time.perf_counter()
    for kind, shape, sd, a in TRAIN_FIELDS:
        if kind == "fronts_spikes":
            x = fields_gpu.fronts_spikes(shape, seed=sd, n_fronts=8, device=device)
        elif kind == "positions":
            x = fields_gpu.sorted_positions(shape[0], seed=sd, device=device)
        else:
            x = fields_gpu.grf(shape, alpha=a, seed=sd, device=device)
        for eb in TRAIN_EBS:
            feats.append(ctx.block_features(x, eb, fz.EB_REL))
            costs.append(ctx.block_trial(x, eb, fz.EB_REL)[1])
    f = torch.cat(feats).contiguous()
    c = torch.cat(costs).contiguous()
    torch.cuda.synchronize()
    t_lab = time.perf_counter() - t0
    t = time.perf_counter()
    loss = ctx.selector_train(f, c, epochs=epochs, batch=1024, seed=1)
    torch.cuda.synchronize()
    return {"seconds": round(time.perf_counter() - t, 2), "labelling_seconds": round(t_lab, 2),
            "samples": int(f.shape[0]), "loss_first_epoch": float(loss[0]), "loss_last_epoch": float(loss[-1]),
            "fields": "3D fronts/spikes 128^3 (seeds 101-104), 3D k^-3/k^-11/3/k^-5 128^3 (111-114), "
                      "2D k^-3 1024^2 (121-122), 1D sorted positions 2^21 (131-132); rel eb 1e-2..1e-5"}


def bench_selector(args):
    import torch
    from inputs import fields_gpu
    from paper_2509_20563_amd import fz, metrics
    dev = torch.device("cuda", 0)
    shape = tuple(int(s) for s in (args.shape or "1024,1024,1024").split(","))
    ctx = fz.Context(0)
    print("[bench] training the selector", file=sys.stderr, flush=True)
    training = train_selector(ctx, fz, dev)
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
          training=training)


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
    training = train_selector(ctx, fz, dev)
    print(f"[bench] generating {nf} mixed fields", file=sys.stderr, flush=True)
    batch = fields_gpu.batch_mixed(n_fields=nf, device=dev)
    r0 = _bench_batch(args, fz, ctx, batch, "batchmixed lorenzo1")
    r1 = _bench_batch(args, fz, ctx, batch, "batchmixed selector", preds=[fz.PRED_AUTO_MLP] * nf)
    _line("batched compress GB/s of a mixed 1D/2D/3D batch with the learned selector; CR vs first-order Lorenzo",
          r1["batch_compress_gbps"], "GB/s", args, r1["ms_batch_compress"],
          {"workload": f"{nf} fields: 1D sorted positions 1M-64M values, 2D k^-3 (as the 2D batch), 3D 64^3-384^3 "
                       "k^-3..k^-5; rel eb log-uniform 1e-5..1e-2", "n_values": r1["n_values"]},
          selector=r1, lorenzo1=r0, cr_gain_over_lorenzo1=round(r1["cr"] / r0["cr"], 4),
          training=training)


if __name__ == "__main__":
    main()
