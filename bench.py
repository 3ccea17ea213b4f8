#!/usr/bin/env python3
"""Throughput of the fused wave-tiled unsharp-mask pipeline on one MI355X.

Workload: 4-stage unsharp mask (5-tap binomial blur in x, blur in y,
sharpen = img + 1.5 (img - blur), select(|img - blur| < 0.01, img, sharpen))
on a 3x2048x2048 FP32 image, pixels uniform in [0, 1) from a seeded
splitmix64 stream.  One step = one run of the whole pipeline over the image.

value = output Mpixels/s of the fused path (one kernel per step), with the
inputs resident in HBM.  Input/output buffer sets rotate over more than the
256 MB Infinity Cache so each step reads from and writes to HBM.  The unfused
path (one kernel per stage, intermediates through HBM), the FP16-intermediate
variant and the FP64 oracle on the host cores are reported beside it.

Roofline: algorithmic bytes = 12 B in + 12 B out per output pixel (3 FP32
channels), divided by the fused kernel's average duration over the timed
region (HIP events on the launch stream), against MI355X's 8 TB/s HBM peak.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixels/s per pipeline, fused vs unfused on 1 GPU; % of HBM roofline"
C, H, W = 3, 2048, 2048
BYTES_PER_PX = 24  # 3 channels x (4 B in + 4 B out)
HBM_PEAK_GBS = 8000.0
OTPTB_FUSED = "nodes=1,2,3,4 V=1 TX=1 TY=16 WPB=4 BLK=1"
DEFAULT_FUSED = "nodes=1,2,3,4 V=2 TX=1 SX=0 TY=32 PF=2 NT=1"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_sets(torch, img, nsets):
    dev = torch.device("cuda:0")
    base = torch.from_numpy(img).to(dev)
    ins, outs = [], []
    for i in range(nsets):
        x = base.clone() if i else base
        ins.append(x)
        outs.append(torch.empty_like(x))
    return ins, outs


def calibrate_sleep(torch):
    """GPU spin cycles per millisecond of torch.cuda._sleep."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    torch.cuda._sleep(10_000_000)
    e1.record(s)
    torch.cuda.synchronize()
    ms = max(e0.elapsed_time(e1), 1e-3)
    return 10_000_000 / ms


def time_plan(torch, plan, ins, outs, steps, warmup, cycles_per_ms):
    """Average ms per step over `steps` back-to-back runs on the current
    stream.  The stream is held by a GPU spin while the launches are queued,
    so host launch overhead does not appear as gaps between kernels."""
    n = len(ins)
    t0 = time.perf_counter()
    for i in range(warmup):
        plan.run([ins[i % n]], [outs[i % n]])
    torch.cuda.synchronize()
    host_ms = (time.perf_counter() - t0) * 1e3 / max(warmup, 1)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    torch.cuda._sleep(int(cycles_per_ms * (host_ms * steps * 1.5 + 5.0)))
    e0.record(s)
    for i in range(steps):
        plan.run([ins[i % n]], [outs[i % n]])
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def copy_reference(torch, ins, outs, steps, cycles_per_ms):
    """HBM bandwidth of a plain device copy of the same buffers (read + write
    of one 3x2048x2048 FP32 image per step), timed like the pipeline."""
    n = len(ins)
    for i in range(5):
        outs[i % n].copy_(ins[i % n])
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(int(cycles_per_ms * 5.0))
    e0.record(s)
    for i in range(steps):
        outs[i % n].copy_(ins[i % n])
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nbytes = 2 * ins[0].numel() * ins[0].element_size()
    # the library's streaming copy (16 B per thread, nontemporal), same buffers
    import paper_1909_07190_amd as wt
    for i in range(5):
        wt.stream_copy(ins[i % n], outs[i % n])
    torch.cuda.synchronize()
    torch.cuda._sleep(int(cycles_per_ms * (0.05 * steps + 5.0)))  # covers the host's enqueue time
    e0.record(s)
    for i in range(steps):
        wt.stream_copy(ins[i % n], outs[i % n], s)
    e1.record(s)
    torch.cuda.synchronize()
    ms_s = e0.elapsed_time(e1) / steps
    return {"GB/s": nbytes / (ms * 1e-3) / 1e9, "us_per_copy": ms * 1e3, "bytes": nbytes,
            "streaming_GB/s": nbytes / (ms_s * 1e-3) / 1e9, "streaming_us_per_copy": ms_s * 1e3}


def cpu_baseline(img, seconds=10.0):
    """The FP64 oracle, as it stands, on a band of rows of the same image."""
    import numpy as np
    import oracle
    from synth import pipelines as P
    spec = P.unsharp_mask()
    rows = 128
    band = np.ascontiguousarray(img[:, :rows, :])
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.evaluate(spec, {"img": band})
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    per = el / n
    return {"value": rows * W / per / 1e6, "unit": "Mpixels/s", "cores": 1, "kind": "oracle",
            "sample": f"rows 0..{rows - 1} of the 3x{H}x{W} input ({n} runs, {el:.1f} s; "
                      "numpy float64, single-threaded)"}


def bench_other(args, torch, wt, synth, P):
    """Secondary workloads (same timing method), one JSON line each."""
    import numpy as np
    cyc = calibrate_sleep(torch)
    dev = torch.device("cuda:0")
    res = {"workload": args.workload}
    if args.workload in ("harris", "blur"):
        if args.workload == "harris":
            C_, H_, W_, spec, seed = 3, 4096, 4096, P.harris(), 3
            img = synth.white_squares(synth.uniform_image(seed, C_, H_, W_), seed, count=200)
            bpp = 16  # 12 B RGB in + 4 B out
        else:
            C_, H_, W_, spec, seed = 1, 256, 256, P.gaussian_blur(), 1
            img = synth.uniform_image(seed, C_, H_, W_)
            bpp = 8
        base = torch.from_numpy(img).to(dev)
        nsets = max(2, min(8, int(1.2e9 // (base.numel() * 4 * 1.33)) or 2))
        ins = [base.clone() for _ in range(nsets)]
        outs = [torch.empty((1, H_, W_), device=dev) for _ in range(nsets)]
        legs = (("autotune", True, None), ("autotune", False, None), ("mlp", False, None),
                ("autotune", False, wt.GFX950_COST_MODEL), ("unfused", False, None))
        for mode, fp16, model in legs:
            plan = wt.from_spec(spec).plan(W_, H_, mode=mode, fp16=fp16, model_path=model)
            ms = time_plan(torch, plan, ins, outs, args.steps, args.warmup, cyc)
            key = f"{'mlp_' if model else ''}{mode}{'_fp16' if fp16 else ''}"
            res[key] = {"Mpix/s": H_ * W_ / (ms * 1e-3) / 1e6, "us": ms * 1e3,
                        "GB/s_algorithmic": bpp * H_ * W_ / (ms * 1e-3) / 1e9,
                        "kernels": plan.num_groups, "schedule": plan.describe().strip()}
            log(f"{args.workload} {key}: {ms * 1e3:.1f} us, {res[key]['GB/s_algorithmic']:.0f} GB/s")
    elif args.workload == "pyramid":
        spec = P.pyramid_blend(4)
        sizes = synth.batch_sizes(4, 64)
        ins, outs, px = [], [], 0
        for i, (w, h) in enumerate(sizes):
            a = torch.from_numpy(synth.uniform_image(4000 + 2 * i, 1, h, w)).to(dev)
            b = torch.from_numpy(synth.uniform_image(4001 + 2 * i, 1, h, w)).to(dev)
            m = torch.from_numpy(synth.ramp_mask(h, w)).to(dev)
            ins.append([a, b, m])
            outs.append([torch.empty((1, h, w), device=dev)])
            px += w * h
        # plans are scheduled (and autotuned) at the median image size
        mw, mh = sorted(sizes, key=lambda s: s[0] * s[1])[len(sizes) // 2]
        legs = (("autotune", None), ("autotune", wt.GFX950_COST_MODEL), ("mlp", None), ("analytic", None),
                ("unfused", None))
        for mode, model in legs:
            plan = wt.from_spec(spec).plan(mw, mh, mode=mode, any_width=True, batch_images=len(sizes),
                                           model_path=model)
            key = f"mlp_{mode}" if model else mode
            for _ in range(2):
                plan.run_batch(ins, outs)
            torch.cuda.synchronize()
            s = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            # median of 5 samples of 3 batches each: a rare multi-millisecond
            # stall of a single launch does not decide the figure
            reps, samples = 3, []
            for _ in range(5):
                e0.record(s)
                for _ in range(reps):
                    plan.run_batch(ins, outs)
                e1.record(s)
                torch.cuda.synchronize()
                samples.append(e0.elapsed_time(e1) / reps)
            ms = sorted(samples)[len(samples) // 2]
            res[key] = {"Mpix/s": px / (ms * 1e-3) / 1e6, "ms": ms, "ms_samples": samples,
                        "groups": plan.num_groups, "GB/s_algorithmic": 16 * px / (ms * 1e-3) / 1e9,
                        "schedule": plan.describe().strip()}
            log(f"pyramid batch {key}: {ms:.2f} ms, {res[key]['Mpix/s']:.0f} Mpix/s, {plan.num_groups} launches")
            # the same schedule, one plan per image size, images run one by one
            fixed = plan.describe()
            plans = [wt.from_spec(spec).plan(w, h, mode="fixed", fixed=fixed, any_width=True) for (w, h) in sizes]
            for pl, i, o in zip(plans, ins, outs):
                pl.run(i, o)
            torch.cuda.synchronize()
            e0.record(s)
            for _ in range(reps):
                for pl, i, o in zip(plans, ins, outs):
                    pl.run(i, o)
            e1.record(s)
            torch.cuda.synchronize()
            ms1 = e0.elapsed_time(e1) / reps
            res[key]["per_image_ms"] = ms1
            log(f"pyramid per-image {key}: {ms1:.2f} ms, {px / (ms1 * 1e-3) / 1e6:.0f} Mpix/s")
            del plans
        res["pixels"] = px
    print(json.dumps(res), flush=True)


def profile_traffic(kname):
    """HBM bytes per launch of kernel `kname` from the committed rocprofv3
    counter summaries (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each
    scaled by what the counter reads for a copy kernel of known size), or
    None when no summary covers this exact kernel (its name carries a hash of
    its source, so a changed kernel has no figure until it is profiled)."""
    import glob
    import re
    pat = re.compile(r"^traffic (\S+) fetch_kib=([\d.]+) write_kib=([\d.]+) "
                     r"fetch_scale=([\d.]+) write_scale=([\d.]+)\s*$")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            m = pat.match(line.strip())
            if m and m.group(1) == kname:
                f, w, fs, ws = (float(m.group(i)) for i in range(2, 6))
                return (f * fs + w * ws) * 1024.0
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--mode", default="fixed", help="schedule mode of the fused path")
    ap.add_argument("--schedule", default=DEFAULT_FUSED, help="fixed schedule of the fused path")
    ap.add_argument("--sets", type=int, default=6, help="rotating buffer sets (>256 MB total)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the unfused and FP16 legs")
    ap.add_argument("--workload", default="unsharp", choices=["unsharp", "harris", "blur", "pyramid"],
                    help="unsharp (default, the reported metric) or a secondary workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (tiles and images "
              "are independent, so a batch or the tile rows of an image would be split across "
              "GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1909_07190_amd as wt
    import synth
    from synth import pipelines as P

    if args.workload != "unsharp":
        return bench_other(args, torch, wt, synth, P)
    img = synth.uniform_image(2, C, H, W)
    ins, outs = make_sets(torch, img, args.sets)
    cyc = calibrate_sleep(torch)
    spec = P.unsharp_mask()
    fixed = args.schedule if args.mode == "fixed" else None

    log(f"fused plan ({args.mode}: {fixed})")
    fused = wt.from_spec(spec).plan(W, H, mode=args.mode, fixed=fixed)
    ms = time_plan(torch, fused, ins, outs, args.steps, args.warmup, cyc)
    mpix = H * W / (ms * 1e-3) / 1e6
    achieved = BYTES_PER_PX * H * W / (ms * 1e-3) / 1e9
    log(f"fused: {ms * 1e3:.2f} us/step, {mpix:.0f} Mpix/s, {achieved:.0f} GB/s")
    ref_out = outs[(args.steps - 1) % len(outs)].clone()

    extra = {}
    if not args.no_extra:
        unf = wt.from_spec(spec).plan(W, H, mode="unfused")
        ms_u = time_plan(torch, unf, ins, outs, args.steps, args.warmup, cyc)
        chk = outs[(args.steps - 1) % len(outs)]
        diff = float((chk - ref_out).abs().max() / ref_out.abs().max())
        extra["unfused"] = {"value": H * W / (ms_u * 1e-3) / 1e6, "ms_per_step": ms_u,
                            "kernels_per_step": unf.num_groups, "fused_speedup": ms_u / ms,
                            "max_rel_diff_vs_fused": diff}
        log(f"unfused: {ms_u * 1e3:.2f} us/step ({unf.num_groups} kernels), fused speedup {ms_u / ms:.2f}x")
        f16 = wt.from_spec(spec).plan(W, H, mode="fixed", fixed=(fixed or DEFAULT_FUSED) + " fp16=1",
                                      fp16=True)
        ms_h = time_plan(torch, f16, ins, outs, args.steps, args.warmup, cyc)
        extra["fp16_intermediates"] = {"value": H * W / (ms_h * 1e-3) / 1e6, "ms_per_step": ms_h}
        log(f"fp16 intermediates: {ms_h * 1e3:.2f} us/step")
        # the paper's baseline execution model: one overlapped tile per
        # workgroup, stages in LDS with workgroup barriers (same fusion)
        blk = wt.from_spec(spec).plan(W, H, mode="fixed", fixed=OTPTB_FUSED)
        ms_b = time_plan(torch, blk, ins, outs, args.steps, args.warmup, cyc)
        extra["one_tile_per_workgroup"] = {"value": H * W / (ms_b * 1e-3) / 1e6, "ms_per_step": ms_b,
                                           "schedule": OTPTB_FUSED, "wave_tile_speedup": ms_b / ms}
        log(f"one tile per workgroup: {ms_b * 1e3:.2f} us/step, wave tiles {ms_b / ms:.2f}x faster")
        # what the schedulers choose for this pipeline on their own
        sched = {}
        for mode in ("mlp", "analytic"):
            pl = wt.from_spec(spec).plan(W, H, mode=mode)
            ms_s = time_plan(torch, pl, ins, outs, args.steps, args.warmup, cyc)
            sched[mode] = {"value": H * W / (ms_s * 1e-3) / 1e6, "ms_per_step": ms_s,
                           "schedule": pl.describe().strip()}
            log(f"{mode} schedule: {ms_s * 1e3:.2f} us/step ({pl.describe().strip()})")
        extra["schedulers"] = sched
    copy = copy_reference(torch, ins, outs, args.steps, cyc)
    log(f"device copy reference: {copy['GB/s']:.0f} GB/s (runtime copy), "
        f"{copy['streaming_GB/s']:.0f} GB/s (streaming copy kernel)")
    cpu = None if args.no_cpu else cpu_baseline(img)
    if cpu:
        log(f"oracle: {cpu['value']:.2f} Mpix/s on {cpu['cores']} core(s)")

    import re
    kname = re.search(r"wt_g0_fused_[0-9a-f]+", fused.source(0)).group(0)
    traffic = profile_traffic(kname)
    out = {
        "metric": METRIC, "value": mpix, "unit": "Mpixels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "unsharp mask 3x2048x2048 FP32, uniform [0,1) seed 2; "
                               "blur x, blur y, sharpen, select fused in one wave-tiled kernel",
                   "schedule": fused.describe().strip(), "kernel": kname, "buffer_sets": args.sets},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "cpu_baseline": cpu,
    }
    out["copy_reference"] = copy
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
