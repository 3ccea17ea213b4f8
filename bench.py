#!/usr/bin/env python3
"""Throughput of fused wave-tiled stencil pipelines on one MI355X.

Headline workload: the batched four-level Laplacian-pyramid blend -- 64
image pairs (A, B) with each side uniform in 512..4096 (seeded), FP32
uniform in [0, 1), a ramp mask per pair; per level a 5-tap binomial blur
in x and y with 2x decimation, 2x expansion and subtraction for the
Laplacian bands, the bands blended under the mask's Gaussian pyramid and
collapsed.  The plan is the autotuner's: the fusion search (with the cost
network shipped with the package ranking groupings and tile configurations)
proposes groupings with and without folded expansions, the candidates'
configurations are timed on the device and the faster measured plan is kept;
every group runs as one launch over the tiles of all 64 pairs, the sequence
replayed from a hipGraph.  One step = one run of the whole batch.

value = level-0 output Mpixels/s of the batch (inputs resident in HBM).
Beside it: the same batch unfused and planned by the analytical and the
learned cost models alone;
the unsharp mask on 3x2048x2048 and the Harris corner response on
3x4096x4096 (each fused, unfused, with FP16 intermediates, and the
unsharp mask also as one tile per workgroup, the paper's baseline); the FP64
oracle on the host cores; a streaming device copy as the achievable
bandwidth.

Roofline: the dominant kernel of the headline plan (the group with the
longest launch) is timed on its own with HIP events on the stream it runs
on (the library launches groups of a batched run directly for this); its
achieved bandwidth is its algorithmic bytes (every buffer it reads or
writes, once, at the buffer's pyramid level, summed over the batch)
divided by that time, against MI355X's 8 TB/s.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixels/s per pipeline, fused vs unfused on 1 GPU; % of HBM roofline"
HBM_PEAK_GBS = 8000.0
# headline workload: 64 pyramid-blend pairs, sides uniform in 512..4096
PYR_LEVELS, PYR_PAIRS, PYR_SEED = 4, 64, 4
HEADLINE_MODE = "autotune"  # ranked by the shipped cost network
# secondary workloads: (channels, height, width, input seed)
UNSHARP = (3, 2048, 2048, 2)
HARRIS = (3, 4096, 4096, 3)
HIST_WORKLOAD = (3, 2048, 2048, 6)  # blur + 256-bin histogram
# the best unsharp-mask schedule found by sweeps, and the paper's baseline
SWEPT_UNSHARP = "nodes=1,2,3,4 V=2 TX=1 SX=0 TY=32 PF=2 NT=1"
OTPTB_UNSHARP = "nodes=1,2,3,4 V=1 TX=1 TY=16 WPB=4 BLK=1"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ inputs --

def pyramid_batch(synth):
    """(sizes, [[A, B, M] per pair] as numpy arrays) of the headline batch."""
    sizes = synth.batch_sizes(PYR_SEED, PYR_PAIRS)
    return sizes, [pyramid_pair(synth, i, w, h) for i, (w, h) in enumerate(sizes)]


def pyramid_pair(synth, i, w, h):
    return [synth.uniform_image(4000 + 2 * i, 1, h, w), synth.uniform_image(4001 + 2 * i, 1, h, w),
            synth.ramp_mask(h, w)]


PITCH = 64  # caller images' row pitch in elements for the pyramid batch


def pitched_empty(torch, c, h, w, dev):
    """A c x h x w device image whose rows start every PITCH elements (a
    strided view of a padded allocation)."""
    p = (w + PITCH - 1) // PITCH * PITCH
    return torch.empty((c, h, p), device=dev)[:, :, :w]


def pitched(torch, x, dev):
    """A device copy of CHW array x with rows on the PITCH pitch."""
    v = pitched_empty(torch, *x.shape, dev)
    v.copy_(torch.from_numpy(x).to(dev))
    return v


def median_size(sizes):
    return sorted(sizes, key=lambda s: s[0] * s[1])[len(sizes) // 2]


def plan_pyramid(wt, P, sizes, mode, model=None, topk=0):
    if mode == "autotune" and model is None:
        model = wt.GFX950_COST_MODEL
    mw, mh = median_size(sizes)
    return wt.from_spec(P.pyramid_blend(PYR_LEVELS)).plan(mw, mh, mode=mode, any_width=True,
                                                          batch_images=len(sizes), model_path=model,
                                                          autotune_topk=topk)


# --------------------------------------------------------- algorithmic bytes --

def node_levels(spec):
    lv = {i["name"]: 0 for i in spec["inputs"]}
    for st in spec["stages"]:
        k = st["kind"]
        src = st["src"] if k in ("stencil", "down2", "up2") else st["srcs"][0]
        lv[st["name"]] = lv[src] + (1 if k == "down2" else -1 if k == "up2" else 0)
    return lv


def node_channels(spec):
    ch = {i["name"]: i["channels"] for i in spec["inputs"]}
    for st in spec["stages"]:
        ch[st["name"]] = st["channels"] if st["kind"] == "pointwise" else ch[st["src"]]
    return ch


def level_dims(w, h, level):
    for _ in range(level):
        w, h = (w + 1) // 2, (h + 1) // 2
    return w, h


ESIZE = {0: 4, 1: 2, 2: 1, 3: 2, 4: 2, 5: 4}  # wt_dtype -> bytes


def group_bytes(wt, plan, pipe, spec, group, sizes):
    """Algorithmic bytes of one launch of `group` over images of `sizes`:
    every buffer it reads (loaded nodes; an expanded up2 reads its coarse
    source) or writes (live-outs and decimated outputs) counted once, at its
    own level's size."""
    import ctypes
    gi = wt.GroupInfo()
    wt._check(wt.lib.wt_plan_group_info(plan._h, group, ctypes.byref(gi)))
    names = {v: k for k, v in pipe.names.items()}
    lv, ch = node_levels(spec), node_channels(spec)
    bufs = [(gi.loaded[i], gi.loaded_dtype[i], gi.loaded_half[i]) for i in range(gi.nloaded)]
    bufs += [(gi.liveouts[i], gi.liveout_dtype[i], gi.liveout_half[i]) for i in range(gi.nliveouts)]
    total = 0
    for nid, dt, half in bufs:
        n = names[nid]
        esz = 2 if half else ESIZE[dt]
        for (w, h) in sizes:
            lw, lh = level_dims(w, h, lv[n])
            total += ch[n] * lw * lh * esz
    return total


# ------------------------------------------------------------------ timing --

def calibrate_sleep(torch):
    """GPU spin cycles per millisecond of torch.cuda._sleep."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    torch.cuda._sleep(10_000_000)
    e1.record(s)
    torch.cuda.synchronize()
    return 10_000_000 / max(e0.elapsed_time(e1), 1e-3)


def timed(torch, fn, steps, warmup, cycles_per_ms, host_ms_hint=0.05):
    """Average ms per call of fn(i) over `steps` back-to-back calls on the
    current stream, bracketed by synchronisations; the stream is held by a
    GPU spin while the calls are queued, so host launch overhead does not
    show as gaps between kernels."""
    t0 = time.perf_counter()
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    host_ms = max(host_ms_hint, (time.perf_counter() - t0) * 1e3 / max(warmup, 1))
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    torch.cuda._sleep(int(cycles_per_ms * (host_ms * steps * 1.5 + 2.0)))
    e0.record(s)
    for i in range(steps):
        fn(i)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def profile_traffic(kname):
    """HBM bytes per launch of kernel `kname` from the committed rocprofv3
    counter summaries (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each
    scaled by what the counter reads for a copy of known size), or None when
    no summary covers this exact kernel (its name carries a hash of its
    source, so a changed kernel has no figure until it is profiled)."""
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


def kernel_name(plan, group, batched):
    import re
    m = re.search(r"wt_g\d+_\w+?_[0-9a-f]{12}", plan.source(group))
    return (m.group(0) + ("_batch" if batched else "")) if m else None


# ------------------------------------------------------------- CPU oracle --

def _oracle_worker(i, w, h, barrier, samples, out):
    import numpy as np  # noqa: F401
    import oracle
    import synth
    from synth import pipelines as P
    a, b, m = pyramid_pair(synth, i, w, h)
    spec = P.pyramid_blend(PYR_LEVELS)
    res = []
    for _ in range(samples):
        barrier.wait()
        t0 = time.monotonic()
        oracle.evaluate(spec, {"A": a, "B": b, "M": m})
        res.append((t0, time.monotonic()))
    out.put((i, res))


def cpu_cores():
    """Host cores this process may use, at most 16 (one GPU's share of the
    host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sizes, samples=3):
    """The FP64 oracle, as it stands, on a sample of the headline batch: the
    first `cores` pairs, one process per pair on all usable host cores
    (started together at a barrier; a sample lasts until the last pair is
    done), and the first pair alone on one core; `samples` samples each, the
    best kept (the minimum of the per-sample times)."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    cores = cpu_cores()

    def run(pairs):
        bar = ctx.Barrier(len(pairs))
        q = ctx.Queue()
        procs = [ctx.Process(target=_oracle_worker, args=(i, w, h, bar, samples, q)) for i, (w, h) in pairs]
        for p in procs:
            p.start()
        res = dict(q.get() for _ in procs)
        for p in procs:
            p.join()
        walls = [max(res[i][s][1] for i, _ in pairs) - min(res[i][s][0] for i, _ in pairs) for s in range(samples)]
        px = sum(w * h for _, (w, h) in pairs)
        return px, min(walls), walls

    env_threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_threads:
        os.environ[k] = "1"
    try:
        pairs = list(enumerate(sizes))[:cores]
        px, best, walls = run(pairs)
        px1, best1, walls1 = run(pairs[:1])
    finally:
        for k, v in env_threads.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return {"value": px / best / 1e6, "unit": "Mpixels/s", "cores": cores, "kind": "oracle",
            "sample": f"pairs 0..{len(pairs) - 1} of the 64-pair batch ({px / 1e6:.1f} Mpx of level-0 output), one "
                      f"process per pair on {cores} cores, numpy float64; best of {samples} samples "
                      f"({', '.join(f'{t:.1f}' for t in walls)} s)",
            "one_core": {"value": px1 / best1 / 1e6, "unit": "Mpixels/s",
                         "sample": f"pair 0 ({sizes[0][0]}x{sizes[0][1]}) on one core, best of {samples} "
                                   f"({', '.join(f'{t:.1f}' for t in walls1)} s)"},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


# ------------------------------------------------------------ workloads --

def bench_pyramid(args, torch, wt, synth, P, cyc):
    dev = torch.device("cuda:0")
    spec = P.pyramid_blend(PYR_LEVELS)
    sizes, host = pyramid_batch(synth)
    # Caller images live with rows on a 64-element (256-byte) pitch, the
    # library's own layout for intermediates: a tile's row segment then
    # starts on a cache line.  The same plan is also timed on dense rows.
    ins = [[pitched(torch, x, dev) for x in pair] for pair in host]
    outs = [[pitched_empty(torch, 1, h, w, dev)] for (w, h) in sizes]
    px = sum(w * h for w, h in sizes)

    def run_mode(mode, model=None):
        plan = plan_pyramid(wt, P, sizes, mode, model)
        if mode == "autotune":
            # the autotuner's last step: its candidates timed on this batch
            t0 = time.time()
            plan.tune_batch(ins, outs)
            torch.cuda.synchronize()
            log(f"pyramid {mode}: tuned on the batch in {time.time() - t0:.1f} s")
        ms = timed(torch, lambda i: plan.run_batch(ins, outs), args.steps, args.warmup, cyc, host_ms_hint=0.5)
        return plan, ms

    log(f"pyramid batch: {len(sizes)} pairs, {px / 1e6:.1f} Mpx; planning ({HEADLINE_MODE})")
    plan, ms = run_mode(HEADLINE_MODE)
    log(f"pyramid {HEADLINE_MODE}: {ms:.3f} ms per batch, {px / (ms * 1e-3) / 1e6:.0f} Mpix/s, "
        f"{plan.num_groups} launches")
    # per-group launch times (each group launched directly, same grid)
    pipe = plan.pipe
    groups = []
    for g in range(plan.num_groups):
        gms = timed(torch, lambda i, g=g: plan.run_batch_groups(g, 1, ins, outs), args.steps, 2, cyc,
                    host_ms_hint=0.5)
        nbytes = group_bytes(wt, plan, pipe, spec, g, sizes)
        groups.append({"group": g, "ms": gms, "bytes": nbytes, "GB/s": nbytes / (gms * 1e-3) / 1e9,
                       "kernel": kernel_name(plan, g, True)})
    dom = max(groups, key=lambda r: r["ms"])
    log(f"dominant kernel g{dom['group']} {dom['kernel']}: {dom['ms']:.3f} ms, {dom['GB/s']:.0f} GB/s algorithmic")
    # the headline plan's output, kept to check the other modes against
    ref = [o[0].clone() for o in outs]
    dense_in = [[torch.from_numpy(x).to(dev) for x in pair] for pair in host]
    dense_out = [[torch.empty((1, h, w), device=dev)] for (w, h) in sizes]
    del host
    dms = timed(torch, lambda i: plan.run_batch(dense_in, dense_out), args.steps, args.warmup, cyc, host_ms_hint=0.5)
    ddiff = max(float((o[0] - r).abs().max() / r.abs().max()) for o, r in zip(dense_out, ref))
    del dense_in, dense_out
    log(f"pyramid {HEADLINE_MODE}, dense rows: {dms:.3f} ms, max rel diff {ddiff:.1e}")

    extra = {"groups": groups,
             "dense_rows": {"value": px / (dms * 1e-3) / 1e6, "ms_per_step": dms, "vs_headline": dms / ms,
                            "max_rel_diff_vs_headline": ddiff}}
    if not args.no_extra:
        legs = (("unfused", None), ("analytic", None), ("mlp", wt.GFX950_COST_MODEL))
        for mode, model in legs:
            pl, mms = run_mode(mode, model)
            key = mode
            diff = max(float((o[0] - r).abs().max() / r.abs().max()) for o, r in zip(outs, ref))
            extra[key] = {"value": px / (mms * 1e-3) / 1e6, "ms_per_step": mms, "launches": pl.num_groups,
                          "vs_headline": mms / ms, "max_rel_diff_vs_headline": diff,
                          "schedule": pl.describe().strip()}
            log(f"pyramid {key}: {mms:.3f} ms ({pl.num_groups} launches), max rel diff {diff:.1e}")
            del pl
    result = {
        "value": px / (ms * 1e-3) / 1e6, "ms_per_step": ms,
        "config": {"workload": f"pyramid blend, {len(sizes)} pairs of uneven sizes (sides uniform in 512..4096, "
                               f"seed {PYR_SEED}), FP32 uniform [0,1) and a ramp mask, rows on a {PITCH}-element "
                               f"pitch, 4 levels, one launch per group over all pairs replayed from a hipGraph",
                   "pairs": len(sizes), "level0_pixels": px, "mode": HEADLINE_MODE, "launches": plan.num_groups,
                   "schedule": plan.describe().strip()},
        "roofline": {"bound": "hbm", "achieved": dom["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom["GB/s"] / HBM_PEAK_GBS, "traffic": profile_traffic(dom["kernel"]),
                     "kernel": dom["kernel"], "group": dom["group"], "algorithmic_bytes": dom["bytes"],
                     "kernel_ms": dom["ms"]},
        "batch_GB/s_algorithmic_16B_per_px": 16 * px / (ms * 1e-3) / 1e9,
    }
    result.update(extra)
    return result, sizes


def bench_image(args, torch, wt, synth, P, cyc, name):
    """A single-image workload (unsharp mask or Harris): the learned
    scheduler's plan with its roofline, plus unfused, FP16-intermediate and
    (unsharp mask) the swept schedule and the one-tile-per-workgroup
    baseline."""
    dev = torch.device("cuda:0")
    if name == "unsharp":
        C, H, W, seed = UNSHARP
        spec = P.unsharp_mask()
        img = synth.uniform_image(seed, C, H, W)
        oc = C
    else:
        C, H, W, seed = HARRIS
        spec = P.harris()
        img = synth.white_squares(synth.uniform_image(seed, C, H, W), seed, count=200)
        oc = 1
    base = torch.from_numpy(img).to(dev)
    # rotate buffer sets over more than the 256 MB Infinity Cache
    per_set = base.numel() * 4 + oc * H * W * 4
    nsets = max(2, min(16, int(1.1e9 // per_set) + 1))
    ins = [base.clone() for _ in range(nsets)]
    outs = [torch.empty((oc, H, W), device=dev) for _ in range(nsets)]

    def leg(mode, fixed=None, fp16=False, model=None):
        if mode == "autotune" and model is None:
            model = wt.GFX950_COST_MODEL
        plan = wt.from_spec(spec).plan(W, H, mode=mode, fixed=fixed, fp16=fp16, model_path=model)
        ms = timed(torch, lambda i: plan.run([ins[i % nsets]], [outs[i % nsets]]), args.steps, args.warmup, cyc)
        return plan, ms

    plan, ms = leg(HEADLINE_MODE)
    pipe = plan.pipe
    nbytes = sum(group_bytes(wt, plan, pipe, spec, g, [(W, H)]) for g in range(plan.num_groups))
    kname = kernel_name(plan, 0, False) if plan.num_groups == 1 else None
    res = {"value": H * W / (ms * 1e-3) / 1e6, "ms_per_step": ms, "mode": HEADLINE_MODE,
           "launches": plan.num_groups, "schedule": plan.describe().strip(), "buffer_sets": nsets,
           "roofline": {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": profile_traffic(kname) if kname else None, "kernel": kname,
                        "algorithmic_bytes": nbytes}}
    log(f"{name} {HEADLINE_MODE}: {ms * 1e3:.2f} us, {res['roofline']['achieved']:.0f} GB/s ({plan.describe().strip()})")
    ref = outs[(args.steps - 1) % nsets].clone()
    if name == "unsharp":
        res["copy_reference"] = copy_reference(torch, wt, ins, outs, args.steps, cyc)
    if args.no_extra:
        return res
    legs = [("unfused", dict(mode="unfused")),
            ("mlp", dict(mode="mlp", model=wt.GFX950_COST_MODEL)),
            ("fp16_intermediates", dict(mode=HEADLINE_MODE, fp16=True))]
    if name == "unsharp":
        legs += [("swept_schedule", dict(mode="fixed", fixed=SWEPT_UNSHARP)),
                 ("one_tile_per_workgroup", dict(mode="fixed", fixed=OTPTB_UNSHARP))]
    for key, kw in legs:
        pl, lms = leg(**kw)
        got = outs[(args.steps - 1) % nsets]
        diff = float((got - ref).abs().max() / ref.abs().max())
        res[key] = {"value": H * W / (lms * 1e-3) / 1e6, "ms_per_step": lms, "launches": pl.num_groups,
                    "vs_scheduled": lms / ms, "max_rel_diff": diff, "schedule": pl.describe().strip()}
        log(f"{name} {key}: {lms * 1e3:.2f} us ({pl.num_groups} launches), max rel diff {diff:.1e}")
        del pl
    return res


def bench_histogram(args, torch, wt, synth, P, cyc):
    """A reduction stage fused with its producer: the 256-bin histogram of
    the blurred 3x2048x2048 image, counted by the blur's group (the blurred
    image is never stored) against the unfused pipeline (the blur stored,
    then read back by the lone histogram kernel)."""
    dev = torch.device("cuda:0")
    C, H, W, seed = HIST_WORKLOAD
    spec = P.blur_histogram(channels=C, bins=256)
    base = torch.from_numpy(synth.uniform_image(seed, C, H, W)).to(dev)
    nsets = max(2, min(16, int(1.1e9 // (base.numel() * 4)) + 1))
    ins = [base.clone() for _ in range(nsets)]
    outs = [torch.zeros((C, 1, 256), dtype=torch.int32, device=dev) for _ in range(nsets)]

    def leg(mode, model=None):
        plan = wt.from_spec(spec).plan(W, H, mode=mode, model_path=model)
        ms = timed(torch, lambda i: plan.run([ins[i % nsets]], [outs[i % nsets]]), args.steps, args.warmup, cyc)
        return plan, ms, outs[(args.steps - 1) % nsets].clone()

    plan, ms, ref = leg(HEADLINE_MODE, wt.GFX950_COST_MODEL)
    nbytes = C * H * W * 4 + C * 256 * 4  # the image in, the counts out
    kname = kernel_name(plan, 0, False) if plan.num_groups == 1 else None
    res = {"value": H * W / (ms * 1e-3) / 1e6, "ms_per_step": ms, "mode": HEADLINE_MODE,
           "launches": plan.num_groups, "schedule": plan.describe().strip(), "buffer_sets": nsets,
           "roofline": {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "traffic": profile_traffic(kname) if kname else None, "kernel": kname,
                        "algorithmic_bytes": nbytes},
           "counted": int(ref.sum().item())}
    log(f"histogram {HEADLINE_MODE}: {ms * 1e3:.2f} us, {res['roofline']['achieved']:.0f} GB/s "
        f"({plan.describe().strip()})")
    if not args.no_extra:
        pl, lms, got = leg("unfused")
        res["unfused"] = {"value": H * W / (lms * 1e-3) / 1e6, "ms_per_step": lms, "launches": pl.num_groups,
                          "vs_scheduled": lms / ms, "counts_equal": bool(torch.equal(got, ref)),
                          "schedule": pl.describe().strip()}
        log(f"histogram unfused: {lms * 1e3:.2f} us ({pl.num_groups} launches), counts equal "
            f"{res['unfused']['counts_equal']}")
        # the counts' consumer: equalisation of the blur and a blend with
        # the input, in the kernel after the counting one
        espec = P.blur_equalize(channels=C, bins=256)
        eouts = [torch.empty((C, H, W), device=dev) for _ in range(nsets)]
        for emode in (HEADLINE_MODE, "unfused"):
            epl = wt.from_spec(espec).plan(W, H, mode=emode, model_path=wt.GFX950_COST_MODEL)
            ems = timed(torch, lambda i: epl.run([ins[i % nsets]], [eouts[i % nsets]]), args.steps, args.warmup, cyc)
            res["equalize_" + emode] = {"value": H * W / (ems * 1e-3) / 1e6, "ms_per_step": ems,
                                        "launches": epl.num_groups, "schedule": epl.describe().strip()}
            log(f"equalize {emode}: {ems * 1e3:.2f} us ({epl.num_groups} launches)")
    return res


def copy_reference(torch, wt, ins, outs, steps, cyc):
    """The same bytes as the unsharp mask's compulsory traffic (one image in,
    one out) moved by the runtime's copy and by the library's streaming copy
    kernel."""
    n = len(ins)
    ms = timed(torch, lambda i: outs[i % n].copy_(ins[i % n]), steps, 5, cyc)
    ms_s = timed(torch, lambda i: wt.stream_copy(ins[i % n], outs[i % n]), steps, 5, cyc)
    nbytes = 2 * ins[0].numel() * ins[0].element_size()
    return {"bytes": nbytes, "GB/s": nbytes / (ms * 1e-3) / 1e9, "streaming_GB/s": nbytes / (ms_s * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the headline plan of each workload")
    ap.add_argument("--no-secondary", action="store_true", help="skip the unsharp-mask and Harris workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (tiles and images "
              "are independent, so a batch or the tile rows of an image would be split across "
              "GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    # the autotuner reports each group it tunes on stderr
    os.environ.setdefault("WT_VERBOSE", "1")
    import torch
    import paper_1909_07190_amd as wt
    import synth
    from synth import pipelines as P

    # the host baseline runs first, in child processes forked before this
    # process initialises the GPU
    cpu = None if args.no_cpu else cpu_baseline(synth.batch_sizes(PYR_SEED, PYR_PAIRS))
    if cpu:
        log(f"oracle: {cpu['value']:.2f} Mpix/s on {cpu['cores']} cores, {cpu['one_core']['value']:.2f} on one")
    cyc = calibrate_sleep(torch)
    head, sizes = bench_pyramid(args, torch, wt, synth, P, cyc)
    torch.cuda.empty_cache()
    secondary = {}
    if not args.no_secondary:
        for name in ("unsharp", "harris"):
            secondary[name] = bench_image(args, torch, wt, synth, P, cyc, name)
            torch.cuda.empty_cache()
        secondary["histogram"] = bench_histogram(args, torch, wt, synth, P, cyc)
        torch.cuda.empty_cache()
    out = {
        "metric": METRIC, "value": head.pop("value"), "unit": "Mpixels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": head.pop("config"), "roofline": head.pop("roofline"),
        "cpu_baseline": cpu,
    }
    out.update(head)
    if "unsharp" in secondary:
        out["unsharp_3x2048x2048"] = secondary["unsharp"]
    if "harris" in secondary:
        out["harris_3x4096x4096"] = secondary["harris"]
    if "histogram" in secondary:
        out["blur_histogram_3x2048x2048"] = secondary["histogram"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
