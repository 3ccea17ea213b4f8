"""GPU parity on the paths the benchmark runs: the plans the schedulers
choose on their own (the learned model's, the autotuner's) and the exact
configurations the benchmark times, at the configured full sizes, against
the FP64 oracle (FP32 normwise 1e-5 per output channel, FP16 intermediates
2e-3; the unsharp mask's select accepts either branch within the tie band).
Also the host-side refusals of batched runs with bad strides or aliased
outputs."""
import ctypes
import sys

import numpy as np
import pytest

import bench
import oracle
import synth
from synth import dags
from synth import pipelines as P
from wt_helpers import assert_normwise, check_unsharp, run_gpu

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _model():
    import paper_1909_07190_amd as wt
    return wt.GFX950_COST_MODEL


def _unsharp_image():
    C, H, W, seed = bench.UNSHARP
    return synth.uniform_image(seed, C, H, W)


def _harris_image():
    C, H, W, seed = bench.HARRIS
    return synth.white_squares(synth.uniform_image(seed, C, H, W), seed, count=200)


def test_unsharp_benchmark_schedules_full_size():
    """The swept schedule, the benchmark's autotuned plan (FP32 and FP16
    intermediates), the learned scheduler's plan and the one-tile-per-
    workgroup baseline on the 3x2048x2048 unsharp-mask workload."""
    spec = P.unsharp_mask()
    img = _unsharp_image()
    for kw, rtol in ((dict(mode="fixed", fixed=bench.SWEPT_UNSHARP), 1e-5),
                     (dict(mode=bench.HEADLINE_MODE, model_path=_model()), 1e-5),
                     (dict(mode=bench.HEADLINE_MODE, fp16=True, model_path=_model()), 2e-3),
                     (dict(mode="mlp"), 1e-5),
                     (dict(mode="fixed", fixed=bench.OTPTB_UNSHARP), 1e-5)):
        _say(f"unsharp 3x2048x2048 {kw}")
        got, plan = run_gpu(spec, {"img": img}, **kw)
        _say(f"  plan: {plan.describe().strip()}")
        check_unsharp(got["mask"], img, rtol, spec)


@pytest.mark.parametrize("mode", ["mlp", "autotune"])
def test_harris_scheduled_full_size(mode, tmp_path, monkeypatch):
    """The learned scheduler's and the (network-ranked) autotuner's Harris
    plans at 3x4096x4096 with 200 white squares, FP32 and FP16."""
    import paper_1909_07190_amd as wt
    monkeypatch.setenv("WT_CACHE_DIR", str(tmp_path))
    spec = P.harris()
    img = _harris_image()
    ref = oracle.evaluate(spec, {"img": img})["R"]
    model = wt.GFX950_COST_MODEL
    for fp16, rtol in ((False, 1e-5), (True, 2e-3)):
        _say(f"harris 3x4096x4096 {mode} fp16={fp16}")
        got, plan = run_gpu(spec, {"img": img}, mode=mode, fp16=fp16, model_path=model)
        _say(f"  plan: {plan.describe().strip()}")
        assert_normwise(got["R"], ref, rtol, f"harris {mode} fp16={fp16}")


@pytest.mark.parametrize("seed", [200, 201, 202])
def test_random_dag_learned_schedule_full_size(seed):
    """The learned scheduler's plans for random pipelines of the
    learned-scheduler workload at 2048 x 2048."""
    spec = dags.random_dag(seed)
    _say(f"random dag {seed} ({len(spec['stages'])} stages), mlp plan")
    imgs = {inp["name"]: synth.uniform_image(seed * 7 + k, 1, 2048, 2048) for k, inp in enumerate(spec["inputs"])}
    got, plan = run_gpu(spec, imgs, mode="mlp")
    _say(f"  plan: {plan.describe().strip()}")
    ref = oracle.evaluate(spec, imgs)
    for k in spec["outputs"]:
        assert_normwise(got[k], ref[k], 1e-5, f"{k}: {plan.describe()}")


def _pyramid_tensors(torch, sizes, idx):
    dev = torch.device("cuda:0")
    tin, host = [], {}
    for i, (w, h) in enumerate(sizes):
        pair = bench.pyramid_pair(synth, i, w, h)
        if i in idx:
            host[i] = pair
        tin.append([torch.from_numpy(x).to(dev) for x in pair])
    tout = [[torch.full((1, h, w), float("nan"), device=dev)] for (w, h) in sizes]
    return tin, tout, host


def test_pyramid_headline_batch_full_workload():
    """The benchmark's headline workload: the 64-pair batch under the learned
    scheduler's plan, one launch per group over all pairs from a hipGraph.
    Every image is finite; the three smallest and the three largest are
    checked entirely against the oracle.  Relaunching the last group alone
    (the benchmark's per-kernel timing path) rewrites the same outputs.
    (The benchmark's own plan is the autotuner's, tested on a sub-batch
    below: tuning the whole batch takes minutes.)"""
    import torch
    import paper_1909_07190_amd as wt
    spec = P.pyramid_blend(bench.PYR_LEVELS)
    sizes = synth.batch_sizes(bench.PYR_SEED, bench.PYR_PAIRS)
    order = sorted(range(len(sizes)), key=lambda k: sizes[k][0] * sizes[k][1])
    check = order[:3] + order[-3:]
    _say(f"pyramid headline batch: {len(sizes)} pairs, checking {[sizes[k] for k in check]}")
    tin, tout, host = _pyramid_tensors(torch, sizes, set(check))
    plan = bench.plan_pyramid(wt, P, sizes, "mlp", wt.GFX950_COST_MODEL)
    _say(f"  plan: {plan.describe().strip()}")
    plan.run_batch(tin, tout)
    torch.cuda.synchronize()
    for i in range(len(sizes)):
        assert torch.isfinite(tout[i][0]).all(), f"image {i}"
    first = [t[0].clone() for t in tout]
    g = plan.num_groups - 1
    for t in tout:
        t[0].fill_(float("nan"))
    plan.run_batch(tin, tout)
    plan.run_batch_groups(g, 1, tin, tout)
    torch.cuda.synchronize()
    for i in range(len(sizes)):
        assert torch.equal(tout[i][0], first[i]), f"image {i} after relaunching group {g}"
    for i in check:
        w, h = sizes[i]
        _say(f"  oracle {w}x{h}")
        a, b, m = host[i]
        ref = oracle.evaluate(spec, {"A": a, "B": b, "M": m})
        assert_normwise(first[i].cpu().numpy(), ref[spec["outputs"][0]], 1e-5, f"image {i} {w}x{h}")


def test_pyramid_autotuned_sub_batch(tmp_path, monkeypatch):
    """The benchmark's planning path (autotune ranked by the learned model,
    with and without folded expansions, candidates timed on stacked images)
    on 4 pairs of the headline batch, one candidate per ranking; the
    smallest and the largest pair against the oracle."""
    import torch
    import paper_1909_07190_amd as wt
    monkeypatch.setenv("WT_CACHE_DIR", str(tmp_path))
    spec = P.pyramid_blend(bench.PYR_LEVELS)
    sizes = synth.batch_sizes(bench.PYR_SEED, bench.PYR_PAIRS)[:4]
    order = sorted(range(len(sizes)), key=lambda k: sizes[k][0] * sizes[k][1])
    check = [order[0], order[-1]]
    tin, tout, host = _pyramid_tensors(torch, sizes, set(check))
    plan = bench.plan_pyramid(wt, P, sizes, bench.HEADLINE_MODE, topk=1)
    _say(f"  plan: {plan.describe().strip()}")
    plan.run_batch(tin, tout)
    torch.cuda.synchronize()
    for i in check:
        w, h = sizes[i]
        _say(f"  oracle {w}x{h}")
        a, b, m = host[i]
        ref = oracle.evaluate(spec, {"A": a, "B": b, "M": m})
        assert_normwise(tout[i][0].cpu().numpy(), ref[spec["outputs"][0]], 1e-5, f"image {i} {w}x{h}")


def test_batch_refuses_bad_strides_and_aliases():
    """wt_plan_run_batch checks every image as wt_plan_run does, on the host,
    before any launch: a negative row stride is WT_E_SHAPE, an output that
    aliases another image of the batch WT_E_INVALID, a group range outside
    the plan WT_E_INVALID."""
    import torch
    import paper_1909_07190_amd as wt
    spec = P.gaussian_blur()
    dev = torch.device("cuda:0")
    plan = wt.from_spec(spec).plan(64, 32, mode="analytic", any_width=True)
    imgs = [torch.rand((1, 32, 64), device=dev) for _ in range(4)]

    def run(ins, outs, first=None):
        a_in = (wt.WtImage * len(ins))(*ins)
        a_out = (wt.WtImage * len(outs))(*outs)
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        if first is None:
            return wt.lib.wt_plan_run_batch(plan._h, len(ins), a_in, a_out, s)
        return wt.lib.wt_plan_run_batch_groups(plan._h, first, 1, len(ins), a_in, a_out, s)

    ok_in = [wt._image(imgs[0]), wt._image(imgs[1])]
    ok_out = [wt._image(imgs[2]), wt._image(imgs[3])]
    assert run(ok_in, ok_out) == 0
    torch.cuda.synchronize()
    neg = wt._image(imgs[1])
    neg.row_stride = -64
    assert run([ok_in[0], neg], ok_out) == -3
    short = wt._image(imgs[1])
    short.row_stride = 32
    assert run([ok_in[0], short], ok_out) == -3
    assert run(ok_in, [ok_out[0], wt._image(imgs[0])]) == -1      # output = another image's input
    assert run(ok_in, [ok_out[0], ok_out[0]]) == -1               # two outputs share a buffer
    assert run(ok_in, ok_out, first=plan.num_groups) == -1
    assert run(ok_in, ok_out, first=0) == 0
    torch.cuda.synchronize()


def test_pyramid_tuned_on_the_batch():
    """Tuning a plan on the batch itself (every group's configuration and
    its neighbours timed as batched kernels over these images) leaves a plan
    whose outputs, written by the tuning call and by a later replay, match
    the oracle."""
    import torch
    import paper_1909_07190_amd as wt
    spec = P.pyramid_blend(bench.PYR_LEVELS)
    sizes = synth.batch_sizes(bench.PYR_SEED, bench.PYR_PAIRS)[:5]
    order = sorted(range(len(sizes)), key=lambda k: sizes[k][0] * sizes[k][1])
    check = [order[0], order[-1]]
    tin, tout, host = _pyramid_tensors(torch, sizes, set(check))
    plan = bench.plan_pyramid(wt, P, sizes, "analytic")
    before = plan.describe()
    plan.tune_batch(tin, tout)
    torch.cuda.synchronize()
    _say(f"  tuned: {plan.describe().strip()}")
    for rep in range(2):
        if rep:
            tout = [[torch.full((1, h, w), float("nan"), device=tin[0][0].device)] for (w, h) in sizes]
            plan.run_batch(tin, tout)
            torch.cuda.synchronize()
        for i in check:
            w, h = sizes[i]
            a, b, m = host[i]
            ref = oracle.evaluate(spec, {"A": a, "B": b, "M": m})
            assert_normwise(tout[i][0].cpu().numpy(), ref[spec["outputs"][0]], 1e-5, f"rep {rep} image {i} {w}x{h}")
    assert len(plan.describe().splitlines()) == len(before.splitlines())


@pytest.mark.skip(reason="the whole-pipeline launch is switched off on the device: its first run went silent for "
                         "three minutes and was killed, cause not found (host emulation is bit-identical); "
                         "wt_plan_run_batch refuses WT_PLAN_BATCH_WHOLE until the cause is fixed")
def test_whole_pipeline_launch():
    """The whole group sequence as one persistent launch (every group's
    tiles taken in ticket order, each chunk started once its producer groups
    have finished that image) writes exactly what the per-group launches
    write, on a batch of uneven pyramid pairs and on a Harris batch; replays
    of its graph with other work between them give the same outputs; no wait
    gives up; the smallest and largest pairs match the oracle.  A plan with a
    lone histogram group is refused on the host before any launch."""
    import torch
    import paper_1909_07190_amd as wt
    spec = P.pyramid_blend(bench.PYR_LEVELS)
    sizes = synth.batch_sizes(bench.PYR_SEED, bench.PYR_PAIRS)[:6]
    order = sorted(range(len(sizes)), key=lambda k: sizes[k][0] * sizes[k][1])
    check = [order[0], order[-1]]
    tin, tout, host = _pyramid_tensors(torch, sizes, set(check))
    plan = bench.plan_pyramid(wt, P, sizes, "analytic")
    mw, mh = bench.median_size(sizes)
    whole = wt.from_spec(spec).plan(mw, mh, mode="fixed", fixed=plan.describe(), any_width=True,
                                    batch_images=len(sizes), batch_whole=True)
    _say(f"  {len(sizes)} pairs, {plan.num_groups} groups")
    plan.run_batch(tin, tout)
    wout = [[torch.full_like(t[0], float("nan"))] for t in tout]
    whole.run_batch(tin, wout)
    whole.batch_check()
    for i in range(len(sizes)):
        assert torch.equal(wout[i][0], tout[i][0]), f"pair {i} {sizes[i]}"
    for rep in range(3):
        torch.cuda.synchronize()
        junk = torch.ones((1 << 20,), device=tin[0][0].device).cumsum(0)  # eager work between replays
        rout = [[torch.full_like(t[0], float("nan"))] for t in tout]
        whole.run_batch(tin, rout)
        whole.batch_check()
        del junk
        for i in range(len(sizes)):
            assert torch.equal(rout[i][0], tout[i][0]), f"replay {rep} pair {i}"
    for i in check:
        a, b, m = host[i]
        ref = oracle.evaluate(spec, {"A": a, "B": b, "M": m})
        assert_normwise(wout[i][0].cpu().numpy(), ref[spec["outputs"][0]], 1e-5, f"pair {i} {sizes[i]}")
    _say("  pyramid batch ok")

    dev = torch.device("cuda:0")
    hs = [(300, 200), (517, 129)]
    imgs = [torch.from_numpy(synth.uniform_image(30 + k, 3, h, w)).to(dev) for k, (w, h) in enumerate(hs)]
    fixed = "nodes=1,2,3,4,5,6,7,8,9,10 V=2 TX=1 SX=0 TY=16 WPB=2 PF=2"
    ref_plan = wt.from_spec(P.harris()).plan(300, 200, mode="fixed", fixed=fixed, batch_images=2)
    hw = wt.from_spec(P.harris()).plan(300, 200, mode="fixed", fixed=fixed, batch_images=2, batch_whole=True)
    o1 = [[torch.empty((1, h, w), device=dev)] for (w, h) in hs]
    o2 = [[torch.full((1, h, w), float("nan"), device=dev)] for (w, h) in hs]
    ref_plan.run_batch([[x] for x in imgs], o1)
    hw.run_batch([[x] for x in imgs], o2)
    hw.batch_check()
    for k in range(len(hs)):
        assert torch.equal(o1[k][0], o2[k][0]), f"harris image {k}"
    _say("  harris batch ok")

    hp = wt.from_spec(P.blur_histogram()).plan(256, 128, mode="unfused", batch_images=2, batch_whole=True)
    x = [torch.rand((1, 128, 256), device=dev) for _ in range(2)]
    hout = [[torch.empty((1, 1, 64), dtype=torch.int32, device=dev)] for _ in range(2)]
    with pytest.raises(wt.WtError) as e:
        hp.run_batch([[t] for t in x], hout)
    assert e.value.status == -2


def test_whole_pipeline_launch_refused():
    """While the whole-pipeline launch is switched off, a batch run of a plan
    made with it is refused with WT_E_UNSUPPORTED on the host, before any
    allocation or launch; the same plan still runs groups one by one."""
    import torch
    import paper_1909_07190_amd as wt
    dev = torch.device("cuda:0")
    fixed = "nodes=1,2,3,4 V=1 TX=2 SX=0 TY=8 PF=1"
    pl = wt.from_spec(P.unsharp_mask(channels=1)).plan(128, 64, mode="fixed", fixed=fixed, batch_images=2,
                                                      batch_whole=True)
    x = [torch.rand((1, 64, 128), device=dev) for _ in range(2)]
    y = [torch.empty((1, 64, 128), device=dev) for _ in range(2)]
    with pytest.raises(wt.WtError) as e:
        pl.run_batch([[t] for t in x], [[t] for t in y])
    assert e.value.status == -2
    pl.batch_check()  # no whole-pipeline launch ran: nothing to report
