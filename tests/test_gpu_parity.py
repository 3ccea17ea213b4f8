"""GPU parity: the generated HIP kernels against the FP64 oracle.

Every case builds the pipeline through the C ABI, runs it on cuda:0 and
compares element by element with the oracle on the same seeded inputs.
Tolerances: FP32 normwise 1e-5, FP16 intermediates 2e-3 (per output
channel, inf-norm relative); bit-exact where every intermediate is exact in
FP32 (dyadic inputs).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import pipelines as P
from wt_helpers import assert_exact, assert_normwise, check_unsharp, run_gpu

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


BLUR = P.gaussian_blur()
UM = P.unsharp_mask()

# (schedule text, width, height): several tiles, ragged tails, LDS sub-tiles,
# the paper's left-only alignment, and all vector widths.
BLUR_CASES = [
    ("nodes=1,2 V=4 TX=1 SX=0 TY=16 PF=2", 256, 256),
    ("nodes=1,2 V=4 TX=2 SX=1 TY=13 PF=1", 260, 77),
    ("nodes=1,2 V=2 TX=2 SX=0 TY=7 PF=0", 302, 45),
    ("nodes=1,2 V=1 TX=3 SX=2 TY=9 PF=1", 205, 33),
    ("nodes=1,2 V=4 TX=2 SX=0 TY=8 PF=1 align=1", 516, 40),
    ("nodes=1,2 V=1 TX=2 SX=1 TY=5 PF=2 align=1", 131, 19),
    ("nodes=1,2 V=4 TX=1 SX=1 TY=3 PF=0 WPB=4", 1028, 10),
    ("nodes=1 V=4 TX=1 SX=0 TY=16;nodes=2 V=4 TX=1 SX=0 TY=16", 300, 300),
]


@pytest.mark.parametrize("fixed,w,h", BLUR_CASES)
def test_blur_schedules(fixed, w, h):
    _say(f"blur {w}x{h} [{fixed}]")
    img = synth.uniform_image(1, 1, h, w)
    got, _ = run_gpu(BLUR, {"img": img}, mode="fixed", fixed=fixed)
    ref = oracle.evaluate(BLUR, {"img": img})["by"]
    assert_normwise(got["by"], ref, 1e-5, fixed)
    dy = synth.dyadic_image(2, 1, h, w)
    got, _ = run_gpu(BLUR, {"img": dy}, mode="fixed", fixed=fixed)
    assert_exact(got["by"], oracle.evaluate(BLUR, {"img": dy})["by"], fixed)


WIDE = P.wide_chain()
WIDE_NODES = ",".join(str(i) for i in range(1, 12))


@pytest.mark.parametrize("cfg,w,h", [
    ("V=1 TX=3 SX=0 TY=16 PF=2 align=1", 1500, 130),
    ("V=1 TX=3 SX=1 TY=8 PF=1 align=1", 777, 41),
    ("V=1 TX=4 SX=2 TY=5 PF=1 align=1", 640, 23),
    ("V=1 TX=3 SX=3 TY=8 PF=1 align=1", 301, 17),
])
def test_lookback_across_sub_tiles(cfg, w, h):
    """Right-hyperplane tiles of a ten-stencil chain: the input edge spans
    70 columns, more than one wavefront at one element per lane."""
    fixed = f"nodes={WIDE_NODES} {cfg}"
    _say(f"wide chain {w}x{h} [{fixed}]")
    img = synth.uniform_image(32, 1, h, w)
    got, _ = run_gpu(WIDE, {"img": img}, mode="fixed", fixed=fixed)
    assert_normwise(got["out"], oracle.evaluate(WIDE, {"img": img})["out"], 1e-5, fixed)


@pytest.mark.parametrize("w,h", [(1, 1), (3, 2), (5, 7), (64, 1), (1, 64)])
def test_blur_tiny(w, h):
    _say(f"blur tiny {w}x{h}")
    img = synth.dyadic_image(3, 1, h, w)
    got, _ = run_gpu(BLUR, {"img": img}, mode="fixed", fixed="nodes=1,2 V=1 TX=1 SX=0 TY=4 PF=1")
    assert_exact(got["by"], oracle.evaluate(BLUR, {"img": img})["by"], f"{w}x{h}")


def test_blur_256_default_and_unfused():
    _say("blur 256x256 default / unfused")
    img = synth.uniform_image(1, 1, 256, 256)
    ref = oracle.evaluate(BLUR, {"img": img})["by"]
    for mode in ("analytic", "unfused"):
        got, _ = run_gpu(BLUR, {"img": img}, mode=mode)
        assert_normwise(got["by"], ref, 1e-5, mode)


UM_CASES = [
    ("nodes=1,2,3,4 V=4 TX=1 SX=0 TY=16 PF=2", False),
    ("nodes=1,2,3,4 V=4 TX=2 SX=1 TY=10 PF=1", False),
    ("nodes=1,2,3,4 V=2 TX=2 SX=0 TY=12 PF=1 align=1", False),
    ("nodes=1,2,3,4 V=4 TX=1 SX=0 TY=16 PF=2 fp16=1", True),
    ("nodes=1,2 V=4 TX=1 SX=0 TY=8;nodes=3,4 V=4 TX=1 SX=0 TY=8", False),
]


@pytest.mark.parametrize("fixed,fp16", UM_CASES)
def test_unsharp_schedules(fixed, fp16):
    h, w = 70, 516
    _say(f"unsharp {w}x{h} [{fixed}]")
    img = synth.uniform_image(2, 3, h, w)
    got, _ = run_gpu(UM, {"img": img}, mode="fixed", fixed=fixed, fp16=fp16)
    check_unsharp(got["mask"], img, 2e-3 if fp16 else 1e-5, UM)
    if not fp16:
        dy = synth.dyadic_image(4, 3, h, w)
        got, _ = run_gpu(UM, {"img": dy}, mode="fixed", fixed=fixed)
        assert_exact(got["mask"], oracle.evaluate(UM, {"img": dy})["mask"], fixed)


def test_unsharp_full_size():
    _say("unsharp 3x2048x2048 fused / unfused / fp16")
    img = synth.uniform_image(2, 3, 2048, 2048)
    fixed = "nodes=1,2,3,4 V=4 TX=1 SX=0 TY=16 PF=2"
    got, _ = run_gpu(UM, {"img": img}, mode="fixed", fixed=fixed)
    check_unsharp(got["mask"], img, 1e-5, UM)
    got, _ = run_gpu(UM, {"img": img}, mode="unfused")
    check_unsharp(got["mask"], img, 1e-5, UM)
    got, _ = run_gpu(UM, {"img": img}, mode="fixed", fixed=fixed + " fp16=1", fp16=True)
    check_unsharp(got["mask"], img, 2e-3, UM)


HARRIS = P.harris()
HARRIS_EXACT = P.harris(gray_weights=(1.0, 0.0, 0.0), k=1.0 / 32)
HARRIS_FUSED = "nodes=1,2,3,4,5,6,7,8,9,10 V=4 TX=1 SX=0 TY=16 PF=1"
HARRIS_CASES = [
    HARRIS_FUSED,
    "nodes=1,2,3,4,5,6,7,8,9,10 V=2 TX=2 SX=1 TY=8 PF=1 align=1",
    "nodes=1,2,3 V=4 TX=1 SX=0 TY=16;nodes=4,5,6,7,8,9,10 V=4 TX=1 SX=0 TY=16 PF=2",
]


@pytest.mark.parametrize("fixed", HARRIS_CASES)
def test_harris_schedules(fixed):
    h, w = 67, 520
    _say(f"harris {w}x{h} [{fixed}]")
    sq = synth.white_squares(np.zeros((3, h, w), np.float32), 5, count=20, side_lo=3, side_hi=30)
    got, _ = run_gpu(HARRIS_EXACT, {"img": sq}, mode="fixed", fixed=fixed)
    assert_exact(got["R"], oracle.evaluate(HARRIS_EXACT, {"img": sq})["R"], fixed)
    got, _ = run_gpu(HARRIS_EXACT, {"img": sq}, mode="fixed", fixed=fixed + " fp16=1", fp16=True)
    assert_exact(got["R"], oracle.evaluate(HARRIS_EXACT, {"img": sq})["R"], fixed + " fp16")
    img = synth.uniform_image(3, 3, h, w)
    got, _ = run_gpu(HARRIS, {"img": img}, mode="fixed", fixed=fixed)
    assert_normwise(got["R"], oracle.evaluate(HARRIS, {"img": img})["R"], 1e-5, fixed)


def test_harris_full_size_fp16():
    _say("harris 3x4096x4096 + 200 squares, FP16 intermediates")
    img = synth.white_squares(synth.uniform_image(3, 3, 4096, 4096), 3, count=200)
    got, _ = run_gpu(HARRIS, {"img": img}, mode="fixed", fixed=HARRIS_FUSED + " fp16=1", fp16=True)
    ref = oracle.evaluate(HARRIS, {"img": img})["R"]
    assert_normwise(got["R"], ref, 2e-3, "harris fp16")
    got, _ = run_gpu(HARRIS, {"img": img}, mode="fixed", fixed=HARRIS_FUSED)
    assert_normwise(got["R"], ref, 1e-5, "harris fp32")


@pytest.mark.parametrize("mode", ["unfused", "analytic"])
def test_pyramid_blend(mode):
    spec = P.pyramid_blend(4)
    for (w, h) in [(45, 37), (700, 513)]:
        _say(f"pyramid {w}x{h} {mode}")
        ins = {"A": synth.uniform_image(21, 1, h, w), "B": synth.uniform_image(22, 1, h, w),
               "M": synth.ramp_mask(h, w)}
        got, _ = run_gpu(spec, ins, mode=mode)
        assert_normwise(got["R0"], oracle.evaluate(spec, ins)["R0"], 1e-5, mode)


def test_pyramid_two_level_exact():
    _say("pyramid 2-level exact")
    spec = P.pyramid_blend(2)
    a, b = synth.dyadic_image(31, 1, 130, 260), synth.dyadic_image(32, 1, 130, 260)
    for m in (np.ones((1, 130, 260), np.float32), np.zeros((1, 130, 260), np.float32)):
        got, _ = run_gpu(spec, {"A": a, "B": b, "M": m}, mode="analytic")
        assert_exact(got["R0"], oracle.evaluate(spec, {"A": a, "B": b, "M": m})["R0"], "pyramid")


def _batch_inputs(spec, sizes, seed):
    ins = []
    for i, (w, h) in enumerate(sizes):
        d = {}
        for k, inp in enumerate(spec["inputs"]):
            if inp["name"] == "M":
                d["M"] = synth.ramp_mask(h, w)
            else:
                d[inp["name"]] = synth.uniform_image(seed + 10 * i + k, inp["channels"], h, w)
        ins.append(d)
    return ins


@pytest.mark.parametrize("spec_name", ["pyramid", "unsharp"])
def test_batched_persistent_graph(spec_name):
    """One persistent launch per group over all images of a batch, replayed
    from a hipGraph: equal to per-image runs of the same schedule (bit for
    bit) and to the oracle; a second run with new output buffers replays the
    captured graph."""
    import torch
    import paper_1909_07190_amd as wt
    from wt_helpers import _channels, _levels
    spec = P.pyramid_blend(4) if spec_name == "pyramid" else P.unsharp_mask()
    sizes = [(130, 67), (201, 150), (64, 64), (513, 300), (97, 41)]
    _say(f"batched {spec_name} {sizes}")
    images = _batch_inputs(spec, sizes, 70)
    w0, h0 = sizes[0]
    bplan = wt.from_spec(spec).plan(w0, h0, mode="analytic", any_width=True)
    sched = bplan.describe()
    dev = torch.device("cuda:0")
    lv, ch = _levels(spec), _channels(spec)

    def alloc_outs(w, h):
        outs = []
        for o in spec["outputs"]:
            ow, oh = oracle.level_size(w, h, lv[o])
            outs.append(torch.full((ch[o], oh, ow), float("nan"), device=dev))
        return outs

    tin = [[torch.from_numpy(img[i["name"]]).to(dev) for i in spec["inputs"]] for img in images]
    tout = [alloc_outs(w, h) for (w, h) in sizes]
    bplan.run_batch(tin, tout)
    torch.cuda.synchronize()
    for k, (w, h) in enumerate(sizes):
        single = wt.from_spec(spec).plan(w, h, mode="fixed", fixed=sched, any_width=True)
        sout = alloc_outs(w, h)
        single.run(tin[k], sout)
        torch.cuda.synchronize()
        for o, a, b in zip(spec["outputs"], tout[k], sout):
            assert torch.equal(a, b), f"image {k} output {o}: batched != single"
        ref = oracle.evaluate(spec, images[k])
        o = spec["outputs"][0]
        if spec_name == "unsharp":
            check_unsharp(tout[k][0].cpu().numpy(), images[k]["img"], 1e-5, spec)
        else:
            assert_normwise(tout[k][0].cpu().numpy(), ref[o], 1e-5, f"batched image {k}")
    # graph replay with fresh output buffers
    tout2 = [alloc_outs(w, h) for (w, h) in sizes]
    bplan.run_batch(tin, tout2)
    torch.cuda.synchronize()
    for k in range(len(sizes)):
        for a, b in zip(tout[k], tout2[k]):
            assert torch.equal(a, b), f"replay differs for image {k}"


def test_batch_grid_resident_equals_per_tile(monkeypatch):
    """A batched launch with one workgroup per work unit (the default) and
    one sized to the resident workgroups, each looping over several units
    (the plan flag, or WT_BATCH_GRID=resident), give bit-identical outputs."""
    import re
    import torch
    import paper_1909_07190_amd as wt
    spec = P.unsharp_mask()
    sizes = [(2050, 1030), (130, 67), (201, 150), (97, 41)]
    fixed = "nodes=1,2,3,4 V=1 TX=1 SX=0 TY=8 PF=2"
    _say(f"batch grids unsharp {sizes} {fixed}")
    images = _batch_inputs(spec, sizes, 110)
    dev = torch.device("cuda:0")
    tin = [[torch.from_numpy(img["img"]).to(dev)] for img in images]

    def run(grid, flag=False):
        if grid:
            monkeypatch.setenv("WT_BATCH_GRID", grid)
        else:
            monkeypatch.delenv("WT_BATCH_GRID", raising=False)
        plan = wt.from_spec(spec).plan(130, 67, mode="fixed", fixed=fixed, any_width=True, batch_resident=flag)
        outs = [[torch.full((3, h, w), float("nan"), device=dev)] for (w, h) in sizes]
        plan.run_batch(tin, outs)
        torch.cuda.synchronize()
        return [int(x) for x in re.findall(r"batch_grid=(\d+)", plan.describe())], outs

    g1, a = run(None)
    g2, b = run("resident")
    g3, c = run(None, flag=True)
    # 35 x 129 tiles x 3 channels of the large image alone exceed the
    # resident workgroups, so the resident grid loops
    assert len(g1) == len(g2) == 1 and g1[0] > g2[0] and g3 == g2
    for k in range(len(sizes)):
        assert torch.isfinite(a[k][0]).all() and torch.equal(a[k][0], b[k][0]), f"image {k}"
        assert torch.equal(a[k][0], c[k][0]), f"image {k} (plan flag)"
    check_unsharp(a[1][0].cpu().numpy(), images[1]["img"], 1e-5, spec)


def test_autotune_batched_times_stacked_images(tmp_path, monkeypatch):
    """Autotuning a plan for a batch times each fused group's candidates on
    an image as tall as the batch (the database records that height), and
    the tuned plan's batched run matches the oracle on every image."""
    import json
    import torch
    import paper_1909_07190_amd as wt
    from wt_helpers import _channels, _levels
    db = tmp_path / "measure.jsonl"
    monkeypatch.setenv("WT_MEASURE_DB", str(db))
    spec = P.pyramid_blend(3)
    sizes = [(130, 67), (201, 150), (64, 64), (97, 41)]
    _say(f"autotune batched pyramid {sizes}")
    w0, h0 = sizes[0]
    plan = wt.from_spec(spec).plan(w0, h0, mode="autotune", autotune_topk=2, any_width=True,
                                   batch_images=len(sizes))
    rows = [json.loads(l) for l in db.read_text().splitlines()]
    assert rows and {(r["W"], r["H"]) for r in rows} == {(w0, h0 * len(sizes))}
    images = _batch_inputs(spec, sizes, 90)
    dev = torch.device("cuda:0")
    lv, ch = _levels(spec), _channels(spec)
    tin = [[torch.from_numpy(img[i["name"]]).to(dev) for i in spec["inputs"]] for img in images]
    tout = []
    for (w, h) in sizes:
        outs = []
        for o in spec["outputs"]:
            ow, oh = oracle.level_size(w, h, lv[o])
            outs.append(torch.full((ch[o], oh, ow), float("nan"), device=dev))
        tout.append(outs)
    plan.run_batch(tin, tout)
    torch.cuda.synchronize()
    o = spec["outputs"][0]
    for k in range(len(sizes)):
        ref = oracle.evaluate(spec, images[k])
        assert_normwise(tout[k][0].cpu().numpy(), ref[o], 1e-5, f"image {k}: {plan.describe()}")


# ------------------------------------------------------------ integer stages
# Bit-exact against the oracle's int64 arithmetic (sums, rounded divisions and
# saturation), through fused, split and unfused schedules, LDS sub-tiles,
# both alignments, ragged sizes and every integer type.
INT_CASES = [
    ("binomial_u8", "nodes=1,2 V=4 TX=1 SX=0 TY=16 PF=2", 256, 256, 0, 255),
    ("binomial_u8", "nodes=1,2 V=1 TX=2 SX=1 TY=5 PF=1 align=1", 131, 19, 0, 255),
    ("integer_unsharp", "nodes=1,2,3,4 V=2 TX=2 SX=0 TY=6 PF=1", 150, 37, 0, 255),
    ("integer_unsharp", "nodes=1,2,3,4 V=4 TX=2 SX=1 TY=4 PF=2 align=1", 300, 13, 0, 255),
    ("integer_unsharp", "nodes=1 V=2 TY=4;nodes=2 V=1 TY=8;nodes=3,4 V=4 TY=16", 76, 21, 0, 255),
    ("integer_gradient", "nodes=1,2,3,4 V=2 TX=1 SX=0 TY=8;nodes=5;nodes=6 V=1", 90, 33, 0, 65535),
    ("integer_gradient", "nodes=1 V=4;nodes=2 V=1 TY=3;nodes=3 V=2;nodes=4 V=4 TX=2 SX=1;nodes=5;nodes=6 V=2",
     132, 17, 0, 65535),
    ("integer_unsharp", None, 2048, 2048, 0, 255),
]


@pytest.mark.parametrize("name,fixed,w,h,lo,hi", INT_CASES)
def test_integer_pipelines_bit_exact(name, fixed, w, h, lo, hi):
    _say(f"integer {name} {fixed} {w}x{h}")
    spec = getattr(P, name)()
    img = synth.integer_image(w + h, 1, h, w, lo, hi)
    kw = {"mode": "fixed", "fixed": fixed} if fixed else {"mode": "unfused"}
    got, _ = run_gpu(spec, {"img": img}, **kw)
    if fixed is None:
        fused, _ = run_gpu(spec, {"img": img}, mode="fixed", fixed="nodes=1,2,3,4 V=4 TX=1 SX=0 TY=32 PF=2")
        for k in got:
            assert np.array_equal(got[k], fused[k])
    ref = oracle.evaluate(spec, {"img": img})
    for k, r in ref.items():
        if r.dtype == np.int64:
            assert np.array_equal(got[k], r), f"{k}: max diff {np.abs(got[k] - r).max()}"
        else:
            assert_normwise(got[k], r, 1e-5, k)


def test_integer_saturation_corners():
    _say("integer saturation")
    spec = P.integer_unsharp()
    img = np.full((1, 40, 300), 255, dtype=np.int64)
    img[:, :, 150:] = 0
    img[:, 20:, 100:200] = 128
    got, _ = run_gpu(spec, {"img": img}, mode="fixed", fixed="nodes=1,2,3,4 V=4 TX=1 SX=0 TY=8")
    ref = oracle.evaluate(spec, {"img": img})
    assert ref["sharp"].max() == 255 and ref["sharp"].min() == 0 and ref["detail"].min() < 0
    for k in ref:
        assert np.array_equal(got[k], ref[k])


# ------------------------------- fused resampling: decimated stores, expansion
RESAMPLE_SPEC = {"inputs": [{"name": "img", "channels": 2}],
                 "stages": [P.blur_x("bx", "img"), P.blur_y("by", "bx"),
                            {"name": "d", "kind": "down2", "src": "by"},
                            {"name": "u", "kind": "up2", "src": "d"},
                            {"name": "s", "kind": "stencil", "src": "u", "kw": 3, "kh": 3, "ax": 1, "ay": 1,
                             "weights": [1, 2, 1, 2, 4, 2, 1, 2, 1], "scale": 1.0 / 16},
                            {"name": "o", "kind": "pointwise", "srcs": ["img", "s", "u"],
                             "expr": "s0 - s1 + 0.5 * s2", "channels": 2}],
                 "outputs": ["o", "d"]}


@pytest.mark.parametrize("fixed,w,h", [
    ("nodes=1,2 V=4 TX=1 SX=0 TY=8 dec=3;nodes=5,6 V=4 TX=1 SX=0 TY=16 exp=4", 132, 37),
    ("nodes=1,2 V=2 TX=2 SX=1 TY=5 PF=1 dec=3;nodes=5,6 V=2 TX=2 SX=1 TY=7 exp=4", 130, 17),
    ("nodes=1,2 V=1 TX=1 SX=0 TY=6 align=1 dec=3;nodes=5 V=1 exp=4;nodes=6 V=1 exp=4", 67, 13),
    (None, 2048, 1024),
    # interior waves with even V (the shared-coarse-column expansion)
    ("nodes=1,2 V=4 TX=1 SX=0 TY=8 dec=3;nodes=5,6 V=4 TX=1 SX=0 TY=16 exp=4", 1032, 37),
    ("nodes=1,2 V=2 TX=1 SX=0 TY=8 dec=3;nodes=5,6 V=2 TX=2 SX=1 TY=7 PF=1 exp=4", 602, 23),
    ("nodes=1,2 V=1 TX=2 SX=0 TY=8 dec=3;nodes=5,6 V=1 TX=2 SX=1 TY=7 PF=1 exp=4", 517, 29),
    ("nodes=1,2 V=1 TX=1 SX=0 TY=8 dec=3;nodes=5,6 V=1 TX=1 SX=0 TY=16 PF=2 align=1 exp=4", 389, 40),
])
def test_fused_resampling(fixed, w, h):
    _say(f"fused resampling {fixed} {w}x{h}")
    img = synth.uniform_image(9, 2, h, w)
    kw = {"mode": "fixed", "fixed": fixed} if fixed else {"mode": "analytic"}
    got, plan = run_gpu(RESAMPLE_SPEC, {"img": img}, **kw)
    if fixed is None:
        # the down2 is written by its source's group; the up2 is read by
        # expansion or folded into that group
        d = plan.describe()
        folded = any("dec=3" in ln and "nodes=" in ln and "4" in ln.split()[1][6:].split(",") for ln in d.splitlines())
        assert "dec=3" in d and ("exp=4" in d or folded), d
    ref = oracle.evaluate(RESAMPLE_SPEC, {"img": img})
    for k in ref:
        assert_normwise(got[k], ref[k], 1e-5, f"{k}: {plan.describe()}")


# ---------------------------------- one tile per workgroup (OTPTB ablation)
@pytest.mark.parametrize("name,fixed,w,h", [
    ("blur", "nodes=1,2 V=2 TX=1 TY=16 WPB=4 BLK=1", 300, 77),
    ("unsharp", "nodes=1,2,3,4 V=2 TX=1 TY=8 WPB=4 BLK=1", 260, 96),
    ("harris", "nodes=1,2,3,4,5,6,7,8,9,10 V=1 TX=1 TY=8 WPB=4 BLK=1", 200, 50),
    ("unsharp", "nodes=1,2,3,4 V=2 TX=1 TY=32 WPB=4 BLK=1", 600, 150),                # 85 KiB of LDS
    ("harris", "nodes=1,2,3,4,5,6,7,8,9,10 V=1 TX=1 TY=32 WPB=4 BLK=1", 300, 130),  # 114 KiB of LDS
])
def test_one_tile_per_workgroup(name, fixed, w, h):
    _say(f"otptb {name} {fixed} {w}x{h}")
    spec = {"blur": BLUR, "unsharp": UM, "harris": P.harris()}[name]
    img = synth.uniform_image(11, spec["inputs"][0]["channels"], h, w)
    got, _ = run_gpu(spec, {"img": img}, mode="fixed", fixed=fixed)
    ref = oracle.evaluate(spec, {"img": img}, keep_all=(name == "unsharp"))
    if name == "unsharp":
        check_unsharp(got["mask"], img, 1e-5, UM)
    else:
        for k in spec["outputs"]:
            assert_normwise(got[k], ref[k], 1e-5, fixed)


# ------------------------------------------------ full-size configured workloads
def test_pyramid_batch_full_workload():
    """The configured batch (64 pairs, sides uniform in 512..4096) through the
    analytical schedule in one persistent launch per group; the three
    smallest images are checked entirely against the oracle, every image for
    finiteness."""
    import torch
    import paper_1909_07190_amd as wt
    spec = P.pyramid_blend(4)
    sizes = synth.batch_sizes(4, 64)
    _say(f"pyramid full batch {len(sizes)} pairs")
    dev = torch.device("cuda:0")
    tin, tout = [], []
    for i, (w, h) in enumerate(sizes):
        a = torch.from_numpy(synth.uniform_image(4000 + 2 * i, 1, h, w)).to(dev)
        b = torch.from_numpy(synth.uniform_image(4001 + 2 * i, 1, h, w)).to(dev)
        m = torch.from_numpy(synth.ramp_mask(h, w)).to(dev)
        tin.append([a, b, m])
        tout.append([torch.full((1, h, w), float("nan"), device=dev)])
    mw, mh = sorted(sizes, key=lambda s: s[0] * s[1])[len(sizes) // 2]
    plan = wt.from_spec(spec).plan(mw, mh, mode="analytic", any_width=True, batch_images=len(sizes))
    plan.run_batch(tin, tout)
    torch.cuda.synchronize()
    for i in range(len(sizes)):
        assert torch.isfinite(tout[i][0]).all(), f"image {i}"
    for i in sorted(range(len(sizes)), key=lambda k: sizes[k][0] * sizes[k][1])[:3]:
        w, h = sizes[i]
        ref = oracle.evaluate(spec, {"A": tin[i][0].cpu().numpy(), "B": tin[i][1].cpu().numpy(),
                                     "M": tin[i][2].cpu().numpy()})
        assert_normwise(tout[i][0].cpu().numpy(), ref[spec["outputs"][0]], 1e-5, f"image {i} {w}x{h}")


@pytest.mark.parametrize("seed", [200, 201, 202])
def test_random_dag_full_size(seed):
    """Random pipelines of the learned-scheduler workload at 2048 x 2048
    under the analytical schedule (fused groups, decimated stores, expanded
    up-sampling) against the oracle."""
    from synth import dags
    spec = dags.random_dag(seed)
    _say(f"random dag {seed}: {len(spec['stages'])} stages")
    imgs = {inp["name"]: synth.uniform_image(seed * 7 + k, 1, 2048, 2048) for k, inp in enumerate(spec["inputs"])}
    got, plan = run_gpu(spec, imgs, mode="analytic")
    ref = oracle.evaluate(spec, imgs)
    for k in spec["outputs"]:
        assert_normwise(got[k], ref[k], 1e-5, f"{k}: {plan.describe()}")


# ------------------------------------------- consumed live-outs in a group
BLUR_BOTH = dict(BLUR, outputs=["bx", "by"])


@pytest.mark.parametrize("fixed,w,h", [
    ("nodes=1,2 V=2 TX=1 SX=0 TY=8 PF=2", 300, 77),
    ("nodes=1,2 V=4 TX=2 SX=1 TY=5 PF=1 align=1", 516, 45),
    ("nodes=1,2 V=1 TX=1 TY=8 WPB=4 BLK=1", 200, 41),
])
def test_consumed_liveout_rows_stored(fixed, w, h):
    """Both blur passes are outputs: the horizontal pass is read by the
    vertical one inside the group, so its first rows of every tile come out
    of the warm-up steps and are stored there."""
    _say(f"consumed live-out {fixed} {w}x{h}")
    img = synth.dyadic_image(9, 1, h, w)
    got, _ = run_gpu(BLUR_BOTH, {"img": img}, mode="fixed", fixed=fixed)
    ref = oracle.evaluate(BLUR_BOTH, {"img": img})
    for k in BLUR_BOTH["outputs"]:
        assert_exact(got[k], ref[k], f"{fixed}: {k}")


# --------------------------------------------- achievable-bandwidth reference
@pytest.mark.parametrize("nbytes", [16, 4096 + 12, 3 * 2048 * 2048 * 4])
def test_stream_copy_reference(nbytes):
    """The library's streaming copy reproduces its source byte for byte,
    including a tail shorter than one 16-byte element."""
    import torch
    import paper_1909_07190_amd as wt
    _say(f"stream copy {nbytes} bytes")
    g = torch.Generator(device="cuda:0").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda:0", generator=g)
    dst = torch.zeros_like(src)
    wt.stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


# ------------------------------------- ghost columns of loaded rows (GH=1)
@pytest.mark.parametrize("name,fixed,w,h", [
    ("unsharp", "nodes=1,2,3,4 V=2 TX=1 SX=0 TY=32 PF=2 NT=1 GH=1", 2048, 2048),
    ("unsharp", "nodes=1,2,3,4 V=4 TX=1 SX=0 TY=16 PF=2 GH=1", 772, 45),
    ("unsharp", "nodes=1,2,3,4 V=1 TX=2 SX=0 TY=7 PF=1 GH=1", 301, 33),
    ("blur", "nodes=1,2 V=2 TX=1 SX=0 TY=8 PF=1 GH=1", 258, 77),
    ("harris", "nodes=1,2,3,4,5,6,7,8,9,10 V=2 TX=1 SX=0 TY=16 PF=2 GH=1", 516, 70),
])
def test_ghost_columns(name, fixed, w, h):
    """Loaded rows with ghost columns: aligned tiles with no horizontal
    overlap, against the oracle."""
    _say(f"ghost columns {name} {fixed} {w}x{h}")
    spec = {"blur": BLUR, "unsharp": UM, "harris": P.harris()}[name]
    img = synth.uniform_image(13, spec["inputs"][0]["channels"], h, w)
    got, plan = run_gpu(spec, {"img": img}, mode="fixed", fixed=fixed)
    assert "GH=1" in plan.describe()
    if name == "unsharp":
        check_unsharp(got["mask"], img, 1e-5, UM)
    else:
        ref = oracle.evaluate(spec, {"img": img})
        for k in spec["outputs"]:
            assert_normwise(got[k], ref[k], 1e-5, fixed)


# ------------------------------------------------- autotune schedule cache
def test_autotune_schedule_cache(tmp_path, monkeypatch):
    """An autotuned schedule is measured once per (pipeline, device, size
    bucket, options): a second plan in the same bucket measures nothing and
    takes the same schedule, which is also on disk; retune measures again."""
    import re
    import paper_1909_07190_amd as wt
    db = tmp_path / "measure.jsonl"
    monkeypatch.setenv("WT_MEASURE_DB", str(db))
    spec = P.unsharp_mask(channels=1)
    _say("autotune cache: first plan")

    def lines():
        return len(db.read_text().splitlines()) if db.exists() else 0

    def groups(plan):
        return [re.sub(r" batch_\S+", "", g) for g in plan.describe().strip().splitlines()]

    p1 = wt.from_spec(spec).plan(512, 256, mode="autotune", autotune_topk=2, cache_dir=str(tmp_path))
    n1 = lines()
    assert n1 > 0
    p2 = wt.from_spec(spec).plan(500, 250, mode="autotune", autotune_topk=2, cache_dir=str(tmp_path))
    assert lines() == n1 and groups(p2) == groups(p1)
    tsv = (tmp_path / "autotune.tsv").read_text().splitlines()
    assert len(tsv) == 1 and "\t" in tsv[0]
    img = synth.uniform_image(21, 1, 250, 500)
    got, _ = run_gpu(spec, {"img": img}, mode="autotune", autotune_topk=2, cache_dir=str(tmp_path))
    check_unsharp(got["mask"], img, 1e-5, spec)
    assert lines() == n1
    wt.from_spec(spec).plan(512, 256, mode="autotune", autotune_topk=2, cache_dir=str(tmp_path), retune=True)
    assert lines() > n1


# ---------------------------------------------------------------- histogram --

def _near_bin_edges(vals, bins, lo, hi, eps=1e-3):
    """Per channel, how many values of a stage (FP64, from the oracle) lie
    within eps of a bin edge, in bin units: the only values whose bin the
    device's FP32 evaluation of the stage may legitimately move."""
    t = (vals - lo) * (bins / (hi - lo))
    return [int(np.sum(np.abs(t[c] - np.round(t[c])) < eps)) for c in range(vals.shape[0])]


@pytest.mark.parametrize("mode,fixed", [
    ("analytic", None),
    ("fixed", "nodes=1,2 V=4 TX=1 SX=0 TY=16 PF=2 hst=3"),
    ("fixed", "nodes=1,2 V=1 TX=2 SX=1 TY=8 PF=1 WPB=2 hst=3"),
    ("unfused", None),
])
def test_histogram_full_size(mode, fixed):
    """A 256-bin histogram of the blurred 3x2048x2048 image, counted by the
    blur's fused group or by the lone kernel: every pixel counted once, and
    the counts equal the oracle's except where FP32 rounding of the blur
    moves a value across a bin edge (at most two counts per such value);
    on a dyadic image (every value exact in FP32) bit-exact."""
    spec = P.blur_histogram(channels=3, bins=256)
    _say(f"histogram 3x2048x2048 {mode} [{fixed}]")
    img = synth.uniform_image(41, 3, 2048, 2048)
    got, plan = run_gpu(spec, {"img": img}, mode=mode, fixed=fixed)
    if mode == "analytic":
        assert "hst=3" in plan.describe()
    ref = oracle.evaluate(spec, {"img": img}, keep_all=True)
    near = _near_bin_edges(ref["by"], 256, 0.0, 1.0)
    for c in range(3):
        assert got["h"][c].sum() == 2048 * 2048
        assert np.abs(got["h"][c] - ref["h"][c]).sum() <= 2 * near[c], (c, near[c])
    dy = synth.dyadic_image(42, 3, 2048, 2048)
    got, _ = run_gpu(spec, {"img": dy}, mode=mode, fixed=fixed)
    assert np.array_equal(got["h"], oracle.evaluate(spec, {"img": dy})["h"])


def test_histogram_u8_4096():
    spec = P.u8_histogram()
    _say("u8 histogram 4096x4096")
    img = synth.integer_image(43, 1, 4096, 4096, 0, 255)
    for mode in ("analytic", "unfused"):
        got, _ = run_gpu(spec, {"img": img}, mode=mode)
        assert np.array_equal(got["h"], oracle.evaluate(spec, {"img": img})["h"]), mode


def test_histogram_batch_and_replays():
    """Batched histograms of images of uneven sizes, from a hipGraph: each
    image's counts equal the oracle's, and replaying the graph (which clears
    the counts with a kernel node before accumulating) gives the same counts,
    not twice them."""
    import torch
    import paper_1909_07190_amd as wt
    spec = P.blur_histogram(channels=2, bins=128)
    sizes = [(1000, 517), (64, 33), (2047, 1500), (300, 2001)]
    _say(f"batched histogram {sizes}")
    imgs = [synth.dyadic_image(50 + k, 2, h, w) for k, (w, h) in enumerate(sizes)]
    plan = wt.from_spec(spec).plan(1000, 1000, mode="analytic", any_width=True, batch_images=len(sizes))
    assert "hst=3" in plan.describe()
    dev = torch.device("cuda:0")
    tin = [[torch.from_numpy(im).to(dev)] for im in imgs]
    for rep in range(3):
        tout = [[torch.full((2, 1, 128), 0x5A, dtype=torch.int32, device=dev)] for _ in sizes]
        plan.run_batch(tin, tout)
        torch.cuda.synchronize()
        for k, im in enumerate(imgs):
            ref = oracle.evaluate(spec, {"img": im})["h"]
            assert np.array_equal(tout[k][0].cpu().numpy().astype(np.int64), ref), (rep, k)
    # single-image runs of the same plan also start from zero every time
    single = wt.from_spec(spec).plan(300, 2001, mode="analytic")
    out = torch.full((2, 1, 128), 7, dtype=torch.int32, device=dev)
    for _ in range(2):
        single.run(tin[3], [out])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.int64), oracle.evaluate(spec, {"img": imgs[3]})["h"])


def test_equalize_full_size_and_batch():
    """Histogram equalisation of the blurred 3x2048x2048 image (the counts
    from the blur's kernel, the equalisation and blend in the next): on a
    dyadic image the equalised values equal the oracle's bit for bit; on a
    random image only pixels whose blurred value FP32 rounding may move
    across a bin edge may differ.  Then a batch of three sizes from a
    hipGraph: every image equalised by its own counts."""
    import torch
    import paper_1909_07190_amd as wt
    spec = P.blur_equalize(channels=3, bins=256)
    only = dict(spec, stages=spec["stages"][:4], outputs=["eq"])
    _say("equalize 3x2048x2048")
    dy = synth.dyadic_image(44, 3, 2048, 2048)
    got, plan = run_gpu(only, {"img": dy}, mode="analytic")
    assert "hst=3" in plan.describe()
    assert_exact(got["eq"], oracle.evaluate(only, {"img": dy})["eq"], "equalize dyadic")
    img = synth.uniform_image(45, 3, 2048, 2048)
    got, _ = run_gpu(spec, {"img": img}, mode="analytic")
    ref = oracle.evaluate(spec, {"img": img}, keep_all=True)
    near = sum(_near_bin_edges(ref["by"], 256, 0.0, 1.0, eps=1e-4))
    bad = int(np.sum(np.abs(got["out"] - ref["out"]) > 1e-5))
    assert bad <= near, (bad, near)
    sizes = [(700, 300), (129, 1000), (2048, 64)]
    _say(f"equalize batch {sizes}")
    imgs = [synth.dyadic_image(46 + k, 3, h, w) for k, (w, h) in enumerate(sizes)]
    bplan = wt.from_spec(only).plan(700, 300, mode="analytic", any_width=True, batch_images=3)
    dev = torch.device("cuda:0")
    tin = [[torch.from_numpy(im).to(dev)] for im in imgs]
    for rep in range(2):
        tout = [[torch.full((3, h, w), float("nan"), device=dev)] for (w, h) in sizes]
        bplan.run_batch(tin, tout)
        torch.cuda.synchronize()
        for k, im in enumerate(imgs):
            assert_exact(tout[k][0].cpu().numpy(), oracle.evaluate(only, {"img": im})["eq"], f"batch {rep} {k}")
