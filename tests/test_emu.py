"""Hybrid-tiling correctness on the CPU: the generated kernels, run by the
lane emulator (64 lock-stepped threads per wavefront, DPP / ds_bpermute /
readlane as exchanges), against the FP64 oracle.  Covers every producer-load
type (own VGPR, LDS sub-tile, other lane of the same / neighbouring register
sub-tile), both alignments, clamp fix-ups at all four image edges, channel-
mixing groups, FP16 intermediates and multi-level pyramids."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1909_07190_amd as wt
import synth
from synth import pipelines as P
from emu_runner import emulate
from wt_helpers import assert_exact, assert_normwise, check_unsharp

BLUR = P.gaussian_blur()
UM = P.unsharp_mask()
HARRIS = P.harris()
# Harris with gray = R and k = 1/32: on 0/1 images every intermediate is an
# integer or a multiple of 1/32, exact in FP32 and FP16.
HARRIS_EXACT = P.harris(gray_weights=(1.0, 0.0, 0.0), k=1.0 / 32)

BLUR_SCHED = [
    ("nodes=1,2 V=4 TX=1 SX=0 TY=16 PF=2", 256, 40),
    ("nodes=1,2 V=4 TX=2 SX=0 TY=8 PF=1 align=1", 516, 40),
    ("nodes=1,2 V=1 TX=2 SX=1 TY=5 PF=2 align=1", 131, 19),
    ("nodes=1,2 V=4 TX=2 SX=1 TY=13 PF=1", 260, 37),
    ("nodes=1,2 V=2 TX=3 SX=3 TY=4 PF=0", 90, 11),
    ("nodes=1,2 V=1 TX=1 SX=0 TY=3 PF=1", 7, 5),
]


@pytest.mark.parametrize("fixed,w,h", BLUR_SCHED)
def test_blur_emulated_exact(fixed, w, h):
    img = synth.dyadic_image(2, 1, h, w)
    got, _ = emulate(BLUR, {"img": img}, mode="fixed", fixed=fixed)
    assert_exact(got["by"], oracle.evaluate(BLUR, {"img": img})["by"], fixed)


@pytest.mark.parametrize("fixed,fp16", [
    ("nodes=1,2,3,4 V=4 TX=1 SX=0 TY=8 PF=2", False),
    ("nodes=1,2,3,4 V=2 TX=2 SX=1 TY=6 PF=1 align=1", False),
    ("nodes=1,2,3,4 V=4 TX=1 SX=0 TY=8 PF=2 fp16=1", True),
    ("nodes=1,2 V=4 TX=1 SX=0 TY=8 fp16=1;nodes=3,4 V=4 TX=1 SX=0 TY=8", True),
])
def test_unsharp_emulated(fixed, fp16):
    img = synth.uniform_image(5, 3, 29, 260)
    got, _ = emulate(UM, {"img": img}, mode="fixed", fixed=fixed, fp16=fp16)
    check_unsharp(got["mask"], img, 2e-3 if fp16 else 1e-5, UM)


HARRIS_SCHED = [
    "nodes=1,2,3,4,5,6,7,8,9,10 V=4 TX=1 SX=0 TY=8 PF=1",
    "nodes=1,2,3,4,5,6,7,8,9,10 V=1 TX=2 SX=1 TY=5 PF=1 align=1",
    "nodes=1,2,3 V=2 TX=1 SX=0 TY=8;nodes=4,5,6,7,8,9,10 V=2 TX=2 SX=1 TY=6 PF=0",
]


@pytest.mark.parametrize("fixed", HARRIS_SCHED)
def test_harris_emulated(fixed):
    h, w = 21, 152
    sq = synth.white_squares(np.zeros((3, h, w), np.float32), 5, count=6, side_lo=3, side_hi=12)
    got, _ = emulate(HARRIS_EXACT, {"img": sq}, mode="fixed", fixed=fixed)
    assert_exact(got["R"], oracle.evaluate(HARRIS_EXACT, {"img": sq})["R"], fixed)
    got, _ = emulate(HARRIS_EXACT, {"img": sq}, mode="fixed", fixed=fixed.replace(" PF", " fp16=1 PF"),
                     fp16=True)
    assert_exact(got["R"], oracle.evaluate(HARRIS_EXACT, {"img": sq})["R"], fixed + " fp16")
    img = synth.uniform_image(3, 3, h, w)
    got, _ = emulate(HARRIS, {"img": img}, mode="fixed", fixed=fixed)
    assert_normwise(got["R"], oracle.evaluate(HARRIS, {"img": img})["R"], 1e-5, fixed)


@pytest.mark.parametrize("mode", ["unfused", "analytic"])
def test_pyramid_emulated(mode):
    spec = P.pyramid_blend(4)
    h, w = 37, 45
    ins = {"A": synth.uniform_image(21, 1, h, w), "B": synth.uniform_image(22, 1, h, w),
           "M": synth.ramp_mask(h, w)}
    got, _ = emulate(spec, ins, mode=mode)
    assert_normwise(got["R0"], oracle.evaluate(spec, ins)["R0"], 1e-5, mode)


def test_pyramid_two_level_exact():
    spec = P.pyramid_blend(2)
    a, b = synth.dyadic_image(31, 1, 21, 33), synth.dyadic_image(32, 1, 21, 33)
    for m in (np.ones((1, 21, 33), np.float32), np.zeros((1, 21, 33), np.float32)):
        got, _ = emulate(spec, {"A": a, "B": b, "M": m}, mode="analytic")
        assert_exact(got["R0"], oracle.evaluate(spec, {"A": a, "B": b, "M": m})["R0"], "pyramid")


def test_batched_persistent_kernels_emulated():
    """Persistent batch kernels over images of different sizes (grid-stride
    loop with a deliberately small grid) equal the oracle per image."""
    from emu_runner import emulate_batch
    spec = P.unsharp_mask(channels=1)
    sizes = [(60, 17), (131, 40), (97, 9)]
    images = [{"img": synth.uniform_image(40 + i, 1, h, w)} for i, (w, h) in enumerate(sizes)]
    outs = emulate_batch(spec, images, nblocks=3, mode="fixed",
                         fixed="nodes=1,2,3,4 V=1 TX=2 SX=0 TY=8 PF=1")
    for inp, got in zip(images, outs):
        check_unsharp(got["mask"], inp["img"], 1e-5, spec)
    # one tile per workgroup, four waves sharing each tile
    outs = emulate_batch(spec, images, nblocks=2, mode="fixed", fixed="nodes=1,2,3,4 V=1 TX=1 TY=8 WPB=4 BLK=1")
    for inp, got in zip(images, outs):
        check_unsharp(got["mask"], inp["img"], 1e-5, spec)
    # ghost columns on loaded rows
    outs = emulate_batch(spec, images, nblocks=3, mode="fixed", fixed="nodes=1,2,3,4 V=1 TX=2 SX=0 TY=8 PF=1 GH=1")
    for inp, got in zip(images, outs):
        check_unsharp(got["mask"], inp["img"], 1e-5, spec)
    spec = P.pyramid_blend(3)
    sizes = [(45, 37), (30, 21)]
    images = [{"A": synth.uniform_image(50 + i, 1, h, w), "B": synth.uniform_image(60 + i, 1, h, w),
               "M": synth.ramp_mask(h, w)} for i, (w, h) in enumerate(sizes)]
    outs = emulate_batch(spec, images, nblocks=2, mode="analytic", any_width=True)
    for inp, got in zip(images, outs):
        assert_normwise(got["R0"], oracle.evaluate(spec, inp)["R0"], 1e-5, "batched pyramid")


# ------------------------------------------------------------ integer stages
INT_CASES = [
    (P.binomial_u8(), "nodes=1,2 V=4 TX=1 SX=0 TY=8 PF=2", 260, 29, 0, 255),
    (P.binomial_u8(), "nodes=1,2 V=1 TX=2 SX=1 TY=5 PF=1 align=1", 131, 19, 0, 255),
    (P.integer_unsharp(), "nodes=1,2,3,4 V=2 TX=2 SX=0 TY=6 PF=1", 150, 37, 0, 255),
    (P.integer_unsharp(), "nodes=1,2,3,4 V=4 TX=2 SX=1 TY=4 PF=2 align=1", 300, 13, 0, 255),
    (P.integer_unsharp(), "nodes=1 V=2 TY=4;nodes=2 V=1 TY=8;nodes=3,4 V=4 TY=16", 76, 21, 0, 255),
    (P.integer_gradient(), "nodes=1,2,3,4 V=2 TX=1 SX=0 TY=8;nodes=5;nodes=6 V=1", 90, 33, 0, 65535),
    (P.integer_gradient(), "nodes=1 V=4;nodes=2 V=1 TY=3;nodes=3 V=2;nodes=4 V=4 TX=2 SX=1;nodes=5;nodes=6 V=2",
     132, 17, 0, 65535),
]


@pytest.mark.parametrize("spec,fixed,w,h,lo,hi", INT_CASES)
def test_integer_pipelines_emulated_bit_exact(spec, fixed, w, h, lo, hi):
    img = synth.integer_image(w * h, 1, h, w, lo, hi)
    got, _ = emulate(spec, {"img": img}, mode="fixed", fixed=fixed)
    ref = oracle.evaluate(spec, {"img": img})
    for k, r in ref.items():
        if r.dtype == np.int64:
            assert got[k].dtype == np.int64 and np.array_equal(got[k], r), f"{k}: {fixed}"
        else:
            assert_normwise(got[k], r, 1e-5, f"{k}: {fixed}")


def test_integer_saturation_emulated():
    """All-255 input: the 8-bit sharpen saturates; a zero region clips at 0."""
    spec = P.integer_unsharp()
    img = np.full((1, 20, 70), 255, dtype=np.int64)
    img[:, :, 30:] = 0
    got, _ = emulate(spec, {"img": img}, mode="fixed", fixed="nodes=1,2,3,4 V=2 TX=1 SX=0 TY=8")
    ref = oracle.evaluate(spec, {"img": img})
    assert ref["sharp"].max() == 255 and ref["sharp"].min() == 0
    for k in ref:
        assert np.array_equal(got[k], ref[k])


# ------------------------------------------------- down2 fused into producer
DEC_SPEC = {"inputs": [{"name": "img", "channels": 2}],
            "stages": [P.blur_x("bx", "img"), P.blur_y("by", "bx"),
                       {"name": "d", "kind": "down2", "src": "by"},
                       {"name": "e", "kind": "pointwise", "srcs": ["d"], "expr": "s0 * 2", "channels": 2}],
            "outputs": ["e", "by"]}


@pytest.mark.parametrize("fixed,w,h", [
    ("nodes=1,2 V=4 TX=1 SX=0 TY=8 dec=3;nodes=4 V=1", 132, 21),
    ("nodes=1,2 V=2 TX=2 SX=1 TY=5 PF=1 dec=3;nodes=4 V=2", 130, 17),
    ("nodes=1,2 V=1 TX=1 SX=0 TY=6 align=1 dec=3;nodes=4 V=1", 67, 13),
])
def test_decimated_store_emulated(fixed, w, h):
    img = synth.dyadic_image(7, 2, h, w)
    got, _ = emulate(DEC_SPEC, {"img": img}, mode="fixed", fixed=fixed)
    ref = oracle.evaluate(DEC_SPEC, {"img": img})
    for k in ref:
        assert_exact(got[k], ref[k], f"{k}: {fixed}")


def test_decimated_only_output_emulated():
    """A member whose only consumer is the down2 is never stored itself."""
    spec = {"inputs": [{"name": "img", "channels": 1}],
            "stages": [P.blur_x("bx", "img"), P.blur_y("by", "bx"), {"name": "d", "kind": "down2", "src": "by"}],
            "outputs": ["d"]}
    img = synth.dyadic_image(8, 1, 29, 97)
    got, plan = emulate(spec, {"img": img}, mode="analytic", any_width=True)
    assert "dec=3" in plan.describe() and plan.num_groups == 1
    assert_exact(got["d"], oracle.evaluate(spec, {"img": img})["d"], plan.describe())


# ----------------------------------------- up2 read by expansion in a group
# node 1 = down2(img) (materialised), node 2 = up2(node 1) read by expansion,
# node 3 = 3x3 stencil of it, node 4 = pointwise of img, node 3 and node 2
EXP_SPEC = {"inputs": [{"name": "img", "channels": 1}],
            "stages": [{"name": "small", "kind": "down2", "src": "img"},
                       {"name": "u", "kind": "up2", "src": "small"},
                       {"name": "s", "kind": "stencil", "src": "u", "kw": 3, "kh": 3, "ax": 1, "ay": 1,
                        "weights": [1, 2, 1, 2, 4, 2, 1, 2, 1], "scale": 1.0 / 16},
                       {"name": "o", "kind": "pointwise", "srcs": ["img", "s", "u"], "expr": "s0 - s1 + 0.5 * s2",
                        "channels": 1}],
            "outputs": ["o"]}


@pytest.mark.parametrize("fixed,w,h,fp16", [
    ("nodes=1;nodes=3,4 V=4 TX=1 SX=0 TY=8 exp=2", 132, 21, False),
    ("nodes=1;nodes=3,4 V=2 TX=2 SX=1 TY=5 PF=1 exp=2", 130, 17, False),
    ("nodes=1;nodes=3,4 V=1 TX=1 SX=0 TY=6 align=1 exp=2", 67, 13, False),
    ("nodes=1;nodes=3 V=1 TY=4 exp=2;nodes=4 V=1 exp=2", 67, 13, False),
    ("nodes=1;nodes=3,4 V=1 TX=2 SX=0 TY=7 exp=2 fp16=1", 65, 15, True),
    # wide enough for interior waves (their even-V expansion path)
    ("nodes=1;nodes=3,4 V=4 TX=1 SX=0 TY=8 exp=2", 700, 21, False),
    ("nodes=1;nodes=3,4 V=2 TX=2 SX=1 TY=5 PF=1 exp=2", 602, 17, False),
    ("nodes=1;nodes=3,4 V=2 TX=1 SX=0 TY=6 align=1 exp=2", 390, 13, False),
    ("nodes=1;nodes=3,4 V=2 TX=1 SX=0 TY=8 exp=2 fp16=1", 402, 15, True),
    ("nodes=1;nodes=3,4 V=1 TX=1 SX=0 TY=6 exp=2", 261, 13, False),
    ("nodes=1;nodes=3,4 V=1 TX=2 SX=1 TY=5 PF=1 exp=2", 391, 17, False),
    ("nodes=1;nodes=3,4 V=1 TX=2 SX=0 TY=8 align=1 exp=2 fp16=1", 333, 11, True),
    # even V: coarse rows kept per lane, neighbours by DPP and edge ghosts
    ("nodes=1;nodes=3,4 V=4 TX=2 SX=0 TY=8 exp=2", 1100, 21, False),
    ("nodes=1;nodes=3,4 V=4 TX=2 SX=1 TY=6 exp=2 fp16=1", 1030, 13, True),
    ("nodes=1;nodes=3,4 V=2 TX=3 SX=0 TY=7 exp=2", 1001, 15, False),
])
def test_expanded_up2_emulated(fixed, w, h, fp16):
    img = synth.uniform_image(3, 1, h, w)
    got, _ = emulate(EXP_SPEC, {"img": img}, mode="fixed", fixed=fixed, fp16=fp16)
    ref = oracle.evaluate(EXP_SPEC, {"img": img})
    assert_normwise(got["o"], ref["o"], 2e-3 if fp16 else 1e-5, fixed)


def test_pyramid_schedule_expands_and_decimates():
    spec = P.pyramid_blend(3)
    img = {"A": synth.uniform_image(1, 1, 37, 70), "B": synth.uniform_image(2, 1, 37, 70),
           "M": synth.ramp_mask(37, 70)}
    got, plan = emulate(spec, img, mode="analytic", any_width=True)
    d = plan.describe()
    assert "exp=" in d and "dec=" in d
    ref = oracle.evaluate(spec, img)
    for k in ref:
        assert_normwise(got[k], ref[k], 1e-5, d)


# ---------------------------------- one tile per workgroup (OTPTB ablation)
@pytest.mark.parametrize("spec,fixed,w,h", [
    (BLUR, "nodes=1,2 V=1 TX=1 TY=8 BLK=1", 130, 21),
    (UM, "nodes=1,2,3,4 V=2 TX=1 TY=5 BLK=1", 200, 13),
    (HARRIS_EXACT, "nodes=1,2,3,4,5,6,7,8,9,10 V=1 TX=1 TY=8 BLK=1", 70, 19),
    (P.integer_unsharp(), "nodes=1,2,3,4 V=1 TX=2 TY=6 BLK=1", 150, 11),
    (UM, "nodes=1,2,3,4 V=1 TX=1 TY=16 WPB=4 BLK=1", 140, 37),
    (HARRIS_EXACT, "nodes=1,2,3,4,5,6,7,8,9,10 V=1 TX=1 TY=8 WPB=8 BLK=1", 90, 21),
    (BLUR, "nodes=1,2 V=2 TX=1 TY=8 WPB=16 BLK=1", 260, 20),
    (UM, "nodes=1,2,3,4 V=2 TX=1 TY=32 WPB=4 BLK=1", 300, 70),   # 85 KiB of LDS
])
def test_one_tile_per_workgroup_emulated(spec, fixed, w, h):
    if spec["inputs"][0].get("dtype") == "u8":
        img = synth.integer_image(5, 1, h, w, 0, 255)
    elif spec is HARRIS_EXACT:
        img = synth.white_squares(np.zeros((3, h, w), np.float32), 3, count=6, side_lo=3, side_hi=9)
    else:
        img = synth.dyadic_image(5, spec["inputs"][0]["channels"], h, w)
    got, _ = emulate(spec, {"img": img}, mode="fixed", fixed=fixed)
    ref = oracle.evaluate(spec, {"img": img})
    for k in ref:
        if ref[k].dtype == np.int64:
            assert np.array_equal(got[k], ref[k]), fixed
        else:
            assert_exact(got[k], ref[k], fixed)


# ------------------------------------------- consumed live-outs in a group
# An output that later stages of its own group read with vertical taps is
# computed ahead of the group's last stage: its first rows of each tile come
# out of the warm-up steps and must be stored from there.  Blur with both
# passes as outputs, and a 3-stage chain whose middle stage is an output.
BLUR_BOTH = dict(BLUR, outputs=["bx", "by"])
CHAIN3 = {
    "inputs": [{"name": "img", "channels": 1}],
    "stages": [
        {"name": "a", "kind": "stencil", "src": "img", "kw": 3, "kh": 3, "ax": 1, "ay": 1,
         "weights": [1.0, 2.0, 1.0, 2.0, 4.0, 2.0, 1.0, 2.0, 1.0], "scale": 0.0625},
        {"name": "b", "kind": "pointwise", "srcs": ["a"], "expr": "0.5 * s0 + 0.25", "channels": 1},
        {"name": "c", "kind": "stencil", "src": "b", "kw": 1, "kh": 5, "ax": 0, "ay": 2,
         "weights": [1.0, 4.0, 6.0, 4.0, 1.0], "scale": 0.0625},
        {"name": "d", "kind": "stencil", "src": "c", "kw": 3, "kh": 3, "ax": 1, "ay": 1,
         "weights": [1.0, 1.0, 1.0, 1.0, 0.0, 1.0, 1.0, 1.0, 1.0], "scale": 0.125},
    ],
    "outputs": ["a", "c", "d"],
}


@pytest.mark.parametrize("spec,fixed,w,h", [
    (BLUR_BOTH, "nodes=1,2 V=2 TX=1 SX=0 TY=8 PF=2", 140, 37),
    (BLUR_BOTH, "nodes=1,2 V=4 TX=2 SX=1 TY=5 PF=1 align=1", 260, 23),
    (BLUR_BOTH, "nodes=1,2 V=1 TX=1 TY=6 BLK=1", 70, 19),
    (CHAIN3, "nodes=1,2,3,4 V=2 TX=1 SX=0 TY=8 PF=1", 132, 35),
    (CHAIN3, "nodes=1,2,3,4 V=1 TX=2 SX=1 TY=3 PF=0 align=1", 131, 17),
    (CHAIN3, "nodes=1,2;nodes=3,4 V=4 TX=1 SX=0 TY=16 PF=2", 264, 41),
    (CHAIN3, "nodes=1,2,3,4 V=1 TX=1 TY=8 BLK=1", 70, 21),
])
def test_consumed_liveout_rows_stored(spec, fixed, w, h):
    img = synth.dyadic_image(9, 1, h, w)
    got, _ = emulate(spec, {"img": img}, mode="fixed", fixed=fixed)
    ref = oracle.evaluate(spec, {"img": img})
    for k in spec["outputs"]:
        assert_exact(got[k], ref[k], f"{fixed}: {k}")


@pytest.mark.parametrize("seed", [200, 201])
def test_random_pipeline_analytic_emulated(seed):
    """Random pipelines of the learned-scheduler workload under the
    analytical schedule (fused groups with consumed live-outs, decimated
    stores, expanded up-sampling) against the oracle."""
    from synth import dags
    spec = dags.random_dag(seed)
    imgs = {inp["name"]: synth.uniform_image(seed * 7 + k, 1, 38, 132) for k, inp in enumerate(spec["inputs"])}
    got, plan = emulate(spec, imgs, mode="analytic")
    ref = oracle.evaluate(spec, imgs)
    for k in spec["outputs"]:
        assert_normwise(got[k], ref[k], 1e-5, f"{k}: {plan.describe()}")


# ------------------------------------- ghost columns of loaded rows (GH=1)
# Loaded rows carry the columns their direct consumers read past the tile's
# slots, so those consumers are valid on every slot and tiles are aligned.
@pytest.mark.parametrize("spec,fixed,w,h", [
    (UM, "nodes=1,2,3,4 V=2 TX=1 SX=0 TY=8 PF=2 GH=1", 392, 21),
    (UM, "nodes=1,2,3,4 V=1 TX=2 SX=0 TY=5 PF=1 GH=1", 300, 13),
    (UM, "nodes=1,2,3,4 V=4 TX=1 SX=0 TY=6 PF=2 NT=1 GH=1", 772, 11),
    (UM, "nodes=1,2,3,4 V=1 TX=1 SX=0 TY=4 PF=0 GH=1", 61, 7),
    (UM, "nodes=1,2 V=2 TX=1 SX=0 TY=8 GH=1;nodes=3,4 V=2 TX=1 SX=0 TY=8 GH=1", 260, 17),
    (BLUR, "nodes=1,2 V=1 TX=3 SX=0 TY=8 GH=1", 400, 12),
    (HARRIS_EXACT, "nodes=1,2,3,4,5,6,7,8,9,10 V=2 TX=1 SX=0 TY=8 PF=1 GH=1", 260, 19),
    (CHAIN3, "nodes=1,2,3,4 V=2 TX=1 SX=0 TY=8 PF=1 GH=1", 390, 23),
    (P.integer_unsharp(), "nodes=1,2,3,4 V=4 TX=1 SX=0 TY=6 PF=2 GH=1", 520, 13),
])
def test_ghost_columns_emulated(spec, fixed, w, h):
    if spec["inputs"][0].get("dtype") == "u8":
        img = synth.integer_image(7, 1, h, w, 0, 255)
    elif spec is HARRIS_EXACT:
        img = synth.white_squares(np.zeros((3, h, w), np.float32), 3, count=6, side_lo=3, side_hi=9)
    else:
        img = synth.dyadic_image(7, spec["inputs"][0]["channels"], h, w)
    got, plan = emulate(spec, {"img": img}, mode="fixed", fixed=fixed)
    assert "GH=1" in plan.describe()
    ref = oracle.evaluate(spec, {"img": img})
    for k in spec["outputs"]:
        if ref[k].dtype == np.int64:
            assert np.array_equal(got[k], ref[k]), fixed
        else:
            assert_exact(got[k], ref[k], f"{fixed}: {k}")


def test_ghost_columns_align_tiles():
    """With ghosts the unsharp mask's tiles are the full 64*V*TX columns
    (no overlap), so every tile starts on a 512-byte boundary."""
    import ctypes
    from emu_runner import GroupInfo
    import paper_1909_07190_amd as wt
    for gh, cols in ((0, 124), (1, 128)):
        plan = wt.from_spec(UM).plan(2048, 2048, mode="fixed", no_device=True, no_compile=True,
                                     fixed=f"nodes=1,2,3,4 V=2 TX=1 SX=0 TY=32 PF=2 NT=1 GH={gh}")
        gi = GroupInfo()
        wt._check(wt.lib.wt_plan_group_info(plan._h, 0, ctypes.byref(gi)))
        assert gi.tiles_x == -(-2048 // cols), (gh, gi.tiles_x)
    with pytest.raises(wt.WtError):
        wt.from_spec(UM).plan(256, 64, mode="fixed", no_device=True, no_compile=True,
                              fixed="nodes=1,2,3,4 V=2 TX=2 SX=1 TY=8 GH=1")


def _harris_255():
    spec = P.harris()
    spec["inputs"][0]["bound"] = 255.0
    return spec


def test_fp16_storage_follows_magnitude_bounds():
    """With inputs declared within [-255, 255], the Harris products and box
    sums can exceed FP16's range (|Ix|^2 <= 1020^2): only gray and the Sobel
    gradients are stored FP16, the rest stays FP32 (unfused plan, every
    intermediate in memory)."""
    import ctypes
    import paper_1909_07190_amd as wt
    from emu_runner import GroupInfo
    for spec, want in ((P.harris(), {"gray", "Ix", "Iy", "Ixx", "Iyy", "Ixy", "Sxx", "Syy", "Sxy"}),
                       (_harris_255(), {"gray", "Ix", "Iy"})):
        pipe = wt.from_spec(spec)
        plan = pipe.plan(256, 64, mode="unfused", fp16=True, no_device=True)
        names = {v: k for k, v in pipe.names.items()}
        half = set()
        for g in range(plan.num_groups):
            gi = GroupInfo()
            wt._check(wt.lib.wt_plan_group_info(plan._h, g, ctypes.byref(gi)))
            half |= {names[gi.liveouts[i]] for i in range(gi.nliveouts) if gi.liveout_half[i]}
        assert half == want


def test_fp16_harris_on_0_255_inputs_stays_finite():
    """Harris on 0..255-scaled RGB with FP16 intermediates, fused: the
    stages past FP16's range keep FP32, so the response is finite and within
    the FP16 tolerance of the oracle."""
    spec = _harris_255()
    img = (synth.uniform_image(11, 3, 21, 260) * 255.0).astype(np.float32)
    got, _ = emulate(spec, {"img": img}, mode="fixed", fp16=True,
                     fixed="nodes=1,2,3,4,5,6,7,8,9,10 V=4 TX=1 SX=0 TY=8 PF=1 fp16=1")
    assert_normwise(got["R"], oracle.evaluate(spec, {"img": img})["R"], 2e-3, "harris 0..255 fp16")


# ------------------------------------- folded up2: groups across two levels
# Laplacian band: node 1 bx, 2 by, 3 G1 = down2(by), 4 U = up2(G1),
# 5 L = img - U, 6 c1 = blur_x(G1).  With G1 written decimated by the group
# of by, U is computed from by's rows in the same kernel (the 2x expansion of
# by's even samples), so the band needs no pass over the coarse level.
LAPBAND = P.laplacian_band()
FOLD_CASES = [
    ("nodes=1,2,4,5 V=1 TX=2 SX=0 TY=8 PF=1 dec=3;nodes=6 V=1", 130, 40),
    ("nodes=1,2,4,5 V=1 TX=1 SX=0 TY=5 PF=2 dec=3;nodes=6 V=1", 67, 9),
    ("nodes=1,2,4,5 V=1 TX=1 SX=0 TY=16 PF=2 dec=3;nodes=6 V=1", 400, 30),
    ("nodes=1,2,4,5 V=2 TX=2 SX=1 TY=8 PF=1 dec=3;nodes=6 V=2", 262, 34),
    ("nodes=1,2,4,5 V=4 TX=1 SX=0 TY=16 PF=2 dec=3;nodes=6 V=4", 516, 40),
    ("nodes=1,2,4,5 V=1 TX=2 SX=0 TY=8 PF=1 align=1 dec=3;nodes=6 V=1", 131, 21),
    ("nodes=1,2,4,5 V=2 TX=3 SX=3 TY=4 PF=0 dec=3;nodes=6 V=2", 90, 11),
    # the folded up2 as a live-out of its group, read by a later group
    ("nodes=1,2,4 V=1 TX=1 SX=0 TY=8 dec=3;nodes=5 V=1;nodes=6 V=1", 33, 21),
]


@pytest.mark.parametrize("fixed,w,h", FOLD_CASES)
def test_folded_up2_emulated_exact(fixed, w, h):
    """Dyadic inputs keep every intermediate exact (2^-18 grid), so any
    indexing, parity or edge-clamp error shows as a bit mismatch; odd and
    even sizes cover both right/bottom coarse clamps."""
    img = synth.dyadic_image(9, 1, h, w)
    got, _ = emulate(LAPBAND, {"img": img}, mode="fixed", fixed=fixed)
    ref = oracle.evaluate(LAPBAND, {"img": img})
    for k in ref:
        assert_exact(got[k], ref[k], f"{k}: {fixed}")


def test_folded_up2_fp16_emulated():
    fixed = "nodes=1,2,4,5 V=2 TX=2 SX=0 TY=8 PF=2 fp16=1 dec=3;nodes=6 V=2 fp16=1"
    img = synth.uniform_image(10, 1, 37, 262)
    got, _ = emulate(LAPBAND, {"img": img}, mode="fixed", fixed=fixed, fp16=True)
    ref = oracle.evaluate(LAPBAND, {"img": img})
    for k in ref:
        assert_normwise(got[k], ref[k], 2e-3, f"{k}: {fixed}")


def test_fusion_search_folds_the_band():
    """The analytical search puts the expansion of by's decimation, and the
    band that reads it, into the group of by."""
    img = synth.dyadic_image(11, 1, 29, 97)
    got, plan = emulate(LAPBAND, {"img": img}, mode="analytic", any_width=True)
    first = plan.describe().splitlines()[0]
    assert "nodes=1,2,4,5 " in first and "dec=3" in first, plan.describe()
    ref = oracle.evaluate(LAPBAND, {"img": img})
    for k in ref:
        assert_exact(got[k], ref[k], plan.describe())


def _pyramid_fold_schedule(spec, levels, cfg, m_apart):
    """Every level's analysis in one group: blurs of A, B (and M), the
    decimated next level, the folded expansions, the bands and their blend;
    then the coarsest blend and the collapse, expanding each coarser result."""
    import paper_1909_07190_amd as wt
    ids = wt.from_spec(spec).names

    def grp(nodes, dec=(), exp=(), c=cfg):
        s = "nodes=" + ",".join(str(ids[n]) for n in sorted(nodes, key=lambda n: ids[n])) + " " + c
        if dec:
            s += " dec=" + ",".join(str(ids[n]) for n in dec)
        if exp:
            s += " exp=" + ",".join(str(ids[n]) for n in exp)
        return s

    top = levels - 1
    groups = []
    for l in range(top):
        body = [f"Abx{l}", f"Aby{l}", f"AU{l}", f"AL{l}", f"Bbx{l}", f"Bby{l}", f"BU{l}", f"BL{l}", f"Lb{l}"]
        dec = [f"AG{l + 1}", f"BG{l + 1}"]
        if m_apart:
            groups.append(grp([f"Mbx{l}", f"Mby{l}"], dec=[f"MG{l + 1}"]))
        else:
            body += [f"Mbx{l}", f"Mby{l}"]
            dec.append(f"MG{l + 1}")
        groups.append(grp(body, dec=dec))
    groups.append(grp([f"Lb{top}"]))
    for l in range(top - 1, -1, -1):
        groups.append(grp([f"R{l}"], exp=[f"RU{l}"]))
    return "\n".join(groups)


@pytest.mark.parametrize("cfg,m_apart", [("V=1 TX=1 SX=0 TY=8 PF=2", False), ("V=1 TX=2 SX=1 TY=5 PF=1", True),
                                         ("V=4 TX=1 SX=0 TY=8 PF=2", False)])
def test_pyramid_folded_levels_emulated(cfg, m_apart):
    """The blend with each level's bands computed in the pass that
    decimates it: exact on a two-level pyramid with dyadic inputs and a 0/1
    mask, and within 1e-5 on the four-level pyramid."""
    spec2 = P.pyramid_blend(2)
    h, w = 21, 33
    a, b = synth.dyadic_image(31, 1, h, w), synth.dyadic_image(32, 1, h, w)
    for m in (np.ones((1, h, w), np.float32), np.zeros((1, h, w), np.float32)):
        ins = {"A": a, "B": b, "M": m}
        got, _ = emulate(spec2, ins, mode="fixed", fixed=_pyramid_fold_schedule(spec2, 2, cfg, m_apart),
                         any_width=True)
        assert_exact(got["R0"], oracle.evaluate(spec2, ins)["R0"], cfg)
    spec4 = P.pyramid_blend(4)
    h, w = (37, 70) if "V=1" in cfg else (37, 1203)
    ins = {"A": synth.uniform_image(21, 1, h, w), "B": synth.uniform_image(22, 1, h, w), "M": synth.ramp_mask(h, w)}
    got, _ = emulate(spec4, ins, mode="fixed", fixed=_pyramid_fold_schedule(spec4, 4, cfg, m_apart), any_width=True)
    assert_normwise(got["R0"], oracle.evaluate(spec4, ins)["R0"], 1e-5, cfg)


def test_pyramid_folded_batch_emulated():
    """Batched kernels of the folded schedule over images of different
    sizes, with a grid smaller than the work."""
    from emu_runner import emulate_batch
    spec = P.pyramid_blend(3)
    sizes = [(45, 37), (30, 21), (66, 40)]
    images = [{"A": synth.uniform_image(70 + i, 1, h, w), "B": synth.uniform_image(80 + i, 1, h, w),
               "M": synth.ramp_mask(h, w)} for i, (w, h) in enumerate(sizes)]
    fixed = _pyramid_fold_schedule(spec, 3, "V=1 TX=1 SX=0 TY=8 PF=2", False)
    outs = emulate_batch(spec, images, nblocks=2, mode="fixed", fixed=fixed, any_width=True)
    for inp, got in zip(images, outs):
        assert_normwise(got["R0"], oracle.evaluate(spec, inp)["R0"], 1e-5, "batched folded pyramid")



@pytest.mark.parametrize("case", ["pyramid", "harris"])
def test_whole_pipeline_kernel_emulated(case):
    """The whole-pipeline kernel (every group of the batch in one launch,
    chunks of tiles taken in ticket order, per-image completion counters)
    equals the per-group batched kernels bit for bit and the oracle; every
    chunk is taken, every group completes every tile of every image, and no
    wait gives up."""
    from emu_runner import emulate_batch, emulate_whole
    if case == "harris":
        spec = HARRIS
        sizes = [(70, 19), (131, 33)]
        images = [{"img": synth.uniform_image(90 + i, 3, h, w)} for i, (w, h) in enumerate(sizes)]
        kw = dict(mode="fixed", fixed="nodes=1,2,3,4,5,6,7,8,9,10 V=1 TX=2 SX=0 TY=8 PF=1")
        out = "R"
    else:
        spec = P.pyramid_blend(3)
        sizes = [(45, 37), (66, 21)]
        images = [{"A": synth.uniform_image(70 + i, 1, h, w), "B": synth.uniform_image(80 + i, 1, h, w),
                   "M": synth.ramp_mask(h, w)} for i, (w, h) in enumerate(sizes)]
        kw = dict(mode="analytic", any_width=True)
        out = "R0"
    ref = emulate_batch(spec, images, nblocks=2, **kw)
    # one wave taking every chunk in order, then eight waves at once taking
    # one-tile chunks as they free up (waits on producers still running
    # really block; the lanes of a wave meet at its agent-scope fences)
    # (the second run takes the library's own chunk table and producer
    # masks: one-tile chunks for a million resident waves)
    for chunk, conc, rw in ((3, 0, None), (1, 8, 10 ** 6)):
        got, ctr, deps = emulate_whole(spec, images, chunk=chunk, concurrent=conc, resident_waves=rw, **kw)
        for inp, g, r in zip(images, got, ref):
            assert np.array_equal(g[out], r[out]), (case, conc)
            assert_normwise(g[out], oracle.evaluate(spec, inp)[out], 1e-5, case)
        ngroups, nimg = len(deps), len(images)
        assert ctr[ngroups * nimg + 1] == 0  # status: no wait gave up
        assert ctr[ngroups * nimg] >= 1 and all(ctr[:ngroups * nimg] > 0)
    if case != "harris":
        assert any(deps) and deps[0] == 0  # the first group reads only inputs


WIDE = P.wide_chain()
WIDE_NODES = ",".join(str(i) for i in range(1, 12))


@pytest.mark.parametrize("cfg", [
    "V=1 TX=3 SX=0 TY=5 PF=1 align=1",   # registers only: lanes exchange across two sub-tiles back
    "V=1 TX=3 SX=1 TY=5 PF=2 align=1",   # the wrapping lanes read an LDS sub-tile
    "V=1 TX=4 SX=2 TY=4 PF=1 align=1",   # both sub-tiles of some reads in LDS
    "V=1 TX=3 SX=3 TY=8 PF=1 align=1",   # every sub-tile in LDS
])
def test_lookback_across_sub_tiles_emulated(cfg):
    """The input edge of a ten-stencil chain spans 70 columns under the
    right-hyperplane skew: more than one wavefront at one element per lane,
    so lanes read sub-tiles two back (Appendix A's multi-sub-tile lookback)."""
    img = synth.uniform_image(31, 1, 9, 200)
    fixed = f"nodes={WIDE_NODES} {cfg}"
    got, plan = emulate(WIDE, {"img": img}, mode="fixed", fixed=fixed)
    assert "align=1" in plan.describe()
    gi = wt.GroupInfo()
    wt._check(wt.lib.wt_plan_group_info(plan._h, 0, ctypes.byref(gi)))
    assert gi.tiles_x >= 2 and gi.tiles_y >= 2  # interior and edge tiles, a ragged last row
    assert_normwise(got["out"], oracle.evaluate(WIDE, {"img": img})["out"], 1e-5, fixed)


def test_lookback_source_reads_two_sub_tiles_back():
    """The generated source for the chain exchanges lanes between sub-tiles
    k-1 and k-2 (lane distance 70 = 64 + 6)."""
    src = wt.from_spec(WIDE).plan(300, 13, mode="fixed", fixed=f"nodes={WIDE_NODES} V=1 TX=3 SX=0 TY=5 PF=1 align=1",
                                  no_device=True, no_compile=True).source(0)
    assert ", 6, lane)" in src


# ---------------------------------------------------------------- histogram --

HIST = P.blur_histogram(channels=2, bins=64)


@pytest.mark.parametrize("mode,fixed", [
    ("fixed", "nodes=1,2 V=4 TX=1 SX=0 TY=8 PF=1 hst=3"),
    ("fixed", "nodes=1,2 V=1 TX=2 SX=1 TY=5 PF=1 hst=3"),     # LDS sub-tiles
    ("fixed", "nodes=1,2 V=2 TX=2 SX=0 TY=6 PF=2 align=1 hst=3"),  # right-hyperplane skew
    ("fixed", "nodes=1,2 V=4 TX=1 SX=0 TY=8 PF=1 WPB=2 hst=3"),
    ("unfused", None),                                        # the lone histogram kernel
    ("analytic", None),
])
def test_histogram_emulated_exact(mode, fixed):
    """Counts of the blurred dyadic image, fused into the blur's group (each
    wave counts its tile's output range into LDS bins, then adds them to the
    output) or counted by the lone kernel: bit-exact against the oracle."""
    img = synth.dyadic_image(2, 2, 41, 300)
    got, plan = emulate(HIST, {"img": img}, mode=mode, fixed=fixed)
    if mode == "analytic":
        assert "hst=3" in plan.describe()
    ref = oracle.evaluate(HIST, {"img": img})["h"]
    assert got["h"].shape == ref.shape and np.array_equal(got["h"], ref), (mode, fixed)


def test_histogram_of_a_leading_member_and_a_stored_source_emulated():
    """The histogram of the x-blur, which the y-blur reads (so its rows run
    ahead of the tile's): each row still counted once; and with the blurred
    image also an output, the group both stores and counts it."""
    img = synth.dyadic_image(3, 1, 37, 200)
    spec = P.blur_histogram(channels=1, bins=32, of="bx")
    got, _ = emulate(spec, {"img": img}, mode="fixed", fixed="nodes=1,2 V=2 TX=1 SX=0 TY=8 PF=1 hst=3")
    assert np.array_equal(got["h"], oracle.evaluate(spec, {"img": img})["h"])
    spec = P.blur_histogram(channels=1, bins=32, keep_blur=True)
    got, _ = emulate(spec, {"img": img}, mode="fixed", fixed="nodes=1,2 V=4 TX=1 SX=0 TY=8 PF=1 hst=3")
    ref = oracle.evaluate(spec, {"img": img})
    assert np.array_equal(got["h"], ref["h"])
    assert_exact(got["by"], ref["by"], "stored source")


@pytest.mark.parametrize("mode,fixed", [("fixed", "nodes=1,2 V=4 TX=1 SX=0 TY=8 PF=1 hst=3"), ("unfused", None)])
def test_histogram_u8_emulated_exact(mode, fixed):
    spec = P.u8_histogram()
    img = synth.integer_image(7, 1, 29, 260, 0, 255)
    got, _ = emulate(spec, {"img": img}, mode=mode, fixed=fixed)
    assert np.array_equal(got["h"], oracle.evaluate(spec, {"img": img})["h"])


def test_histogram_batch_emulated_exact():
    """Batched kernels over images of three sizes: every image's histogram
    accumulates in its own output."""
    from emu_runner import emulate_batch
    images = [{"img": synth.dyadic_image(10 + i, 2, h, w)} for i, (w, h) in enumerate([(300, 41), (70, 9), (131, 66)])]
    outs = emulate_batch(HIST, images, mode="fixed", fixed="nodes=1,2 V=2 TX=1 SX=0 TY=8 PF=1 hst=3")
    for im, o in zip(images, outs):
        assert np.array_equal(o["h"], oracle.evaluate(HIST, im)["h"])


def test_histogram_in_a_channel_mixing_group_emulated():
    """A group whose gray stage mixes channels keeps all three channels of
    the x-blur in one wave: the histogram of that blur counts each channel
    slot into its own bins."""
    spec = {"inputs": [{"name": "img", "channels": 3}],
            "stages": [P.blur_x("bx", "img"),
                       {"name": "gray", "kind": "pointwise", "srcs": ["bx"],
                        "expr": "0.25 * s0[0] + 0.5 * s0[1] + 0.25 * s0[2]", "channels": 1},
                       {"name": "h", "kind": "hist", "src": "bx", "bins": 32, "lo": 0.0, "hi": 1.0}],
            "outputs": ["gray", "h"]}
    img = synth.dyadic_image(12, 3, 23, 150)
    got, plan = emulate(spec, {"img": img}, mode="fixed", fixed="nodes=1,2 V=2 TX=1 SX=0 TY=8 PF=1 hst=3")
    assert "chan_parallel=0" in plan.source(0)
    ref = oracle.evaluate(spec, {"img": img})
    assert np.array_equal(got["h"], ref["h"])
    assert_exact(got["gray"], ref["gray"], "gray")


EQ = P.blur_equalize(channels=2, bins=64)
EQ_ONLY = dict(EQ, stages=EQ["stages"][:4], outputs=["eq"])


@pytest.mark.parametrize("mode,fixed", [
    ("analytic", None),
    ("unfused", None),
    ("fixed", "nodes=1,2 V=2 TX=1 SX=0 TY=8 PF=1 hst=3;nodes=4,5 V=1 TX=2 SX=1 TY=5 PF=1"),
    ("fixed", "nodes=1,2 V=4 TX=1 SX=0 TY=8 PF=1 hst=3;nodes=4,5 V=4 TX=1 SX=0 TY=6 PF=2 WPB=2"),
])
def test_equalize_emulated(mode, fixed):
    """Histogram equalisation reading the counts a previous kernel
    accumulated: each tile loads the histogram whole and forms its
    cumulative counts in LDS; the equalised values (exact on dyadic inputs)
    and their blend with the input against the oracle."""
    img = synth.dyadic_image(3, 2, 41, 300)
    got, plan = emulate(EQ_ONLY, {"img": img}, mode=mode, fixed=fixed.replace("4,5", "4") if fixed else None)
    assert_exact(got["eq"], oracle.evaluate(EQ_ONLY, {"img": img})["eq"], f"{mode} {fixed}")
    got, plan = emulate(EQ, {"img": img}, mode=mode, fixed=fixed)
    if mode == "analytic":
        d = plan.describe()
        assert "hst=3" in d and " nodes=4,5 " in d
    assert_normwise(got["out"], oracle.evaluate(EQ, {"img": img})["out"], 1e-6, f"{mode} {fixed}")


def test_equalize_refuses_its_own_histogram_group():
    """A group may not read the counts it accumulates."""
    with pytest.raises(wt.WtError):
        wt.from_spec(EQ).plan(64, 64, mode="fixed", fixed="nodes=1,2,4,5 V=1 TX=1 SX=0 TY=8 hst=3",
                              no_device=True, no_compile=True)


def test_equalize_batch_emulated_exact():
    """Batched kernels whose waves loop over several tiles of images of three
    sizes: every tile reloads its own image's cumulative counts."""
    from emu_runner import emulate_batch
    images = [{"img": synth.dyadic_image(20 + i, 2, h, w)} for i, (w, h) in enumerate([(300, 41), (70, 9), (131, 66)])]
    outs = emulate_batch(EQ_ONLY, images, nblocks=3,
                         mode="fixed", fixed="nodes=1,2 V=2 TX=1 SX=0 TY=8 PF=1 hst=3;nodes=4 V=1 TX=2 SX=0 TY=8 PF=1")
    for im, o in zip(images, outs):
        assert_exact(o["eq"], oracle.evaluate(EQ_ONLY, im)["eq"], "batched equalize")


def test_histogram_of_an_input_and_of_a_decimated_stage_emulated():
    """A histogram of a pipeline input, and one of a down2 stage (level 1),
    are counted by the lone kernel over that node's own domain."""
    spec = {"inputs": [{"name": "img", "channels": 1}],
            "stages": [{"name": "h0", "kind": "hist", "src": "img", "bins": 16, "lo": 0.0, "hi": 1.0},
                       P.blur_x("bx", "img"),
                       {"name": "d", "kind": "down2", "src": "bx"},
                       {"name": "h1", "kind": "hist", "src": "d", "bins": 8, "lo": 0.0, "hi": 1.0}],
            "outputs": ["h0", "h1"]}
    img = synth.dyadic_image(13, 1, 37, 141)
    for mode in ("analytic", "unfused"):
        got, _ = emulate(spec, {"img": img}, mode=mode)
        ref = oracle.evaluate(spec, {"img": img})
        assert np.array_equal(got["h0"], ref["h0"]) and np.array_equal(got["h1"], ref["h1"]), mode
        assert got["h1"].sum() == 19 * 71


def test_equalize_u8_emulated_exact():
    """Equalisation of an 8-bit blurred image by its 256-bin histogram
    (integer values, exact bins), fused with the blur's kernel's successor."""
    spec = P.u8_histogram()
    spec = dict(spec, stages=spec["stages"] + [{"name": "eq", "kind": "equalize", "src": "by", "hist": "h"}],
                outputs=["eq", "h"])
    img = synth.integer_image(17, 1, 33, 200, 0, 255)
    for mode in ("analytic", "unfused"):
        got, _ = emulate(spec, {"img": img}, mode=mode)
        ref = oracle.evaluate(spec, {"img": img})
        assert np.array_equal(got["h"], ref["h"]), mode
        assert_exact(got["eq"], ref["eq"], mode)


def test_histogram_with_fp16_intermediates_emulated():
    """With FP16 intermediates the fused group counts the FP16-rounded blur:
    every pixel is counted once, and the counts differ from the FP64
    oracle's only by values that rounding to FP16 moves across a bin edge."""
    spec = P.blur_histogram(channels=1, bins=64)
    img = synth.uniform_image(18, 1, 40, 260)
    got, _ = emulate(spec, {"img": img}, mode="fixed", fixed="nodes=1,2 V=2 TX=1 SX=0 TY=8 PF=1 hst=3", fp16=True)
    ref = oracle.evaluate(spec, {"img": img}, keep_all=True)
    assert got["h"].sum() == 40 * 260
    t = ref["by"] * 64
    near = int(np.sum(np.abs(t - np.round(t)) < 64 * 2.0 ** -11))  # within an FP16 step of an edge
    assert np.abs(got["h"] - ref["h"]).sum() <= 2 * near
