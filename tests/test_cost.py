"""Pins of the scheduler's models: Section 4's warp geometry, Algorithm 2 on
the paper's motivating blur (GTX 1080Ti, Table 1), gfx950 occupancy rules,
and the fusion DP against exhaustive enumeration."""
import ctypes

import pytest

import paper_1909_07190_amd as wt
from synth import dags
from synth import pipelines as P

lib = wt.lib
lib.wt_alg2_eval.restype = ctypes.c_int
lib.wt_alg2_eval.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double)]
lib.wt_otpw_geometry.restype = ctypes.c_int
lib.wt_otpw_geometry.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int64)]
lib.wt_fusion_costs.restype = ctypes.c_int


def otpw(block, ws, tile, overlap):
    i3 = ctypes.c_int * 3
    w = i3()
    e = ctypes.c_int64()
    wt._check(lib.wt_otpw_geometry(i3(*block), ws, i3(*tile), i3(*overlap), w, ctypes.byref(e)))
    return tuple(w), e.value


def alg2(machine, smem, regs, warps, blocks=1000, tx=1000.0, ctx=1000.0, mem=1e4, comp=1e-6, ovl=0.0, w=None):
    d9 = ctypes.c_double * 9
    out = (ctypes.c_double * 12)()
    wv = (ctypes.c_double * 7)(*w) if w else None
    wt._check(lib.wt_alg2_eval(machine, d9(smem, regs, warps, blocks, tx, ctx, mem, comp, ovl), wv, out))
    return {"feasible": bool(out[0]), "score": out[1], "occupancy": out[2], "smem_warps": out[3],
            "reg_warps": out[4], "terms": list(out[5:12])}


def test_warp_sizes_and_warp_tile():
    # Section 4's example: tile (8,4,1), block (16,8,1) -> warp (16,2,1), warp tile (128,8,1)
    w, _ = otpw((16, 8, 1), 32, (8, 4, 1), (0, 0, 0))
    assert w == (16, 2, 1)
    assert tuple(t * x for t, x in zip((8, 4, 1), w)) == (128, 8, 1)
    # wave64: a 64x4 block makes 64-wide waves
    assert otpw((64, 4, 1), 64, (1, 1, 1), (0, 0, 0))[0] == (64, 1, 1)


def test_motivating_blur_scratchpad_and_occupancy_on_1080ti():
    """The blur of Section 3 on the GTX 1080Ti, block 64x4x1: the scratchpad of
    8 warps x (tile * 32 + 2) points (3-tap halo) is 8,256 B for tile 8 and
    16,448 B for tile 16; the second caps occupancy at 62.5%; keeping half of
    the 16-tile in registers (24 + 8 registers per thread) restores 100%."""
    _, e8 = otpw((64, 4, 1), 32, (8, 1, 1), (2, 0, 0))
    _, e16 = otpw((64, 4, 1), 32, (16, 1, 1), (2, 0, 0))
    assert e8 * 4 == 8256 and e16 * 4 == 16448
    assert alg2(1, 8256, 24, 8)["occupancy"] == 1.0
    r16 = alg2(1, 16448, 24, 8)
    assert r16["occupancy"] == pytest.approx(0.625) and r16["smem_warps"] == 40
    hybrid = alg2(1, 8 * (8 * 32 + 2) * 4, 32, 8)
    assert hybrid["occupancy"] == 1.0
    # redundant computation of the halo, from the scratchpad geometry: each of
    # the 8 warps holds tile*32 + 2 points for tile*32 outputs, 0.78% (tile 8)
    # and 0.39% (tile 16) of overlap
    assert round(100 * (e8 / (8 * 8 * 32) - 1), 2) == 0.78
    assert round(100 * (e16 / (8 * 16 * 32) - 1), 2) == 0.39


def test_alg2_terms_and_weights():
    w = [50, 0.5, 60, 10, 2, 100, 1]
    r = alg2(1, 16448, 24, 8, blocks=28 * 5 + 3, tx=3000, ctx=1500, ovl=0.0039, w=w)
    t = r["terms"]
    assert t[0] == pytest.approx(2.0)             # transactions / compulsory
    assert t[1] == pytest.approx(1 - 0.625)       # 1 - occupancy
    assert t[3] == pytest.approx(1 - 5 * 16448 / (96 * 1024))  # unallocated scratchpad
    assert t[5] == pytest.approx(0.0039)          # overlap
    assert t[6] == pytest.approx(1.0)             # ceil(143 / 28) = 6 blocks per SM, 6 mod 5 resident = 1
    assert r["score"] == pytest.approx(sum(a * b for a, b in zip(w, t)))
    # infeasible: more scratchpad than a block may take
    assert not alg2(1, 64 * 1024, 24, 8)["feasible"]


def test_gfx950_occupancy_rules():
    # VGPR allocation granule 8, 512 per lane per SIMD, at most 8 waves per SIMD, 4 SIMDs
    assert alg2(0, 0, 24, 1)["occupancy"] == 1.0          # 8 waves/SIMD
    assert alg2(0, 0, 128, 1)["occupancy"] == 0.5         # 4 waves/SIMD
    assert alg2(0, 0, 130, 1)["occupancy"] == 0.375       # 136 -> 3 waves/SIMD
    assert alg2(0, 64 * 1024, 24, 1)["occupancy"] == 2 / 32  # 160 KiB LDS: 2 workgroups
    assert not alg2(0, 200 * 1024, 24, 1)["feasible"]


def fusion_costs(spec, w, h, k=12):
    pipe = wt.from_spec(spec)
    dp, ex = ctypes.c_double(), ctypes.c_double()
    wt._check(lib.wt_fusion_costs(pipe._h, w, h, 0, k, ctypes.byref(dp), ctypes.byref(ex)))
    return dp.value, ex.value


@pytest.mark.parametrize("name", ["blur", "unsharp", "harris", "lapband", "dag3", "dag11", "dag21"])
def test_fusion_dp_equals_exhaustive(name):
    spec = {"blur": P.gaussian_blur, "unsharp": P.unsharp_mask, "harris": P.harris,
            "lapband": P.laplacian_band}.get(name)
    spec = spec() if spec else dags.random_dag(int(name[3:]), lo=6, hi=10)
    dp, ex = fusion_costs(spec, 512, 384)
    assert len(spec["stages"]) <= 10
    assert dp == pytest.approx(ex, rel=1e-12)
    dp4, ex4 = fusion_costs(spec, 512, 384, k=3)
    assert dp4 == pytest.approx(ex4, rel=1e-12) and dp4 >= dp - 1e-9


def test_analytic_fit_override_from_environment():
    """WT_ANALYTIC_FIT replaces the built-in calibration (nine numbers); a
    malformed value falls back to the built-in fit with a message."""
    import os
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, '.'); import paper_1909_07190_amd as wt; "
            "from synth import pipelines as P; "
            "print(wt.from_spec(P.unsharp_mask()).plan(2048, 2048, mode='analytic', no_device=True, "
            "no_compile=True).describe())")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

    def plan_text(fit):
        env = dict(os.environ)
        env.pop("WT_ANALYTIC_FIT", None)
        if fit is not None:
            env["WT_ANALYTIC_FIT"] = fit
        r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr
        return r.stdout.strip(), r.stderr

    base, _ = plan_text(None)
    # a huge weight on (1 - occupancy) versus one on the overlap fraction
    # lead to different configurations
    occ, _ = plan_text("0,1,0,50,0,0,0,0,0")
    ovl, _ = plan_text("0,1,0,0,0,0,0,50,0")
    assert occ != ovl
    bad, err = plan_text("1,2,3")
    assert bad == base and "WT_ANALYTIC_FIT" in err


def test_batch_hint_prefers_taller_tiles():
    """With many images per batched run the analytical cost no longer needs
    short tiles for parallelism: the pyramid's level-0 blur-and-decimate
    groups get taller tiles than when planned for one image."""
    import re
    import synth
    spec = P.pyramid_blend(4)
    sizes = synth.batch_sizes(4, 64)
    mw, mh = sorted(sizes, key=lambda s: s[0] * s[1])[len(sizes) // 2]

    def ty(batch):
        d = wt.from_spec(spec).plan(mw, mh, mode="analytic", any_width=True, no_device=True, no_compile=True,
                                    batch_images=batch).describe()
        line = next(l for l in d.splitlines() if " nodes=3,4 " in l or " nodes=3,4," in l)
        return int(re.search(r"TY=(\d+)", line).group(1))

    assert ty(64) > ty(1)
