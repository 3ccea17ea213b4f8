"""CPU tests of the C ABI: exported symbols, argument checking, schedule
text, and that generated kernels compile for gfx950 (no GPU needed: plans
made with WT_PLAN_NO_DEVICE generate and compile code but run nothing)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1909_07190_amd as wt
from synth import pipelines as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "wt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wt_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(wt.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_constants_match_header():
    """The binding's WT_PLAN_* flag bits and the sizes of its option struct
    follow include/wt.h."""
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "wt.h")).read(), flags=re.S)
    flags = {k: int(v) for k, v in re.findall(r"\bWT_PLAN_([A-Z_]+)\s*=\s*(\d+)", text)}
    assert flags == {"NO_DEVICE": 1, "ANY_WIDTH": 2, "NO_COMPILE": 4, "RETUNE": 8, "BATCH_RESIDENT": 16,
                     "NO_FOLD": 32, "BATCH_WHOLE": 64}
    for k, v in flags.items():
        assert getattr(wt, "PLAN_" + k) == v, k
    body = re.search(r"typedef struct \{([^}]*)\} wt_sched_opts;", text).group(1)
    fields = re.findall(r"\b([a-z_0-9]+);", body)
    assert fields == [f for f, _ in wt.WtSchedOpts._fields_]


def test_builder_rejects_bad_arguments():
    p = wt.Pipeline()
    img = p.input(3)
    with pytest.raises(wt.WtError):
        p.stencil(img, 0, 3, 0, 0, [])
    with pytest.raises(wt.WtError):
        p.stencil(img, 3, 1, 3, 0, [1, 1, 1])          # anchor outside kernel
    with pytest.raises(wt.WtError):
        p.stencil(99, 3, 1, 1, 0, [1, 1, 1])           # unknown source
    with pytest.raises(wt.WtError):
        p.pointwise([img], "s0 +", 3)                   # syntax
    with pytest.raises(wt.WtError):
        p.pointwise([img], "s1", 3)                     # source index
    with pytest.raises(wt.WtError):
        p.pointwise([img], "s0[3]", 1)                  # channel subscript
    with pytest.raises(wt.WtError):
        p.pointwise([img], "s0 < 1", 3)                 # bare comparison
    with pytest.raises(wt.WtError):
        p.pointwise([img], "s0", 2)                     # 3 channels into 2
    with pytest.raises(wt.WtError):
        p.resample(img, wt.UP2)                         # up2 at level 0
    with pytest.raises(wt.WtError):
        p.output(img)                                   # inputs are not outputs
    ok = p.pointwise([img], "select(abs(s0[0] - 0.5) <= 0.25, -s0[1], min(s0[2], 2) / 4)", 1)
    p.output(ok)
    with pytest.raises(wt.WtError):
        p.output(ok)


def _status(fn, *a):
    try:
        fn(*a)
    except wt.WtError as e:
        return e.status
    return 0


def test_integer_builder_rules():
    p = wt.Pipeline()
    f = p.input(1)
    u8 = p.input(1, "u8")
    i32 = p.input(1, "i32")
    UNSUP = -2
    # integer stencils read integer stages only
    assert _status(p.stencil_int, f, 3, 1, 1, 0, [1, 2, 1], 4, "u8") == UNSUP
    # sums that may leave 32 bits are refused
    assert _status(p.stencil_int, i32, 3, 1, 1, 0, [1, 2, 1], 4, "i32") == UNSUP
    assert _status(p.stencil_int, u8, 3, 1, 1, 0, [1, 2, 1], 0, "u8") == -1      # divisor
    assert _status(p.stencil_int, u8, 3, 1, 1, 0, [1, 40000, 1], 1, "u8") == -1  # weight range
    assert _status(p.stencil_int, u8, 3, 1, 1, 0, [1, 2, 1], 4, "f32") == -1     # output type
    # integer expressions: integer constants, no division
    assert _status(p.pointwise, [u8], "s0 / 2", 1, "i16") == UNSUP
    assert _status(p.pointwise, [u8], "s0 + 0.5", 1, "i16") == UNSUP
    assert _status(p.pointwise, [u8, f], "s0 + s1", 1, "i16") == UNSUP
    assert _status(p.pointwise, [i32, i32], "s0 * s1", 1, "i32") == UNSUP       # 32-bit bound
    b = p.stencil_int(u8, 5, 1, 2, 0, [1, 4, 6, 4, 1], 16, "u8")
    d = p.resample(b, wt.DOWN2)
    assert _status(p.resample, d, wt.UP2) == UNSUP                              # no integer up2
    # float stages may read integer stages
    p.stencil(b, 3, 1, 1, 0, [1, 2, 1], 0.25)
    p.pointwise([u8, f], "s0 * s1 + 0.5", 1)
    ok = p.pointwise([u8, b], "max(s0 - 2 * s1, -7)", 1, "i16")
    p.output(ok)


def test_plan_errors():
    pipe = wt.from_spec(P.gaussian_blur())
    with pytest.raises(wt.WtError):
        pipe.plan(0, 10, no_device=True)
    with pytest.raises(wt.WtError):
        pipe.plan(64, 64, mode="fixed", fixed="nodes=1 V=4", no_device=True)       # misses node 2
    with pytest.raises(wt.WtError):
        pipe.plan(64, 64, mode="fixed", fixed="nodes=2;nodes=1", no_device=True)   # order
    with pytest.raises(wt.WtError):
        pipe.plan(64, 64, mode="fixed", fixed="nodes=1,2 V=3", no_device=True)     # bad V
    with pytest.raises(wt.WtError):
        pipe.plan(64, 64, mode="fixed", fixed="nodes=1,2 bogus=1", no_device=True)
    plan = pipe.plan(64, 64, mode="fixed", fixed="g0 nodes=1,2 V=2 TX=3 SX=1 TY=9 PF=1",
                     no_device=True)
    text = plan.describe()
    assert "V=2 TX=3 SX=1 TY=9" in text
    with pytest.raises(wt.WtError):
        plan.run([], [], stream=0)                      # no-device plans never run


def _compile(spec, fixed, fp16=False, w=512, h=256):
    plan = wt.from_spec(spec).plan(w, h, mode="fixed", fixed=fixed, fp16=fp16, no_device=True)
    src = plan.source(0)
    assert "wt_g0" in src
    return plan


def test_generated_kernels_compile_for_gfx950():
    from test_gpu_parity import BLUR_CASES, UM_CASES
    for fixed, w, h in BLUR_CASES:
        _compile(P.gaussian_blur(), fixed, w=w, h=h)
    for fixed, fp16 in UM_CASES:
        _compile(P.unsharp_mask(), fixed, fp16=fp16)


def test_load_types_in_generated_source():
    """The four producer-load types appear as the expected primitives: own
    registers, LDS reads from the LDS sub-tiles, DPP shifts inside a register
    sub-tile, and DPP shift-with-fill from the neighbouring sub-tile."""
    plan = _compile(P.gaussian_blur(), "nodes=1,2 V=1 TX=3 SX=1 TY=4 PF=0 align=1")
    src = plan.source(0)
    body = src[src.index("extern \"C\""):]
    assert "wt_shift1(" in body            # types 3 + 4 (register sub-tiles)
    assert "wt_shr1(" in body              # type 3 + 2 (lane 0 from LDS)
    assert "(float)L0[" in body            # type 2
    assert "ds_bpermute" not in body or "wt_shiftd" in body


def test_preprofiling_microbenchmarks_compile_for_gfx950():
    """Without a device, pre-profiling compiles every stage's microbenchmark
    and unfused kernel and the cost model keeps its static estimate."""
    for spec in (P.unsharp_mask(), P.integer_gradient()):
        pipe = wt.from_spec(spec)
        nin = len(spec["inputs"])
        for k, st in enumerate(spec["stages"]):
            if st["kind"] in ("stencil", "pointwise"):
                ns, vg, measured = wt.stage_profile(pipe, nin + k, 128, 64, measure=False)
                assert ns > 0 and vg >= 2 and not measured


def test_stream_copy_argument_checks():
    """The copy reference rejects null, misaligned and overlapping ranges
    before touching the device (host-side checks only)."""
    import ctypes
    lib = wt.lib
    assert lib.wt_stream_copy(None, None, 0, None) == 0  # nothing to copy
    assert lib.wt_stream_copy(None, ctypes.c_void_p(4096), 64, None) == -1
    assert lib.wt_stream_copy(ctypes.c_void_p(4100), ctypes.c_void_p(8192), 64, None) == -1  # misaligned
    assert lib.wt_stream_copy(ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 32), 64, None) == -1  # overlap
    assert "overlap" in lib.wt_last_error().decode()


def test_histogram_builder_and_plan_rules():
    """wt_histogram checks its arguments; no stage may read a histogram; a
    histogram must be an output; the lone and the fused histogram kernels
    compile for gfx950."""
    p = wt.Pipeline()
    img = p.input(1)
    for bins, lo, hi in ((0, 0.0, 1.0), (4097, 0.0, 1.0), (8, 1.0, 1.0), (8, 0.0, float("nan"))):
        with pytest.raises(wt.WtError):
            p.histogram(img, bins, lo, hi)
    h = p.histogram(img, 16, 0.0, 1.0)
    with pytest.raises(wt.WtError):
        p.resample(h, wt.DOWN2)
    with pytest.raises(wt.WtError):
        p.stencil(h, 3, 1, 1, 0, [1.0, 2.0, 1.0], 0.25)
    b = p.stencil(img, 3, 1, 1, 0, [1.0, 2.0, 1.0], 0.25)
    p.histogram(b, 8, 0.0, 1.0)   # never marked as an output
    p.output(b)
    with pytest.raises(wt.WtError, match="not an output"):
        p.plan(64, 64, mode="unfused", no_device=True, no_compile=True)
    spec = P.blur_histogram(channels=3, bins=256)
    wt.from_spec(spec).plan(512, 256, mode="unfused", no_device=True)
    for fixed in ("nodes=1,2 V=4 TX=1 SX=0 TY=16 PF=2 hst=3", "nodes=1,2 V=1 TX=2 SX=1 TY=8 PF=1 WPB=2 hst=3"):
        assert "wt_count_global" in _compile(spec, fixed).source(0)


def test_equalize_builder_rules():
    """wt_equalize needs a histogram with the source's channel count; a
    histogram read by an equalize stage need not be an output (the plan
    keeps its counts in an intermediate buffer)."""
    p = wt.Pipeline()
    img = p.input(2)
    one = p.input(1)
    b = p.stencil(img, 3, 1, 1, 0, [1.0, 2.0, 1.0], 0.25)
    with pytest.raises(wt.WtError):
        p.equalize(b, b)                  # not a histogram
    h1 = p.histogram(one, 16, 0.0, 1.0)
    with pytest.raises(wt.WtError):
        p.equalize(b, h1)                 # 2 channels against 1
    h = p.histogram(b, 16, 0.0, 1.0)
    e = p.equalize(b, h)
    p.output(e)
    p.output(h1)
    plan = p.plan(128, 64, mode="analytic", no_device=True)
    assert "hst=" in plan.describe()


def test_whole_pipeline_source_and_refusals():
    """The whole-pipeline kernel (group -1 of wt_plan_source) holds one tile
    function per group and one persistent kernel; plans with a lone
    resampling or histogram group or a one-tile-per-workgroup group are
    refused with WT_E_UNSUPPORTED."""
    spec = P.pyramid_blend(3)
    pl = wt.from_spec(spec).plan(300, 200, mode="analytic", any_width=True, no_compile=True, batch_images=4)
    src = pl.source(-1)
    for g in range(pl.num_groups):
        assert f"_g{g}(const WtArgs& A, const int wid, const int lane, char* lds)" in src
    assert src.count("__global__") == 1 and "_wait(P, dm, img)" in src
    refused = [
        (P.pyramid_blend(3), dict(mode="unfused", any_width=True)),          # lone down2 / up2 groups
        (P.blur_histogram(), dict(mode="unfused")),                          # lone histogram group
        (P.unsharp_mask(channels=1), dict(mode="fixed", fixed="nodes=1,2,3,4 V=1 TX=1 TY=8 WPB=4 BLK=1")),
    ]
    for sp, kw in refused:
        p2 = wt.from_spec(sp).plan(300, 200, no_compile=True, **kw)
        with pytest.raises(wt.WtError) as e:
            p2.source(-1)
        assert e.value.status == -2
        with pytest.raises(wt.WtError) as e:
            p2.whole_tables([(300, 200)], 64)
        assert e.value.status == -2
    with pytest.raises(wt.WtError) as e:
        pl.source(-2)
    assert e.value.status == -1
    # the launch's host tables: every tile of every group and image in exactly
    # one chunk, group by group; chunk sizes follow the resident waves
    sizes = [(300, 200), (64, 40), (517, 129), (1, 1)]
    small, deps = pl.whole_tables(sizes, 10 ** 6)
    assert set(small[:, 3].tolist()) == {1} and np.all(np.diff(small[:, 0]) >= 0)
    assert deps[0] == 0 and all(d < (1 << g) for g, d in enumerate(deps)) and any(deps)
    big, deps2 = pl.whole_tables(sizes, 1)
    assert deps2 == deps and len(big) < len(small)
    for g in range(pl.num_groups):
        assert small[small[:, 0] == g].shape[0] == big[big[:, 0] == g][:, 3].sum()
    with pytest.raises(wt.WtError) as e:
        pl.whole_tables([(0, 5)], 64)
    assert e.value.status == -3


def test_whole_pipeline_kernel_compiles_for_gfx950():
    """The whole-pipeline kernel of a three-level pyramid blend compiles for
    gfx950 with the library's own run-time compile options (no device)."""
    rtc = ctypes.CDLL("/opt/rocm/lib/libhiprtc.so")
    pl = wt.from_spec(P.pyramid_blend(3)).plan(300, 200, mode="analytic", any_width=True, no_compile=True,
                                               batch_images=4)
    src = pl.source(-1).encode()
    prog = ctypes.c_void_p()
    assert rtc.hiprtcCreateProgram(ctypes.byref(prog), src, b"whole.hip", 0, None, None) == 0
    opts = [b"--offload-arch=gfx950", b"-O3", b"-std=c++17", b"-Xclang", b"-target-feature", b"-Xclang",
            b"-packed-fp32-ops"]
    rc = rtc.hiprtcCompileProgram(prog, len(opts), (ctypes.c_char_p * len(opts))(*opts))
    n = ctypes.c_size_t()
    rtc.hiprtcGetProgramLogSize(prog, ctypes.byref(n))
    log = ctypes.create_string_buffer(max(1, n.value))
    rtc.hiprtcGetProgramLog(prog, log)
    code = ctypes.c_size_t()
    rtc.hiprtcGetCodeSize(prog, ctypes.byref(code))
    rtc.hiprtcDestroyProgram(ctypes.byref(prog))
    assert rc == 0, log.value.decode(errors="replace")[:2000]
    assert code.value > 0
