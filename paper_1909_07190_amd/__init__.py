"""wavetile: fused wave-tiled stencil pipelines on MI355X (gfx950).

Thin ctypes binding over the C ABI in ``include/wt.h``: argument marshalling
only.  Every step of a pipeline runs in the library's generated HIP kernels;
there is no Python or CPU fallback, and importing this package fails loudly
when ``libwavetile.so`` has not been built.  PyTorch supplies device memory
and streams.
"""
from __future__ import annotations

import ctypes
import sys
import os

__all__ = ["Pipeline", "Plan", "WtError", "lib", "SCHED", "from_spec", "LIB_PATH"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwavetile.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: run `python paper_1909_07190_amd/build.py` "
                      "(or __graft_entry__.build()) first")
# One HIP runtime per process: torch ships its own libamdhip64 / libhiprtc
# under the same sonames as the system ROCm's.  Loading torch first makes the
# library bind to those, so its kernels, modules and streams live in the same
# runtime as the tensors it is handed (loaded the other way round, torch would
# then find no device).
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

SCHED = {"unfused": 0, "analytic": 1, "mlp": 2, "autotune": 3, "fixed": 4}
DOWN2, UP2 = 0, 1
F32, F16, U8, U16, I16, I32 = 0, 1, 2, 3, 4, 5
# plain-data names of the element types
DTYPES = {"f32": F32, "u8": U8, "u16": U16, "i16": I16, "i32": I32}
PLAN_NO_DEVICE = 1
PLAN_ANY_WIDTH = 2
PLAN_NO_COMPILE = 4
PLAN_RETUNE = 8
PLAN_BATCH_RESIDENT = 16
PLAN_NO_FOLD = 32
PLAN_BATCH_WHOLE = 64

_c_int_p = ctypes.POINTER(ctypes.c_int)


class WtImage(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("row_stride", ctypes.c_int64), ("chan_stride", ctypes.c_int64)]


class WtSchedOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("fp16_intermediates", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("autotune_topk", ctypes.c_int32),
                ("fixed_schedule", ctypes.c_char_p), ("model_path", ctypes.c_char_p),
                ("cache_dir", ctypes.c_char_p), ("batch_images", ctypes.c_int32)]


class GroupInfo(ctypes.Structure):
    """wt_group_info: a group's launch shape and buffers."""
    _fields_ = [(n, ctypes.c_int32) for n in
                ("resample", "waves_per_group", "nwaves", "tiles_x", "tiles_y", "width", "height",
                 "src_width", "src_height", "channels", "nloaded", "nliveouts")] + \
               [("loaded", ctypes.c_int32 * 16), ("liveouts", ctypes.c_int32 * 16),
                ("loaded_half", ctypes.c_int32 * 16), ("liveout_half", ctypes.c_int32 * 16),
                ("loaded_dtype", ctypes.c_int32 * 16), ("liveout_dtype", ctypes.c_int32 * 16)]


def _sig(name, restype, *args):
    f = getattr(lib, name)
    f.restype = restype
    f.argtypes = list(args)
    return f


_sig("wt_last_error", ctypes.c_char_p)
_sig("wt_pipeline_create", ctypes.c_int, ctypes.POINTER(ctypes.c_void_p))
_sig("wt_pipeline_destroy", None, ctypes.c_void_p)
_sig("wt_input", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, _c_int_p)
_sig("wt_input_bound", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_double)
_sig("wt_input_typed", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int_p)
_sig("wt_stencil_int", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_int, _c_int_p)
_sig("wt_pointwise_typed", ctypes.c_int, ctypes.c_void_p, _c_int_p, ctypes.c_int, ctypes.c_char_p,
     ctypes.c_int, ctypes.c_int, _c_int_p)
_sig("wt_stencil", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_double, _c_int_p)
_sig("wt_pointwise", ctypes.c_int, ctypes.c_void_p, _c_int_p, ctypes.c_int, ctypes.c_char_p,
     ctypes.c_int, _c_int_p)
_sig("wt_resample", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int_p)
_sig("wt_histogram", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
     _c_int_p)
_sig("wt_equalize", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int_p)
_sig("wt_output", ctypes.c_int, ctypes.c_void_p, ctypes.c_int)
_sig("wt_plan_create", ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(WtSchedOpts), ctypes.c_int,
     ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p))
_sig("wt_plan_run", ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(WtImage), ctypes.c_int,
     ctypes.POINTER(WtImage), ctypes.c_int, ctypes.c_void_p)
_sig("wt_plan_run_batch", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(WtImage),
     ctypes.POINTER(WtImage), ctypes.c_void_p)
_sig("wt_plan_run_batch_static", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(WtImage),
     ctypes.POINTER(WtImage), ctypes.c_void_p)
_sig("wt_plan_batch_check", ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p)
_sig("wt_plan_whole_tables", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
     ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_uint64))
_sig("wt_plan_tune_batch", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(WtImage),
     ctypes.POINTER(WtImage), ctypes.c_void_p)
_sig("wt_plan_run_batch_groups", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     ctypes.POINTER(WtImage), ctypes.POINTER(WtImage), ctypes.c_void_p)
_sig("wt_stream_copy", ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_sig("wt_plan_describe", ctypes.c_int, ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t,
     ctypes.POINTER(ctypes.c_size_t))
_sig("wt_plan_source", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t,
     ctypes.POINTER(ctypes.c_size_t))
_sig("wt_plan_num_groups", ctypes.c_int, ctypes.c_void_p)
_sig("wt_plan_group_info", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(GroupInfo))
_sig("wt_plan_destroy", None, ctypes.c_void_p)


class WtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"wavetile error {status}: {msg}")
        self.status = status


def _check(st):
    if st != 0:
        raise WtError(st, lib.wt_last_error().decode(errors="replace"))


class Pipeline:
    """Builder for a pipeline DAG; node ids are returned by each call."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib.wt_pipeline_create(ctypes.byref(h)))
        self._h = h
        self.names: dict[str, int] = {}
        self.channels: dict[int, int] = {}

    def __del__(self, _finalizing=sys.is_finalizing, _destroy=lib.wt_pipeline_destroy):
        # at interpreter exit the module's globals may already be gone and
        # the process is about to release everything anyway
        if getattr(self, "_h", None) and not _finalizing():
            _destroy(self._h)
            self._h = None

    def input(self, channels: int, dtype: str = "f32") -> int:
        i = ctypes.c_int()
        _check(lib.wt_input_typed(self._h, channels, DTYPES[dtype], ctypes.byref(i)))
        self.channels[i.value] = channels
        return i.value

    def input_bound(self, node: int, max_abs: float):
        """Declares |value| <= max_abs for a float input (default 1); stages
        whose propagated bound exceeds FP16's range keep FP32 storage."""
        _check(lib.wt_input_bound(self._h, node, float(max_abs)))

    def stencil_int(self, src, kw, kh, ax, ay, weights, divisor, dtype) -> int:
        w = (ctypes.c_int32 * (kw * kh))(*[int(v) for v in weights])
        i = ctypes.c_int()
        _check(lib.wt_stencil_int(self._h, src, kw, kh, ax, ay, w, int(divisor), DTYPES[dtype],
                                  ctypes.byref(i)))
        self.channels[i.value] = self.channels[src]
        return i.value

    def stencil(self, src, kw, kh, ax, ay, weights, scale=1.0) -> int:
        w = (ctypes.c_double * (kw * kh))(*[float(v) for v in weights])
        i = ctypes.c_int()
        _check(lib.wt_stencil(self._h, src, kw, kh, ax, ay, w, float(scale), ctypes.byref(i)))
        self.channels[i.value] = self.channels[src]
        return i.value

    def pointwise(self, srcs, expr: str, channels: int, dtype: str = "f32") -> int:
        arr = (ctypes.c_int * len(srcs))(*srcs)
        i = ctypes.c_int()
        _check(lib.wt_pointwise_typed(self._h, arr, len(srcs), expr.encode(), channels, DTYPES[dtype],
                                      ctypes.byref(i)))
        self.channels[i.value] = channels
        return i.value

    def resample(self, src, kind) -> int:
        i = ctypes.c_int()
        _check(lib.wt_resample(self._h, src, kind, ctypes.byref(i)))
        self.channels[i.value] = self.channels[src]
        return i.value

    def histogram(self, src, bins, lo, hi) -> int:
        i = ctypes.c_int()
        _check(lib.wt_histogram(self._h, src, bins, float(lo), float(hi), ctypes.byref(i)))
        self.channels[i.value] = self.channels[src]
        return i.value

    def equalize(self, src, hist) -> int:
        i = ctypes.c_int()
        _check(lib.wt_equalize(self._h, src, hist, ctypes.byref(i)))
        self.channels[i.value] = self.channels[src]
        return i.value

    def output(self, node: int):
        _check(lib.wt_output(self._h, node))

    def plan(self, width, height, mode="analytic", fp16=False, fixed=None,
             no_device=False, model_path=None, cache_dir=None, autotune_topk=0,
             any_width=False, no_compile=False, retune=False, batch_images=1,
             batch_resident=False, no_fold=False, batch_whole=False) -> "Plan":
        """Schedules and compiles the pipeline for width x height.  mode
        "mlp" without a model_path uses the network trained on gfx950
        measurements that ships with the package (GFX950_COST_MODEL).  Mode
        "autotune" reuses a cached result for the same pipeline, device and
        size bucket unless `retune`.  `batch_images`: how many images of about
        this size run_batch will process together (the analytical cost then
        counts their waves and traffic; "autotune" times its candidates on an
        image as tall as up to that many).  `batch_resident`: run_batch
        launches only the workgroups resident at once, each looping over its
        share of the tiles, instead of one workgroup per work unit.
        `no_fold`: the fusion search never folds an up2 into the group of
        the stage whose decimation it expands.  `batch_whole`: run_batch
        runs every group in one persistent launch (wave-tiled fused groups
        only), ordered by device-side completion counters."""
        if mode == "mlp" and model_path is None:
            model_path = GFX950_COST_MODEL
        return Plan(self, width, height, mode, fp16, fixed, no_device, model_path, cache_dir,
                    autotune_topk, any_width, no_compile, retune, batch_images, batch_resident, no_fold,
                    batch_whole)


def stream_copy(src, dst, stream=None):
    """Copies device tensor `src` into `dst` (same byte size, contiguous)
    with the library's streaming copy kernel, the achievable-bandwidth
    reference, on `stream` (default: torch's current stream)."""
    import torch
    nbytes = src.numel() * src.element_size()
    if not (src.is_contiguous() and dst.is_contiguous()) or dst.numel() * dst.element_size() != nbytes:
        raise ValueError("stream_copy needs contiguous tensors of equal byte size")
    if stream is None:
        stream = torch.cuda.current_stream()
    s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib.wt_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                              ctypes.c_void_p(s)))


# The cost network trained on gfx950: 4444 timed candidate groups of 93
# random pipelines (learn.py train); its ranking report on the held-out
# pipelines is gfx950_cost_mlp_report.json beside it.
GFX950_COST_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gfx950_cost_mlp.txt")


def from_spec(spec: dict) -> Pipeline:
    """Builds a Pipeline from a plain-data description (see synth.pipelines)."""
    p = Pipeline()
    for inp in spec["inputs"]:
        p.names[inp["name"]] = p.input(inp["channels"], inp.get("dtype", "f32"))
        if "bound" in inp:
            p.input_bound(p.names[inp["name"]], inp["bound"])
    for st in spec["stages"]:
        k = st["kind"]
        dt = st.get("dtype", "f32")
        if k == "stencil" and dt != "f32":
            i = p.stencil_int(p.names[st["src"]], st["kw"], st["kh"], st["ax"], st["ay"],
                              st["weights"], st.get("divisor", 1), dt)
        elif k == "stencil":
            i = p.stencil(p.names[st["src"]], st["kw"], st["kh"], st["ax"], st["ay"],
                          st["weights"], st["scale"])
        elif k == "pointwise":
            i = p.pointwise([p.names[s] for s in st["srcs"]], st["expr"], st["channels"], dt)
        elif k in ("down2", "up2"):
            i = p.resample(p.names[st["src"]], DOWN2 if k == "down2" else UP2)
        elif k == "hist":
            i = p.histogram(p.names[st["src"]], st["bins"], st["lo"], st["hi"])
        elif k == "equalize":
            i = p.equalize(p.names[st["src"]], p.names[st["hist"]])
        else:
            raise ValueError(f"unknown stage kind {k!r}")
        p.names[st["name"]] = i
    for o in spec["outputs"]:
        p.output(p.names[o])
    return p


def _image(t) -> WtImage:
    import torch
    if not t.is_cuda:
        raise ValueError("images must be device tensors")
    tmap = {torch.float32: F32, torch.uint8: U8, torch.uint16: U16, torch.int16: I16, torch.int32: I32}
    if t.dtype not in tmap:
        raise ValueError(f"unsupported image dtype {t.dtype}")
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3 or t.stride(2) != 1:
        raise ValueError("images must be [C, H, W] with unit column stride")
    c, h, w = t.shape
    return WtImage(t.data_ptr(), w, h, c, tmap[t.dtype], t.stride(1), t.stride(0))


class Plan:
    """A compiled schedule for one image size."""

    def __init__(self, pipe: Pipeline, width, height, mode, fp16, fixed, no_device,
                 model_path, cache_dir, autotune_topk, any_width=False, no_compile=False, retune=False,
                 batch_images=1, batch_resident=False, no_fold=False, batch_whole=False):
        self.pipe = pipe  # keeps the pipeline alive
        flags = ((PLAN_NO_DEVICE if no_device else 0) | (PLAN_ANY_WIDTH if any_width else 0)
                 | (PLAN_NO_COMPILE if no_compile else 0) | (PLAN_RETUNE if retune else 0)
                 | (PLAN_BATCH_RESIDENT if batch_resident else 0) | (PLAN_NO_FOLD if no_fold else 0)
                 | (PLAN_BATCH_WHOLE if batch_whole else 0))
        opts = WtSchedOpts(SCHED[mode], int(bool(fp16)), flags,
                           autotune_topk, fixed.encode() if fixed else None,
                           model_path.encode() if model_path else None,
                           cache_dir.encode() if cache_dir else None, int(batch_images))
        h = ctypes.c_void_p()
        s = None
        if not (no_device or no_compile):
            import torch
            s = torch.cuda.current_stream().cuda_stream
        _check(lib.wt_plan_create(pipe._h, ctypes.byref(opts), width, height, ctypes.c_void_p(s), ctypes.byref(h)))
        self._h = h
        self.width, self.height = width, height

    def __del__(self, _finalizing=sys.is_finalizing, _destroy=lib.wt_plan_destroy):
        # at interpreter exit the module's globals may already be gone and
        # the process is about to release everything anyway
        if getattr(self, "_h", None) and not _finalizing():
            _destroy(self._h)
            self._h = None

    def run(self, inputs, outputs, stream=None):
        """Launches the plan on `stream` (default: torch's current stream)."""
        import torch
        ins = (WtImage * max(1, len(inputs)))(*[_image(t) for t in inputs])
        outs = (WtImage * max(1, len(outputs)))(*[_image(t) for t in outputs])
        if stream is None:
            stream = torch.cuda.current_stream()
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(lib.wt_plan_run(self._h, ins, len(inputs), outs, len(outputs), ctypes.c_void_p(s)))

    def run_batch(self, inputs, outputs, stream=None):
        """Runs a batch: inputs[i] / outputs[i] are the tensors of image i."""
        import torch
        ins = [_image(t) for img in inputs for t in img]
        outs = [_image(t) for img in outputs for t in img]
        a_in = (WtImage * len(ins))(*ins)
        a_out = (WtImage * len(outs))(*outs)
        if stream is None:
            stream = torch.cuda.current_stream()
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(lib.wt_plan_run_batch(self._h, len(inputs), a_in, a_out, ctypes.c_void_p(s)))

    def run_batch_static(self, inputs, outputs, stream=None):
        """run_batch with the intermediates in the library's fixed device
        workspace: allocates no device memory (the plan's batched kernels
        must be loaded: plan with batch_images > 1)."""
        import torch
        ins = [_image(t) for img in inputs for t in img]
        outs = [_image(t) for img in outputs for t in img]
        a_in = (WtImage * len(ins))(*ins)
        a_out = (WtImage * len(outs))(*outs)
        if stream is None:
            stream = torch.cuda.current_stream()
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(lib.wt_plan_run_batch_static(self._h, len(inputs), a_in, a_out, ctypes.c_void_p(s)))

    def whole_tables(self, sizes, resident_waves):
        """The whole-pipeline launch's chunk table (rows: group, image, first
        tile, tiles) and per-group producer masks for a batch of (width,
        height) `sizes` with `resident_waves` waves resident."""
        import numpy as np
        wh = (ctypes.c_int * (2 * len(sizes)))(*[v for s in sizes for v in s])
        n = ctypes.c_int()
        deps = (ctypes.c_uint64 * max(1, self.num_groups))()
        _check(lib.wt_plan_whole_tables(self._h, len(sizes), wh, resident_waves, None, 0, ctypes.byref(n), deps))
        tab = np.zeros((n.value, 4), dtype=np.int32)
        _check(lib.wt_plan_whole_tables(self._h, len(sizes), wh, resident_waves,
                                        tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), n.value, ctypes.byref(n),
                                        deps))
        return tab, [int(d) for d in deps[:self.num_groups]]

    def batch_check(self, stream=None):
        """Synchronises `stream` and raises if the last whole-pipeline batch
        launch gave up waiting for a producer group."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(lib.wt_plan_batch_check(self._h, ctypes.c_void_p(s)))

    def tune_batch(self, inputs, outputs, stream=None):
        """Tunes every group's configuration on this batch itself (batched
        kernels over these images) and rebuilds the plan; outputs then hold
        the batch's result."""
        import torch
        ins = [_image(t) for img in inputs for t in img]
        outs = [_image(t) for img in outputs for t in img]
        a_in = (WtImage * len(ins))(*ins)
        a_out = (WtImage * len(outs))(*outs)
        if stream is None:
            stream = torch.cuda.current_stream()
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(lib.wt_plan_tune_batch(self._h, len(inputs), a_in, a_out, ctypes.c_void_p(s)))

    def run_batch_groups(self, first, count, inputs, outputs, stream=None):
        """Launches groups first .. first+count-1 of a batched run directly
        (after a complete run_batch of the same shape)."""
        import torch
        ins = [_image(t) for img in inputs for t in img]
        outs = [_image(t) for img in outputs for t in img]
        a_in = (WtImage * len(ins))(*ins)
        a_out = (WtImage * len(outs))(*outs)
        if stream is None:
            stream = torch.cuda.current_stream()
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(lib.wt_plan_run_batch_groups(self._h, first, count, len(inputs), a_in, a_out, ctypes.c_void_p(s)))

    def describe(self) -> str:
        n = ctypes.c_size_t()
        _check(lib.wt_plan_describe(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib.wt_plan_describe(self._h, buf, n.value, None))
        return buf.value.decode()

    def source(self, group: int) -> str:
        n = ctypes.c_size_t()
        _check(lib.wt_plan_source(self._h, group, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib.wt_plan_source(self._h, group, buf, n.value, None))
        return buf.value.decode()

    @property
    def num_groups(self) -> int:
        return lib.wt_plan_num_groups(self._h)


# ---------------------------------------------------------------------------
# Learned cost model
# ---------------------------------------------------------------------------
_f_p = ctypes.POINTER(ctypes.c_float)
_sig("wt_mlp_create", ctypes.c_int, _c_int_p, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p))
_sig("wt_mlp_destroy", None, ctypes.c_void_p)
_sig("wt_mlp_num_params", ctypes.c_size_t, ctypes.c_void_p)
_sig("wt_mlp_get_params", ctypes.c_int, ctypes.c_void_p, _f_p, ctypes.c_size_t)
_sig("wt_mlp_set_params", ctypes.c_int, ctypes.c_void_p, _f_p, ctypes.c_size_t)
_sig("wt_mlp_forward", ctypes.c_int, ctypes.c_void_p, _f_p, ctypes.c_int, _f_p)
_sig("wt_mlp_forward_backward", ctypes.c_int, ctypes.c_void_p, _f_p, _f_p, ctypes.c_int, _f_p, _f_p)
_sig("wt_mlp_adam_step", ctypes.c_int, ctypes.c_void_p, _f_p, ctypes.c_float)
_sig("wt_mlp_train", ctypes.c_int, ctypes.c_void_p, _f_p, _f_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     ctypes.c_float, ctypes.c_uint64, _f_p)
_sig("wt_model_train", ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_void_p)
_sig("wt_model_rows", ctypes.c_int, ctypes.c_char_p, _c_int_p)
_sig("wt_mlp_predict", ctypes.c_int, ctypes.c_void_p, _f_p, ctypes.c_int, _f_p)
_sig("wt_mlp_save", ctypes.c_int, ctypes.c_void_p, ctypes.c_char_p)
_sig("wt_mlp_load", ctypes.c_int, ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p))
_sig("wt_group_features", ctypes.c_int, ctypes.c_void_p, _c_int_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     ctypes.c_int, _f_p, ctypes.c_int, _c_int_p, ctypes.c_char_p, ctypes.c_size_t)

NUM_FEATURES = 40


def _fbuf(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_f_p)


class Mlp:
    """The learned cost model (device training through the C ABI)."""

    def __init__(self, dims=(NUM_FEATURES, 128, 128, 128, 1), seed=1, _handle=None):
        if _handle is not None:
            self._h = _handle
        else:
            d = (ctypes.c_int * len(dims))(*dims)
            h = ctypes.c_void_p()
            _check(lib.wt_mlp_create(d, len(dims), seed, ctypes.byref(h)))
            self._h = h
        self.dims = tuple(dims)

    def __del__(self, _finalizing=sys.is_finalizing, _destroy=lib.wt_mlp_destroy):
        # at interpreter exit the module's globals may already be gone and
        # the process is about to release everything anyway
        if getattr(self, "_h", None) and not _finalizing():
            _destroy(self._h)
            self._h = None

    @property
    def num_params(self):
        return lib.wt_mlp_num_params(self._h)

    def params(self):
        import numpy as np
        out = np.empty(self.num_params, np.float32)
        _check(lib.wt_mlp_get_params(self._h, out.ctypes.data_as(_f_p), out.size))
        return out

    def set_params(self, p):
        a, ptr = _fbuf(p)
        _check(lib.wt_mlp_set_params(self._h, ptr, a.size))

    def forward(self, x):
        import numpy as np
        a, ptr = _fbuf(x)
        y = np.empty((a.shape[0], self.dims[-1]), np.float32)
        _check(lib.wt_mlp_forward(self._h, ptr, a.shape[0], y.ctypes.data_as(_f_p)))
        return y

    def forward_backward(self, x, t):
        import numpy as np
        a, px = _fbuf(x)
        b, pt = _fbuf(t)
        g = np.empty(self.num_params, np.float32)
        loss = ctypes.c_float()
        _check(lib.wt_mlp_forward_backward(self._h, px, pt, a.shape[0], ctypes.byref(loss),
                                           g.ctypes.data_as(_f_p)))
        return loss.value, g

    def adam_step(self, grads, lr):
        a, p = _fbuf(grads)
        _check(lib.wt_mlp_adam_step(self._h, p, lr))

    def train(self, x, t, epochs=200, batch=256, lr=1e-3, seed=1):
        a, px = _fbuf(x)
        b, pt = _fbuf(t)
        loss = ctypes.c_float()
        _check(lib.wt_mlp_train(self._h, px, pt, a.shape[0], epochs, batch, lr, seed, ctypes.byref(loss)))
        return loss.value

    def predict(self, x):
        import numpy as np
        a, px = _fbuf(x)
        y = np.empty(a.shape[0], np.float32)
        _check(lib.wt_mlp_predict(self._h, px, a.shape[0], y.ctypes.data_as(_f_p)))
        return y

    def save(self, path):
        _check(lib.wt_mlp_save(self._h, path.encode()))

    @classmethod
    def load(cls, path):
        h = ctypes.c_void_p()
        _check(lib.wt_mlp_load(path.encode(), ctypes.byref(h)))
        m = cls(_handle=h)
        return m


def model_train(measure_db, out_model, stream=None):
    """Trains the cost network on a measurement database (JSON lines) on the
    device and saves it to `out_model` (C-ABI wt_model_train)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib.wt_model_train(measure_db.encode(), out_model.encode(), ctypes.c_void_p(s)))


def model_rows(measure_db):
    """Usable lines of a measurement database, as model_train counts them."""
    n = ctypes.c_int()
    _check(lib.wt_model_rows(measure_db.encode(), ctypes.byref(n)))
    return n.value


def group_features(pipe, nodes, width, height, fp16=False, max_rows=4096):
    """(features [rows x 40], schedule texts) of every configuration of a group."""
    import numpy as np
    feats = np.zeros((max_rows, NUM_FEATURES), np.float32)
    n = ctypes.c_int()
    buf = ctypes.create_string_buffer(max_rows * 128)
    arr = (ctypes.c_int * len(nodes))(*nodes)
    _check(lib.wt_group_features(pipe._h, arr, len(nodes), width, height, int(fp16),
                                 feats.ctypes.data_as(_f_p), max_rows, ctypes.byref(n), buf, len(buf)))
    return feats[:n.value], buf.value.decode().split(";") if n.value else []


_sig("wt_measure_groups", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), ctypes.c_int, ctypes.c_char_p,
     ctypes.POINTER(ctypes.c_double))


def measure_groups(pipe, groups, width, height, fp16=False, reps=20, tag=""):
    """Device time in microseconds of each candidate group (schedule text per
    group), on scratch images; appends to $WT_MEASURE_DB when set."""
    n = len(groups)
    arr = (ctypes.c_char_p * max(n, 1))(*[g.encode() for g in groups])
    out = (ctypes.c_double * max(n, 1))()
    _check(lib.wt_measure_groups(pipe._h, width, height, int(fp16), n, arr, reps, tag.encode(), out))
    return [out[i] for i in range(n)]


_sig("wt_stage_profile", ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
     ctypes.POINTER(ctypes.c_double), _c_int_p, _c_int_p)


def stage_profile(pipe, node, width, height, measure=True):
    """(ns per evaluation, VGPRs, measured?) of a stage as the cost model sees it."""
    ns, vg, me = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
    _check(lib.wt_stage_profile(pipe._h, node, width, height, int(measure), ctypes.byref(ns),
                                ctypes.byref(vg), ctypes.byref(me)))
    return ns.value, vg.value, bool(me.value)
