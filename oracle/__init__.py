"""FP64 reference evaluator for stencil pipelines -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The product (the HIP library and its Python binding) never
imports, links or calls it, and it shares no code with the product: it has its
own expression parser, its own stage loops and its own domain bookkeeping.

What it computes is the plain definition of a pipeline of per-pixel stages
(the paper, Section 2.2 and Fig. 2: each stage is a function over an integer
domain whose value at a point is an expression of producer values at constant
offsets).  Overlapped tiling, fusion and hybrid VGPR/LDS storage change only
*where* values are kept and how often they are recomputed, never the values
themselves (Section 2.2, overlapped tiles recompute their halo), so the
oracle evaluates every stage unfused, over its whole domain, in topological
order, in float64.

Readings where the paper is silent (it uses interior-only domains):
  * boundary: every producer read outside the producer's domain takes the
    value at the nearest point of that domain (clamp to edge, per stage);
  * down2 keeps even samples, its domain is ceil(W/2) x ceil(H/2);
  * up2 is the separable 2x expansion with the binomial [1,4,6,4,1]/16
    (Burt-Adelson EXPAND): even output 2i -> (P(i-1) + 6 P(i) + P(i+1)) / 8,
    odd output 2i+1 -> (P(i) + P(i+1)) / 2, coarse indices clamped, output
    domain the size of the finer level;
  * a pointwise stage reads each source at the same point; a one-channel
    source is broadcast over channels;
  * integer stages (types u8, u16, i16, i32): values are int64 in the oracle.
    An integer stencil takes the exact sum of integer weights times producer
    values, divides by its positive integer divisor d rounding halves up,
    floor((sum + floor(d/2)) / d), and saturates to its type's range; an
    integer pointwise expression (integer constants, no division) is
    evaluated exactly and saturated.  A float stage reading an integer stage
    sees its value converted exactly.  Integer stages do not take up2
    (a rounding rule for the expansion is not defined) and never read float
    stages.
  * a histogram stage (a reduction, the kind of stage the paper's Section 7
    names as outside its fusion, as in the bilateral grid's scatter) counts,
    per channel, its source's values in `bins` equal bins over [lo, hi):
    value v goes to bin floor((v - lo) * s), s = bins / (hi - lo), with v,
    lo and s rounded to FP32 and the subtraction and product done in FP32
    (the decision's precision is part of the stage's definition), clamped to
    0..bins-1 (NaN in bin 0).  Its result is [C, 1, bins] int64 counts; no
    stage reads it.

Every function below is pinned by tests under ``tests/`` (brute force on tiny
images, closed forms on ramps, steps, impulses and corners, and invariants).
"""
from __future__ import annotations

import ast

import numpy as np

__all__ = ["evaluate", "evaluate_stage", "parse_expr", "level_size",
           "stencil", "stencil_int", "down2", "up2", "pointwise", "INT_TYPES"]

# Value range of each integer type.
INT_TYPES = {"u8": (0, 255), "u16": (0, 65535), "i16": (-32768, 32767),
             "i32": (-(2 ** 31), 2 ** 31 - 1)}


# --------------------------------------------------------------------------
# Domains
# --------------------------------------------------------------------------

def level_size(width: int, height: int, level: int):
    """Domain of a level-``level`` stage of a pipeline whose inputs are W x H:
    each 2x decimation takes the ceiling of half of each side."""
    for _ in range(level):
        width = (width + 1) // 2
        height = (height + 1) // 2
    return width, height


# --------------------------------------------------------------------------
# Stage kinds (each takes and returns float64 arrays of shape [C, H, W])
# --------------------------------------------------------------------------

def stencil(p: np.ndarray, kw: int, kh: int, ax: int, ay: int,
            weights, scale: float) -> np.ndarray:
    """S_c(x, y) = scale * sum_{j<kh, i<kw} w[j][i] * P_c(clamp(x+i-ax), clamp(y+j-ay)).

    A constant-offset producer-consumer dependence (Section 2.3's dependence
    vectors), with the clamp-to-edge boundary reading.
    """
    c, h, w = p.shape
    wts = np.asarray(weights, dtype=np.float64).reshape(kh, kw)
    xs = np.arange(w)
    ys = np.arange(h)
    acc = np.zeros((c, h, w), dtype=np.float64)
    for j in range(kh):
        yi = np.clip(ys + j - ay, 0, h - 1)
        for i in range(kw):
            if wts[j, i] == 0.0:
                continue
            xi = np.clip(xs + i - ax, 0, w - 1)
            acc += wts[j, i] * p[:, yi][:, :, xi]
    return float(scale) * acc


def stencil_int(p: np.ndarray, kw: int, kh: int, ax: int, ay: int,
                weights, divisor: int, dtype: str) -> np.ndarray:
    """Integer stencil on an int64 producer: the exact sum
    acc = sum_{j,i} w[j][i] * P_c(clamp(x+i-ax), clamp(y+j-ay)), then
    floor((acc + floor(d/2)) / d) (ties round up) saturated to ``dtype``."""
    if p.dtype != np.int64:
        raise ValueError("integer stencils read integer stages")
    if int(divisor) < 1:
        raise ValueError("divisor must be a positive integer")
    wl = [int(v) for v in weights]
    if any(float(v) != float(int(v)) for v in weights):
        raise ValueError("integer stencil weights must be integers")
    c, h, w = p.shape
    wts = np.asarray(wl, dtype=np.int64).reshape(kh, kw)
    xs = np.arange(w)
    ys = np.arange(h)
    acc = np.zeros((c, h, w), dtype=np.int64)
    for j in range(kh):
        yi = np.clip(ys + j - ay, 0, h - 1)
        for i in range(kw):
            if wts[j, i] == 0:
                continue
            xi = np.clip(xs + i - ax, 0, w - 1)
            acc += wts[j, i] * p[:, yi][:, :, xi]
    d = int(divisor)
    q = (acc + d // 2) // d  # numpy's // on integers floors
    lo, hi = INT_TYPES[dtype]
    return np.clip(q, lo, hi)


def down2(p: np.ndarray) -> np.ndarray:
    """D(x, y) = P(2x, 2y) over ceil(W/2) x ceil(H/2)."""
    return p[:, 0::2, 0::2].copy()


def _expand_axis(p: np.ndarray, axis: int, n_out: int) -> np.ndarray:
    n_in = p.shape[axis]
    out_shape = list(p.shape)
    out_shape[axis] = n_out
    out = np.empty(out_shape, dtype=np.float64)
    for x in range(n_out):
        i = x // 2
        if x % 2 == 0:
            a = np.take(p, min(max(i - 1, 0), n_in - 1), axis=axis)
            b = np.take(p, min(i, n_in - 1), axis=axis)
            c = np.take(p, min(i + 1, n_in - 1), axis=axis)
            v = (a + 6.0 * b + c) / 8.0
        else:
            a = np.take(p, min(i, n_in - 1), axis=axis)
            b = np.take(p, min(i + 1, n_in - 1), axis=axis)
            v = (a + b) / 2.0
        idx = [slice(None)] * p.ndim
        idx[axis] = x
        out[tuple(idx)] = v
    return out


def up2(p: np.ndarray, out_w: int, out_h: int) -> np.ndarray:
    """Separable 2x binomial expansion, x first then y, to out_w x out_h."""
    return _expand_axis(_expand_axis(p, 2, out_w), 1, out_h)


# --------------------------------------------------------------------------
# Pointwise expressions: own parser on top of Python's ``ast`` grammar
# --------------------------------------------------------------------------

_FUNCS = {"abs": 1, "min": 2, "max": 2, "select": 3, "sqrt": 1, "floor": 1}
_CMP = {ast.Lt: np.less, ast.LtE: np.less_equal, ast.Gt: np.greater,
        ast.GtE: np.greater_equal}


def parse_expr(expr: str) -> ast.AST:
    """Parses the pointwise expression language and rejects anything outside it.

    Grammar: numbers, ``s<i>`` and ``s<i>[k]`` source references, unary minus,
    + - * /, one comparison (< <= > >=), and calls abs, min, max, select,
    sqrt, floor.
    """
    tree = ast.parse(expr, mode="eval")
    for node in ast.walk(tree):
        ok = isinstance(node, (ast.Expression, ast.BinOp, ast.UnaryOp, ast.Call,
                               ast.Compare, ast.Name, ast.Constant, ast.Subscript,
                               ast.Load, ast.Add, ast.Sub, ast.Mult, ast.Div,
                               ast.USub, ast.UAdd, ast.Lt, ast.LtE, ast.Gt, ast.GtE))
        if not ok:
            raise ValueError(f"unsupported syntax {type(node).__name__} in {expr!r}")
        if isinstance(node, ast.Call):
            if not isinstance(node.func, ast.Name) or node.func.id not in _FUNCS:
                raise ValueError(f"unknown function in {expr!r}")
            if len(node.args) != _FUNCS[node.func.id] or node.keywords:
                raise ValueError(f"wrong arity for {node.func.id} in {expr!r}")
        if isinstance(node, ast.Compare) and len(node.ops) != 1:
            raise ValueError(f"chained comparison in {expr!r}")
        if isinstance(node, ast.Name) and node.id not in _FUNCS:
            if not (node.id.startswith("s") and node.id[1:].isdigit()):
                raise ValueError(f"unknown name {node.id!r} in {expr!r}")
    return tree


def _eval(node, srcs, ch, integer=False):
    if isinstance(node, ast.Expression):
        return _eval(node.body, srcs, ch, integer)
    if isinstance(node, ast.Constant):
        if integer:
            if float(node.value) != int(node.value):
                raise ValueError("integer expressions take integer constants")
            return np.int64(int(node.value))
        return float(node.value)
    if isinstance(node, ast.Name):
        s = srcs[int(node.id[1:])]
        return s[ch] if s.shape[0] > 1 else s[0]
    if isinstance(node, ast.Subscript):
        s = srcs[int(node.value.id[1:])]
        k = node.slice.value if isinstance(node.slice, ast.Constant) else None
        if not isinstance(k, int) or not 0 <= k < s.shape[0]:
            raise ValueError("bad channel subscript")
        return s[k]
    if isinstance(node, ast.UnaryOp):
        v = _eval(node.operand, srcs, ch, integer)
        return -v if isinstance(node.op, ast.USub) else v
    if isinstance(node, ast.BinOp):
        a = _eval(node.left, srcs, ch, integer)
        b = _eval(node.right, srcs, ch, integer)
        if isinstance(node.op, ast.Add):
            return a + b
        if isinstance(node.op, ast.Sub):
            return a - b
        if isinstance(node.op, ast.Mult):
            return a * b
        if integer:
            raise ValueError("integer expressions have no division")
        return a / b
    if isinstance(node, ast.Compare):
        return _CMP[type(node.ops[0])](_eval(node.left, srcs, ch, integer),
                                       _eval(node.comparators[0], srcs, ch, integer))
    if isinstance(node, ast.Call):
        args = [_eval(a, srcs, ch, integer) for a in node.args]
        f = node.func.id
        if integer and f in ("sqrt", "floor"):
            raise ValueError(f"{f} is not an integer operation")
        if f == "abs":
            return np.abs(args[0])
        if f == "min":
            return np.minimum(args[0], args[1])
        if f == "max":
            return np.maximum(args[0], args[1])
        if f == "sqrt":
            return np.sqrt(args[0])
        if f == "floor":
            return np.floor(args[0])
        return np.where(args[0], args[1], args[2])
    raise ValueError("unsupported node")


def pointwise(expr: str, srcs, channels: int, dtype: str = "f32") -> np.ndarray:
    """Evaluates ``expr`` at every point of every output channel, in float64,
    or for an integer ``dtype`` exactly in int64 and saturated to its range."""
    tree = parse_expr(expr)
    integer = dtype in INT_TYPES
    if integer and any(s.dtype != np.int64 for s in srcs):
        raise ValueError("integer pointwise stages read integer stages only")
    shape = None
    for s in srcs:
        if shape is None:
            shape = s.shape[1:]
        elif s.shape[1:] != shape:
            raise ValueError("pointwise sources must share one domain")
    out = np.empty((channels,) + tuple(shape), dtype=np.int64 if integer else np.float64)
    for c in range(channels):
        v = _eval(tree, srcs, c, integer)
        if integer:
            lo, hi = INT_TYPES[dtype]
            v = np.clip(v, lo, hi)
        out[c] = np.broadcast_to(v, shape)
    return out


def histogram(p: np.ndarray, bins: int, lo: float, hi: float) -> np.ndarray:
    """Per channel, the counts of p's values in `bins` equal bins over
    [lo, hi): bin floor((v - lo) * s) with s = bins / (hi - lo), computed in
    FP32 (v, lo and s rounded to FP32 first), clamped to 0..bins-1; NaN
    counts in bin 0.  Returns [C, 1, bins] int64."""
    v = np.asarray(p).astype(np.float32)
    lo32 = np.float32(lo)
    s32 = np.float32(bins / (hi - lo))
    t = (v - lo32) * s32  # float32 operands: each operation rounded to FP32
    with np.errstate(invalid="ignore"):
        idx = np.where(t >= 0, np.where(t >= bins, bins - 1, np.floor(np.where(t >= 0, t, 0))), 0).astype(np.int64)
    out = np.zeros((v.shape[0], 1, bins), dtype=np.int64)
    for c in range(v.shape[0]):
        out[c, 0] = np.bincount(idx[c].ravel(), minlength=bins)
    return out


def equalize(p: np.ndarray, counts: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Histogram equalisation: per channel, value v maps to C(b) / N, b its
    bin under the histogram's rule (bins = counts.shape[-1], [lo, hi)), C the
    inclusive cumulative counts, N their total; C(b) in FP32 times 1/N
    rounded to FP32 (0 when N = 0).  Returns float64 values of those FP32
    results."""
    bins = counts.shape[-1]
    v = np.asarray(p).astype(np.float32)
    lo32, s32 = np.float32(lo), np.float32(bins / (hi - lo))
    t = (v - lo32) * s32
    with np.errstate(invalid="ignore"):
        idx = np.where(t >= 0, np.where(t >= bins, bins - 1, np.floor(np.where(t >= 0, t, 0))), 0).astype(np.int64)
    out = np.zeros(v.shape, dtype=np.float64)
    for c in range(v.shape[0]):
        cum = np.cumsum(counts[c].reshape(-1))
        total = cum[-1]
        rn = np.float32(1.0) / np.float32(total) if total else np.float32(0.0)
        out[c] = (cum[idx[c]].astype(np.float32) * rn).astype(np.float64)
    return out


# --------------------------------------------------------------------------
# Whole pipelines
# --------------------------------------------------------------------------

def _levels(spec):
    lv = {i["name"]: 0 for i in spec["inputs"]}
    for st in spec["stages"]:
        k = st["kind"]
        if k == "stencil":
            lv[st["name"]] = lv[st["src"]]
        elif k == "down2":
            lv[st["name"]] = lv[st["src"]] + 1
        elif k == "up2":
            if lv[st["src"]] < 1:
                raise ValueError("up2 of a level-0 stage")
            lv[st["name"]] = lv[st["src"]] - 1
        elif k in ("hist", "equalize"):
            lv[st["name"]] = lv[st["src"]]
        elif k == "pointwise":
            ls = {lv[s] for s in st["srcs"]}
            if len(ls) != 1:
                raise ValueError("pointwise sources on different levels")
            lv[st["name"]] = ls.pop()
        else:
            raise ValueError(f"unknown stage kind {k!r}")
    return lv


def evaluate_stage(st, vals, lv, width, height, stages=None):
    k = st["kind"]
    dtype = st.get("dtype", "f32")
    if k == "stencil":
        if dtype in INT_TYPES:
            return stencil_int(vals[st["src"]], st["kw"], st["kh"], st["ax"], st["ay"],
                               st["weights"], st.get("divisor", 1), dtype)
        return stencil(vals[st["src"]], st["kw"], st["kh"], st["ax"], st["ay"],
                       st["weights"], st["scale"])
    if k == "down2":
        return down2(vals[st["src"]])
    if k == "hist":
        return histogram(vals[st["src"]], st["bins"], st["lo"], st["hi"])
    if k == "equalize":
        h = stages[st["hist"]]  # the histogram's bin rule
        return equalize(vals[st["src"]], vals[st["hist"]], h["lo"], h["hi"])
    if k == "up2":
        if vals[st["src"]].dtype == np.int64:
            raise ValueError("up2 of an integer stage")
        ow, oh = level_size(width, height, lv[st["name"]])
        return up2(vals[st["src"]], ow, oh)
    return pointwise(st["expr"], [vals[s] for s in st["srcs"]], st["channels"], dtype)


def evaluate(spec: dict, inputs: dict, keep_all: bool = False) -> dict:
    """Evaluates the pipeline on ``inputs`` (name -> [C, H, W] array).

    Returns the outputs (or every stage when ``keep_all``) as float64 arrays,
    int64 for integer stages.
    """
    lv = _levels(spec)
    vals = {}
    shape = None
    for inp in spec["inputs"]:
        dtype = inp.get("dtype", "f32")
        if dtype in INT_TYPES:
            a = np.asarray(inputs[inp["name"]])
            lo, hi = INT_TYPES[dtype]
            if a.size and (a.min() < lo or a.max() > hi or np.any(a != np.floor(a))):
                raise ValueError(f"input {inp['name']} holds values outside {dtype}")
            a = a.astype(np.int64)
        else:
            a = np.asarray(inputs[inp["name"]], dtype=np.float64)
        if a.ndim == 2:
            a = a[None]
        if a.shape[0] != inp["channels"]:
            raise ValueError(f"input {inp['name']} has {a.shape[0]} channels")
        if shape is None:
            shape = a.shape[1:]
        elif a.shape[1:] != shape:
            raise ValueError("pipeline inputs must share one size")
        vals[inp["name"]] = a
    height, width = shape
    for st in spec["stages"]:
        vals[st["name"]] = evaluate_stage(st, vals, lv, width, height, {s["name"]: s for s in spec["stages"]})
    if keep_all:
        return vals
    return {name: vals[name] for name in spec["outputs"]}

