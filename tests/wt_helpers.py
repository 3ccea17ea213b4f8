"""Shared test helpers: run a pipeline spec through the GPU path, and the
comparison rules (normwise tolerance, select tie band, bit-exactness)."""
import numpy as np

import oracle


# numpy storage type of each element type, and the same-size type torch
# moves it as (torch has few uint16 operations: those buffers travel as int16)
_NP = {"f32": np.float32, "u8": np.uint8, "u16": np.uint16, "i16": np.int16, "i32": np.int32}
_MOVE = {"f32": np.float32, "u8": np.uint8, "u16": np.int16, "i16": np.int16, "i32": np.int32}


def _dtypes(spec):
    dt = {i["name"]: i.get("dtype", "f32") for i in spec["inputs"]}
    for st in spec["stages"]:
        dt[st["name"]] = (dt[st["src"]] if st["kind"] in ("down2", "up2") else
                          "i32" if st["kind"] == "hist" else st.get("dtype", "f32"))
    return dt


def run_gpu(spec, inputs, width=None, height=None, **plan_kw):
    """Runs `spec` on the GPU through the C ABI; returns {output name: array}
    (float32 for float outputs, int64 for integer outputs)."""
    import torch
    import paper_1909_07190_amd as wt
    pipe = wt.from_spec(spec)
    first = inputs[spec["inputs"][0]["name"]]
    h, w = first.shape[-2:]
    plan = pipe.plan(width or w, height or h, **plan_kw)
    dev = torch.device("cuda:0")
    dts = _dtypes(spec)

    def to_dev(a, dt):
        t = torch.from_numpy(np.ascontiguousarray(a).astype(_NP[dt]).view(_MOVE[dt])).to(dev)
        return t.view(torch.uint16) if dt == "u16" else t

    ins = [to_dev(inputs[i["name"]], dts[i["name"]]) for i in spec["inputs"]]
    lv = _levels(spec)
    outs = []
    hists = {st["name"]: st["bins"] for st in spec["stages"] if st["kind"] == "hist"}
    for o in spec["outputs"]:
        ow, oh = (hists[o], 1) if o in hists else oracle.level_size(w, h, lv[o])
        ch = _channels(spec)[o]
        if dts[o] == "f32":
            outs.append(torch.full((ch, oh, ow), float("nan"), device=dev, dtype=torch.float32))
        else:  # a value the kernel must overwrite
            outs.append(to_dev(np.full((ch, oh, ow), 0x5A), dts[o]))
    plan.run(ins, outs)
    torch.cuda.synchronize()
    res = {}
    for o, t in zip(spec["outputs"], outs):
        if dts[o] == "f32":
            res[o] = t.cpu().numpy()
        else:
            if dts[o] == "u16":
                t = t.view(torch.int16)
            res[o] = t.cpu().numpy().view(_NP[dts[o]]).astype(np.int64)
    return res, plan


def _levels(spec):
    lv = {i["name"]: 0 for i in spec["inputs"]}
    for st in spec["stages"]:
        if st["kind"] == "down2":
            lv[st["name"]] = lv[st["src"]] + 1
        elif st["kind"] == "up2":
            lv[st["name"]] = lv[st["src"]] - 1
        elif st["kind"] in ("stencil", "hist", "equalize"):
            lv[st["name"]] = lv[st["src"]]
        else:
            lv[st["name"]] = lv[st["srcs"][0]]
    return lv


def _channels(spec):
    ch = {i["name"]: i["channels"] for i in spec["inputs"]}
    for st in spec["stages"]:
        if st["kind"] == "pointwise":
            ch[st["name"]] = st["channels"]
        else:
            ch[st["name"]] = ch[st["src"]]
    return ch


def assert_normwise(got, ref, rtol, what=""):
    """Per channel: max|got - ref| <= rtol * max|ref| (inf-norm relative)."""
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    for c in range(ref.shape[0]):
        m = float(np.max(np.abs(ref[c]))) if ref[c].size else 0.0
        d = float(np.max(np.abs(got[c].astype(np.float64) - ref[c]))) if ref[c].size else 0.0
        assert d <= rtol * max(m, 1e-30), f"{what} channel {c}: err {d:.3e} > {rtol:g} * {m:.3e}"


def assert_exact(got, ref, what=""):
    """Bit-exact equality; `ref` must itself be exactly representable in FP32."""
    r32 = ref.astype(np.float32)
    assert np.array_equal(r32.astype(np.float64), ref), f"{what}: reference not FP32-exact"
    bad = np.argwhere(got != r32)
    assert bad.size == 0, f"{what}: {len(bad)} mismatches, first at {bad[0].tolist()}: " \
                          f"got {got[tuple(bad[0])]!r} want {r32[tuple(bad[0])]!r}"


def unsharp_select_band(img, by, rtol):
    """Pixels whose |img - by| lies within rtol*(|img|+|by|) of the 0.01
    threshold may legitimately take either branch of the select."""
    d = np.abs(img.astype(np.float64) - by)
    return np.abs(d - 0.01) <= rtol * (np.abs(img) + np.abs(by)) + 1e-12


def check_unsharp(got, img, rtol, spec):
    vals = oracle.evaluate(spec, {"img": img}, keep_all=True)
    ref, by, sharp = vals["mask"], vals["by"], vals["sharp"]
    band = unsharp_select_band(img, by, rtol)
    # inside the band accept either branch's value
    alt = np.where(np.isclose(ref, img, rtol=0, atol=0), sharp, img.astype(np.float64))
    pick = np.where(band & (np.abs(got - alt) < np.abs(got - ref)), alt, ref)
    assert_normwise(got, pick, rtol, "unsharp")
    return int(band.sum())
