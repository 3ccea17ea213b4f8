"""Plain-data pipeline descriptions (no arithmetic is performed here).

A pipeline is a dict::

    {"inputs":  [{"name": str, "channels": int}, ...],
     "stages":  [stage, ...],          # in definition (topological) order
     "outputs": [name, ...]}

Stage kinds:

* ``stencil``  -- ``src``, ``kw``, ``kh``, anchor ``ax``, ``ay``, row-major
  ``weights`` (kh*kw numbers) and ``scale``; applied per channel.
* ``pointwise`` -- ``srcs`` (names), ``expr`` (infix; ``s0``, ``s1``... are the
  sources at the same channel, ``s0[k]`` is channel k of source 0),
  ``channels`` (output channel count).
* ``down2`` / ``up2`` -- ``src``; 2x decimation / 2x expansion.

Element types: an input or a stencil / pointwise stage may carry ``dtype``
(``"f32"`` by default, or ``"u8"``, ``"u16"``, ``"i16"``, ``"i32"``); an
integer stencil has integer ``weights`` and a positive integer ``divisor``
(its result is the sum divided by ``divisor``, halves rounded up, saturated
to the type).

Every stage's domain is its image size; producer reads outside the domain
take the value at the nearest edge point (clamp to edge, per stage).
"""
from __future__ import annotations

BINOMIAL5 = [1.0, 4.0, 6.0, 4.0, 1.0]


def _stencil(name, src, kw, kh, ax, ay, weights, scale):
    return {"name": name, "kind": "stencil", "src": src, "kw": kw, "kh": kh,
            "ax": ax, "ay": ay, "weights": list(map(float, weights)),
            "scale": float(scale)}


def _pw(name, srcs, expr, channels):
    return {"name": name, "kind": "pointwise", "srcs": list(srcs),
            "expr": expr, "channels": channels}


def blur_x(name, src):
    return _stencil(name, src, 5, 1, 2, 0, BINOMIAL5, 1.0 / 16.0)


def blur_y(name, src):
    return _stencil(name, src, 1, 5, 0, 2, BINOMIAL5, 1.0 / 16.0)


def gaussian_blur(channels: int = 1) -> dict:
    """Two-stage separable 5-tap binomial blur, x then y."""
    return {"inputs": [{"name": "img", "channels": channels}],
            "stages": [blur_x("bx", "img"), blur_y("by", "bx")],
            "outputs": ["by"]}


def unsharp_mask(channels: int = 3, weight: float = 1.5,
                 threshold: float = 0.01) -> dict:
    """Four-stage unsharp mask: blur x, blur y, sharpen, thresholded select."""
    return {"inputs": [{"name": "img", "channels": channels}],
            "stages": [
                blur_x("bx", "img"),
                blur_y("by", "bx"),
                _pw("sharp", ["img", "by"], f"s0 + {weight!r} * (s0 - s1)", channels),
                _pw("mask", ["img", "by", "sharp"],
                    f"select(abs(s0 - s1) < {threshold!r}, s0, s2)", channels),
            ],
            "outputs": ["mask"]}


SOBEL_X = [-1, 0, 1, -2, 0, 2, -1, 0, 1]
SOBEL_Y = [-1, -2, -1, 0, 0, 0, 1, 2, 1]
BOX3 = [1] * 9


def harris(gray_weights=(0.299, 0.587, 0.114), k: float = 0.04) -> dict:
    """Harris corner response on an RGB image (ten stages)."""
    r, g, b = gray_weights
    return {"inputs": [{"name": "img", "channels": 3}],
            "stages": [
                _pw("gray", ["img"], f"{r!r} * s0[0] + {g!r} * s0[1] + {b!r} * s0[2]", 1),
                _stencil("Ix", "gray", 3, 3, 1, 1, SOBEL_X, 1.0),
                _stencil("Iy", "gray", 3, 3, 1, 1, SOBEL_Y, 1.0),
                _pw("Ixx", ["Ix"], "s0 * s0", 1),
                _pw("Iyy", ["Iy"], "s0 * s0", 1),
                _pw("Ixy", ["Ix", "Iy"], "s0 * s1", 1),
                _stencil("Sxx", "Ixx", 3, 3, 1, 1, BOX3, 1.0),
                _stencil("Syy", "Iyy", 3, 3, 1, 1, BOX3, 1.0),
                _stencil("Sxy", "Ixy", 3, 3, 1, 1, BOX3, 1.0),
                _pw("R", ["Sxx", "Syy", "Sxy"],
                    f"s0 * s1 - s2 * s2 - {k!r} * (s0 + s1) * (s0 + s1)", 1),
            ],
            "outputs": ["R"]}


def pyramid_blend(levels: int = 4) -> dict:
    """Laplacian-pyramid blend of A and B under mask M, then collapse.

    Levels 0..levels-1 (levels-1 decimations).  Gaussian levels are
    G_{l+1} = down2(blur_y(blur_x(G_l))); Laplacian bands L_l = G_l - up2(G_{l+1})
    with the coarsest band equal to the coarsest Gaussian level; bands are
    blended as M_l*LA_l + (1-M_l)*LB_l and collapsed by R_l = Lb_l + up2(R_{l+1}).
    """
    st = []
    top = levels - 1
    for img in ("A", "B", "M"):
        prev = img
        for l in range(top):
            st.append(blur_x(f"{img}bx{l}", prev))
            st.append(blur_y(f"{img}by{l}", f"{img}bx{l}"))
            st.append({"name": f"{img}G{l + 1}", "kind": "down2", "src": f"{img}by{l}"})
            prev = f"{img}G{l + 1}"

    def G(img, l):
        return img if l == 0 else f"{img}G{l}"

    for img in ("A", "B"):
        for l in range(top):
            st.append({"name": f"{img}U{l}", "kind": "up2", "src": G(img, l + 1)})
            st.append(_pw(f"{img}L{l}", [G(img, l), f"{img}U{l}"], "s0 - s1", 1))
    for l in range(levels):
        la = f"AL{l}" if l < top else G("A", top)
        lb = f"BL{l}" if l < top else G("B", top)
        st.append(_pw(f"Lb{l}", [G("M", l), la, lb], "s0 * s1 + (1.0 - s0) * s2", 1))
    prev = f"Lb{top}"
    for l in range(top - 1, -1, -1):
        st.append({"name": f"RU{l}", "kind": "up2", "src": prev})
        st.append(_pw(f"R{l}", [f"Lb{l}", f"RU{l}"], "s0 + s1", 1))
        prev = f"R{l}"
    return {"inputs": [{"name": "A", "channels": 1}, {"name": "B", "channels": 1},
                       {"name": "M", "channels": 1}],
            "stages": st, "outputs": ["R0"]}


def laplacian_band(channels: int = 1) -> dict:
    """One level of a Laplacian pyramid: the Gaussian level below
    (G1 = down2(blur_y(blur_x(img)))) and the band img - up2(G1), plus a
    blur of G1 so the coarse level has a consumer of its own."""
    return {"inputs": [{"name": "img", "channels": channels}],
            "stages": [blur_x("bx", "img"), blur_y("by", "bx"),
                       {"name": "G1", "kind": "down2", "src": "by"},
                       {"name": "U", "kind": "up2", "src": "G1"},
                       _pw("L", ["img", "U"], "s0 - s1", channels),
                       blur_x("c1", "G1")],
            "outputs": ["L", "c1"]}


def _istencil(name, src, kw, kh, ax, ay, weights, divisor, dtype):
    return {"name": name, "kind": "stencil", "src": src, "kw": kw, "kh": kh,
            "ax": ax, "ay": ay, "weights": [int(w) for w in weights],
            "divisor": int(divisor), "dtype": dtype, "scale": 1.0 / divisor}


def binomial_u8(channels: int = 1) -> dict:
    """Separable 5-tap binomial blur on 8-bit images: (sum [1,4,6,4,1] x + 8) >> 4
    per pass, the integer counterpart of the Gaussian blur."""
    return {"inputs": [{"name": "img", "channels": channels, "dtype": "u8"}],
            "stages": [_istencil("bx", "img", 5, 1, 2, 0, [1, 4, 6, 4, 1], 16, "u8"),
                       _istencil("by", "bx", 1, 5, 0, 2, [1, 4, 6, 4, 1], 16, "u8")],
            "outputs": ["by"]}


def integer_unsharp(channels: int = 1) -> dict:
    """8-bit unsharp mask: binomial blur, signed 16-bit detail, sharpened
    result saturated back to 8 bits; the detail is an output too."""
    return {"inputs": [{"name": "img", "channels": channels, "dtype": "u8"}],
            "stages": [_istencil("bx", "img", 5, 1, 2, 0, [1, 4, 6, 4, 1], 16, "u8"),
                       _istencil("by", "bx", 1, 5, 0, 2, [1, 4, 6, 4, 1], 16, "u8"),
                       {"name": "detail", "kind": "pointwise", "srcs": ["img", "by"],
                        "expr": "s0 - s1", "channels": channels, "dtype": "i16"},
                       {"name": "sharp", "kind": "pointwise", "srcs": ["img", "detail"],
                        "expr": "s0 + 2 * s1", "channels": channels, "dtype": "u8"}],
            "outputs": ["sharp", "detail"]}


def integer_gradient() -> dict:
    """16-bit image: Sobel gradients in i32, L1 magnitude saturated to u16, a
    box-filtered i16 response with a non-power-of-two divisor, a decimated
    copy, and a float stage reading integers."""
    return {"inputs": [{"name": "img", "channels": 1, "dtype": "u16"}],
            "stages": [_istencil("gx", "img", 3, 3, 1, 1, [-1, 0, 1, -2, 0, 2, -1, 0, 1], 1, "i32"),
                       _istencil("gy", "img", 3, 3, 1, 1, [-1, -2, -1, 0, 0, 0, 1, 2, 1], 1, "i32"),
                       {"name": "mag", "kind": "pointwise", "srcs": ["gx", "gy"],
                        "expr": "abs(s0) + abs(s1)", "channels": 1, "dtype": "u16"},
                       _istencil("box", "gx", 3, 3, 1, 1, [1] * 9, 9, "i16"),
                       {"name": "small", "kind": "down2", "src": "mag"},
                       {"name": "f", "kind": "stencil", "src": "small", "kw": 3, "kh": 1, "ax": 1, "ay": 0,
                        "weights": [1.0, 2.0, 1.0], "scale": 0.25}],
            "outputs": ["mag", "box", "f"]}



def wide_chain(depth: int = 10, taps: int = 15) -> dict:
    """`depth` horizontal `taps`-wide box-like stencils in a chain, then the
    chain's end minus half the input.  Under right-hyperplane tiles each
    stencil shifts its stage by taps // 2 columns, so the last stage reads the
    input depth * (taps // 2) columns back (70 for the defaults: more than
    one 64-lane wavefront at one element per lane)."""
    w = [float(1 + j % 3) for j in range(taps)]
    stages, src = [], "img"
    for i in range(depth):
        stages.append(_stencil(f"s{i}", src, taps, 1, taps // 2, 0, w, 1.0 / sum(w)))
        src = f"s{i}"
    stages.append(_pw("out", [src, "img"], "s0 - 0.5 * s1", 1))
    return {"inputs": [{"name": "img", "channels": 1}], "stages": stages, "outputs": ["out"]}


def blur_histogram(channels: int = 1, bins: int = 64, lo: float = 0.0, hi: float = 1.0,
                   keep_blur: bool = False, of: str = "by") -> dict:
    """Separable 5-tap blur, then a histogram (`bins` equal bins over
    [lo, hi) per channel) of stage `of` (the blurred image "by", or the
    x-blur "bx" that "by" reads); the blurred image is an output too when
    `keep_blur`."""
    return {"inputs": [{"name": "img", "channels": channels}],
            "stages": [blur_x("bx", "img"), blur_y("by", "bx"),
                       {"name": "h", "kind": "hist", "src": of, "bins": bins, "lo": lo, "hi": hi}],
            "outputs": ["h", "by"] if keep_blur else ["h"]}


def u8_histogram() -> dict:
    """8-bit binomial blur and the 256-bin histogram of its result."""
    return {"inputs": [{"name": "img", "channels": 1, "dtype": "u8"}],
            "stages": [_istencil("bx", "img", 5, 1, 2, 0, [1, 4, 6, 4, 1], 16, "u8"),
                       _istencil("by", "bx", 1, 5, 0, 2, [1, 4, 6, 4, 1], 16, "u8"),
                       {"name": "h", "kind": "hist", "src": "by", "bins": 256, "lo": 0.0, "hi": 256.0}],
            "outputs": ["h"]}


def blur_equalize(channels: int = 1, bins: int = 256) -> dict:
    """Histogram equalisation of a blurred image, then a blend of the result
    with the input: the histogram of the blur (over [0, 1)) is a reduction
    its equalisation reads whole, so they run in separate kernels; the blend
    reads the equalised values at the same point."""
    return {"inputs": [{"name": "img", "channels": channels}],
            "stages": [blur_x("bx", "img"), blur_y("by", "bx"),
                       {"name": "h", "kind": "hist", "src": "by", "bins": bins, "lo": 0.0, "hi": 1.0},
                       {"name": "eq", "kind": "equalize", "src": "by", "hist": "h"},
                       _pw("out", ["eq", "img"], "0.75 * s0 + 0.25 * s1", channels)],
            "outputs": ["out"]}
