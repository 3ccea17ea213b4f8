"""Pins for the FP64 oracle: brute force, closed forms and invariants.

Nothing here calls the GPU path.  Each brute-force reference below is an
independent direct formula (pure Python loops over tiny images) rather than a
retyping of the oracle's stage loops: the separable blur is checked against
the 5x5 outer-product sum, Harris against nested per-stage clamps written as
functions of a point, and the 2x expansion against its 2-D sum form.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from synth import pipelines as P

W5 = [1, 4, 6, 4, 1]
SIZES = [(1, 1), (1, 7), (2, 3), (4, 4), (7, 5), (17, 13), (64, 3)]


def cl(v, n):
    return min(max(v, 0), n - 1)


# ---------------------------------------------------------------- blur ----

def brute_blur(img):
    """by(x,y) = sum_{i,j} w_i w_j I(clamp(x+i-2), clamp(y+j-2)) / 256."""
    h, w = img.shape
    out = np.zeros((h, w))
    for y in range(h):
        for x in range(w):
            s = 0.0
            for j in range(5):
                for i in range(5):
                    s += W5[i] * W5[j] * float(img[cl(y + j - 2, h), cl(x + i - 2, w)])
            out[y, x] = s / 256.0
    return out


@pytest.mark.parametrize("h,w", SIZES)
def test_blur_brute_force(h, w):
    img = synth.uniform_image(11, 1, h, w)
    got = oracle.evaluate(P.gaussian_blur(), {"img": img})["by"][0]
    np.testing.assert_allclose(got, brute_blur(img[0]), rtol=0, atol=1e-12)


def test_blur_constant_image_is_constant():
    img = np.full((1, 9, 11), 0.3725, np.float32)
    got = oracle.evaluate(P.gaussian_blur(), {"img": img})["by"]
    np.testing.assert_allclose(got, float(img[0, 0, 0]), rtol=0, atol=1e-15)


def test_blur_impulse_response():
    img = np.zeros((1, 11, 11), np.float32)
    img[0, 5, 5] = 1.0
    got = oracle.evaluate(P.gaussian_blur(), {"img": img})["by"][0]
    exp = np.zeros((11, 11))
    exp[3:8, 3:8] = np.outer(W5, W5) / 256.0
    np.testing.assert_array_equal(got, exp)


def test_blur_ramp_borders():
    # I(x, y) = x on an 8-wide image.  Interior points reproduce x exactly;
    # at x = 0 the clamped taps read (0,0,0,1,2) -> 6/16, at x = 1 (0,0,1,2,3)
    # -> 17/16, and symmetrically 5.9375 and 6.625 at x = 6, 7.
    img = np.tile(np.arange(8, dtype=np.float32), (1, 6, 1))
    got = oracle.evaluate(P.gaussian_blur(), {"img": img})["by"][0]
    for y in range(6):
        np.testing.assert_array_equal(got[y], [0.375, 1.0625, 2, 3, 4, 5, 5.9375, 6.625])


def test_blur_linear_and_order_free():
    a = synth.uniform_image(1, 1, 13, 21).astype(np.float64)
    b = synth.uniform_image(2, 1, 13, 21).astype(np.float64)
    f = lambda x: oracle.evaluate(P.gaussian_blur(), {"img": x})["by"]
    np.testing.assert_allclose(f(2.5 * a - 0.75 * b), 2.5 * f(a) - 0.75 * f(b), atol=1e-13)
    # y-then-x equals x-then-y, and transposing the image transposes the blur.
    yx = {"inputs": [{"name": "img", "channels": 1}],
          "stages": [P.blur_y("t", "img"), P.blur_x("u", "t")], "outputs": ["u"]}
    np.testing.assert_allclose(oracle.evaluate(yx, {"img": a})["u"], f(a), atol=1e-14)
    np.testing.assert_allclose(f(a[:, ::-1, :].transpose(0, 2, 1)),
                               f(a)[:, ::-1, :].transpose(0, 2, 1), atol=1e-14)


# ------------------------------------------------------------ unsharp ----

def brute_unsharp(img, wgt=1.5, thr=0.01):
    c, h, w = img.shape
    out = np.zeros((c, h, w))
    for ch in range(c):
        by = brute_blur(img[ch])
        for y, x in itertools.product(range(h), range(w)):
            i = float(img[ch, y, x])
            sharp = i + wgt * (i - by[y, x])
            out[ch, y, x] = i if abs(i - by[y, x]) < thr else sharp
    return out


@pytest.mark.parametrize("h,w", [(1, 1), (3, 5), (9, 17), (16, 4)])
def test_unsharp_brute_force(h, w):
    img = synth.uniform_image(5, 3, h, w)
    got = oracle.evaluate(P.unsharp_mask(), {"img": img})["mask"]
    np.testing.assert_allclose(got, brute_unsharp(img), rtol=0, atol=1e-12)


def test_unsharp_constant_and_step_edge():
    img = np.full((3, 6, 9), 0.5, np.float32)
    got = oracle.evaluate(P.unsharp_mask(), {"img": img})["mask"]
    np.testing.assert_array_equal(got, img)
    # Vertical step 0 -> 1 at x0 = 6: blur = 1/16, 5/16, 11/16, 15/16 at
    # x0-2 .. x0+1, output = I + 1.5 (I - blur) there, I elsewhere.
    img = np.zeros((1, 7, 12), np.float32)
    img[:, :, 6:] = 1.0
    vals = oracle.evaluate(P.unsharp_mask(1), {"img": img}, keep_all=True)
    np.testing.assert_array_equal(vals["by"][0, 3, 4:8], [1 / 16, 5 / 16, 11 / 16, 15 / 16])
    exp = img[0, 3].astype(np.float64).copy()
    exp[4:8] = [-0.09375, -0.46875, 1.46875, 1.09375]
    for y in range(7):
        np.testing.assert_allclose(vals["mask"][0, y], exp, rtol=0, atol=1e-15)


# ------------------------------------------------------------- harris ----

def brute_harris(img, gw=(0.299, 0.587, 0.114), k=0.04):
    _, h, w = img.shape

    def gray(x, y):
        x, y = cl(x, w), cl(y, h)
        return gw[0] * float(img[0, y, x]) + gw[1] * float(img[1, y, x]) + gw[2] * float(img[2, y, x])

    def ix(x, y):
        x, y = cl(x, w), cl(y, h)
        return sum(b * (gray(x + 1, y + j) - gray(x - 1, y + j)) for j, b in zip((-1, 0, 1), (1, 2, 1)))

    def iy(x, y):
        x, y = cl(x, w), cl(y, h)
        return sum(b * (gray(x + i, y + 1) - gray(x + i, y - 1)) for i, b in zip((-1, 0, 1), (1, 2, 1)))

    def box(f, x, y):
        return sum(f(cl(x + i, w), cl(y + j, h)) for i in (-1, 0, 1) for j in (-1, 0, 1))

    out = np.zeros((1, h, w))
    for y, x in itertools.product(range(h), range(w)):
        sxx = box(lambda a, b: ix(a, b) ** 2, x, y)
        syy = box(lambda a, b: iy(a, b) ** 2, x, y)
        sxy = box(lambda a, b: ix(a, b) * iy(a, b), x, y)
        out[0, y, x] = sxx * syy - sxy * sxy - k * (sxx + syy) ** 2
    return out


@pytest.mark.parametrize("h,w", [(1, 1), (2, 3), (5, 4), (9, 7)])
def test_harris_brute_force(h, w):
    img = synth.uniform_image(7, 3, h, w)
    got = oracle.evaluate(P.harris(), {"img": img})["R"]
    np.testing.assert_allclose(got, brute_harris(img), rtol=0, atol=1e-11)


def _gray_rgb(g):
    return np.repeat(g[None].astype(np.float32), 3, axis=0)


def test_harris_closed_forms():
    # Constant image: every derivative is 0, so R = 0 exactly.
    r = oracle.evaluate(P.harris(), {"img": np.full((3, 8, 8), 0.7, np.float32)})["R"]
    assert np.all(r == 0.0)
    # Vertical step at x0: Ix = 4 at x0-1, x0; Sxx = 48, 96, 96, 48 at
    # x0-2 .. x0+1; Syy = Sxy = 0, so R = -0.04 Sxx^2.
    g = np.zeros((12, 16))
    g[:, 8:] = 1.0
    r = oracle.evaluate(P.harris(), {"img": _gray_rgb(g)})["R"][0]
    np.testing.assert_allclose(r[5, 5:11], [0, -92.16, -368.64, -368.64, -92.16, 0], atol=1e-9)
    # Quadrant {x >= x0, y >= y0}: with c(-1)=1, c(0)=3, c(>=1)=4 the box sums
    # at the corner are Sxx = Syy = 52, Sxy = 16 -> R = 2015.36; at (x0-1, y0-1)
    # 20, 20, 16 -> 80; at (x0, y0-1): 20, 52, 16 -> 576.64.
    g = np.zeros((16, 16))
    g[8:, 8:] = 1.0
    r = oracle.evaluate(P.harris(), {"img": _gray_rgb(g)})["R"][0]
    np.testing.assert_allclose(r[8, 8], 2015.36, rtol=1e-9)
    np.testing.assert_allclose(r[7, 7], 80.0, rtol=1e-9)
    np.testing.assert_allclose(r[7, 8], 576.64, rtol=1e-9)
    np.testing.assert_allclose(r[8, 7], 576.64, rtol=1e-9)


def test_harris_invariants():
    img = synth.uniform_image(3, 3, 10, 14).astype(np.float64)
    f = lambda x: oracle.evaluate(P.harris(), {"img": x})["R"]
    np.testing.assert_allclose(f(img.transpose(0, 2, 1)), f(img).transpose(0, 2, 1), atol=1e-11)
    np.testing.assert_allclose(f(img[:, :, ::-1]), f(img)[:, :, ::-1], atol=1e-11)
    np.testing.assert_allclose(f(0.5 * img), f(img) / 16.0, atol=1e-11)


# ------------------------------------------------------------ resample ---

def brute_expand(p, ow, oh):
    """EXPAND in its 2-D sum form: U(x,y) = 4 sum_{m,n} w_m w_n P((x-m)/2, (y-n)/2)
    over the m, n in [-2, 2] that make both quotients integers (w = W5/16)."""
    h, w = p.shape
    out = np.zeros((oh, ow))
    for y, x in itertools.product(range(oh), range(ow)):
        s = 0.0
        for m in range(-2, 3):
            for n in range(-2, 3):
                if (x - m) % 2 or (y - n) % 2:
                    continue
                s += W5[m + 2] * W5[n + 2] / 256.0 * float(p[cl((y - n) // 2, h), cl((x - m) // 2, w)])
        out[y, x] = 4.0 * s
    return out


@pytest.mark.parametrize("h,w,oh,ow", [(1, 1, 1, 2), (2, 3, 3, 5), (4, 4, 8, 8), (5, 7, 9, 13)])
def test_up2_brute_force(h, w, oh, ow):
    p = synth.uniform_image(4, 1, h, w).astype(np.float64)
    np.testing.assert_allclose(oracle.up2(p, ow, oh)[0], brute_expand(p[0], ow, oh), atol=1e-14)


def test_up2_reproduces_linear_and_constant():
    p = np.tile(np.arange(9.0), (1, 4, 1))
    u = oracle.up2(p, 18, 8)[0]
    np.testing.assert_array_equal(u[3, 2:16], np.arange(2, 16) / 2.0)
    c = np.full((1, 3, 5), 0.25)
    assert np.all(oracle.up2(c, 10, 6) == 0.25)


def test_down2_and_levels():
    p = np.arange(35.0).reshape(1, 5, 7)
    d = oracle.down2(p)
    assert d.shape == (1, 3, 4)
    for y, x in itertools.product(range(3), range(4)):
        assert d[0, y, x] == p[0, 2 * y, 2 * x]
    assert oracle.level_size(2731, 513, 3) == (342, 65)


def test_pyramid_reconstruction_identities():
    spec = P.pyramid_blend(4)
    a = synth.uniform_image(21, 1, 37, 45)
    b = synth.uniform_image(22, 1, 37, 45)
    one = np.ones_like(a)
    ev = lambda m, x, y: oracle.evaluate(spec, {"A": x, "B": y, "M": m})["R0"]
    np.testing.assert_allclose(ev(one, a, b), a, atol=1e-13)
    np.testing.assert_allclose(ev(0 * one, a, b), b, atol=1e-13)
    m = synth.ramp_mask(37, 45)
    np.testing.assert_allclose(ev(m, a, a), a, atol=1e-13)
    # linear in (A, B) for a fixed mask
    np.testing.assert_allclose(ev(m, 2 * a, 2 * b), 2 * ev(m, a, b), atol=1e-13)


# --------------------------------------------------------------- misc ----

def test_expression_language():
    with pytest.raises(ValueError):
        oracle.parse_expr("__import__('os')")
    with pytest.raises(ValueError):
        oracle.parse_expr("s0 < s1 < s2")
    with pytest.raises(ValueError):
        oracle.parse_expr("min(s0)")
    x = np.array([[[1.0, -2.0]]])
    y = np.array([[[3.0, 4.0]]])
    got = oracle.pointwise("select(s0 < 0, -s0, min(s0, s1) * 2 - s1 / 4)", [x, y], 1)
    np.testing.assert_array_equal(got, [[[1 * 2 - 0.75, 2.0]]])


def test_generators_are_exact_and_seeded():
    a = synth.uniform_image(3, 2, 5, 7)
    assert a.dtype == np.float32 and a.shape == (2, 5, 7)
    assert np.array_equal(a, synth.uniform_image(3, 2, 5, 7))
    assert not np.array_equal(a, synth.uniform_image(4, 2, 5, 7))
    assert np.all((a >= 0) & (a < 1))
    assert np.all(a.astype(np.float64) * (1 << 24) == np.floor(a.astype(np.float64) * (1 << 24)))
    # splitmix64 reference draws for seed 0 (published test vector of the
    # generator: first outputs for state 0).
    z = synth.splitmix64_block(0, 0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    sq = synth.white_squares(np.zeros((3, 64, 64), np.float32), 1, count=5)
    assert sq.max() == 1.0 and np.all(sq[0] == sq[2])


# ---------------------------------------------------------------- histogram --

def test_histogram_of_exact_bin_values():
    """Values k/16 (k = 0..15, each k+1 times) in 16 bins over [0, 1): bin k
    holds exactly k+1 counts."""
    vals = np.concatenate([np.full(k + 1, k / 16.0) for k in range(16)])
    h = oracle.histogram(vals.reshape(1, 1, -1), 16, 0.0, 1.0)
    assert h.shape == (1, 1, 16) and h.dtype == np.int64
    assert h[0, 0].tolist() == list(range(1, 17))


def test_histogram_out_of_range_values():
    """Below lo and NaN go to bin 0; hi and above to the last bin; the value
    one FP32 step below an edge stays in the lower bin, while 0.5 - 1e-9
    (0.5 once rounded to FP32, the decision's precision) goes up."""
    below = float(np.nextafter(np.float32(0.5), np.float32(0.0)))
    v = np.array([[[-5.0, np.nan, 1.0, 7.0, below, 0.5, 0.5 - 1e-9]]])
    h = oracle.histogram(v, 4, 0.0, 1.0)[0, 0]
    assert h.tolist() == [2, 1, 2, 2]


def test_histogram_matches_numpy_away_from_edges():
    """Random values more than 1e-5 from every bin edge: the same counts as
    numpy.histogram over the same edges, channel by channel (the channels
    hold different distributions), and every value counted once."""
    rng = np.random.default_rng(5)
    v = np.stack([rng.uniform(-0.2, 1.2, 20000), rng.beta(2, 5, 20000) * 1.5]).reshape(2, 100, 200)
    lo, hi, nb = -0.1, 1.3, 35
    edges = np.linspace(lo, hi, nb + 1)
    far = np.min(np.abs(v[..., None] - edges), axis=-1) > 1e-5
    h = oracle.histogram(np.where(far, v, lo + 0.5 * (hi - lo) / nb), nb, lo, hi)
    for c in range(2):
        x = np.where(far[c], v[c], lo + 0.5 * (hi - lo) / nb).ravel()
        ref, _ = np.histogram(np.clip(x, lo, np.nextafter(hi, lo)), bins=edges)
        assert h[c, 0].tolist() == ref.tolist()
        assert h[c, 0].sum() == v[c].size


def test_histogram_stage_in_a_pipeline():
    """A histogram stage counts its source stage over the whole image, one
    histogram per channel, of shape [C, 1, bins]."""
    spec = P.blur_histogram(channels=2, bins=8)
    img = np.zeros((2, 5, 7))
    img[1] = 0.999
    out = oracle.evaluate(spec, {"img": img})["h"]
    assert out.shape == (2, 1, 8)
    assert out[0, 0].tolist() == [35, 0, 0, 0, 0, 0, 0, 0]
    assert out[1, 0].tolist() == [0, 0, 0, 0, 0, 0, 0, 35]


def test_equalize_maps_bins_to_cumulative_fractions():
    """Values k/16 (k = 0..15, each k+1 times) in 16 bins: value k/16 maps to
    the fraction of values at or below it, (k+1)(k+2)/2 of 136, to FP32
    rounding; the largest value maps to 1 within one FP32 step; the map is
    non-decreasing in the value."""
    vals = np.concatenate([np.full(k + 1, k / 16.0) for k in range(16)]).reshape(1, 1, -1)
    h = oracle.histogram(vals, 16, 0.0, 1.0)
    e = oracle.equalize(np.arange(16).reshape(1, 1, 16) / 16.0, h, 0.0, 1.0)[0, 0]
    want = np.array([(k + 1) * (k + 2) / 2 / 136 for k in range(16)])
    assert np.max(np.abs(e - want)) <= 2 ** -23
    assert abs(e[-1] - 1.0) <= 2 ** -23 and np.all(np.diff(e) > 0)


def test_equalize_flattens_the_distribution_and_handles_empty_counts():
    """Equalising an image by its own histogram spreads its values evenly:
    the share of pixels mapped at or below q is q, up to the mass of one
    bin; an all-zero histogram maps everything to 0."""
    rng = np.random.default_rng(3)
    img = (rng.beta(5, 2, (1, 300, 400)) * 0.999)
    h = oracle.histogram(img, 256, 0.0, 1.0)
    e = oracle.equalize(img, h, 0.0, 1.0)
    top = h.max() / img.size
    for q in (0.1, 0.25, 0.5, 0.75, 0.9):
        assert abs(np.mean(e <= q) - q) <= top + 1e-9
    assert np.all(oracle.equalize(img, np.zeros_like(h), 0.0, 1.0) == 0.0)
